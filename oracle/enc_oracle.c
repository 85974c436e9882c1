/* Adaptive video encoder oracle (Section 3.1.2); see enc_oracle.h.
 * TEST INFRASTRUCTURE ONLY. */
#include "enc_oracle.h"

#include <stdlib.h>
#include <string.h>

void enc_reduce(const uint8_t* rgb, uint32_t width, uint32_t height, uint32_t factor,
                uint8_t* out) {
  const uint32_t w = width / factor, h = height / factor, area = factor * factor;
  for (uint32_t y = 0; y < h; ++y)
    for (uint32_t x = 0; x < w; ++x)
      for (uint32_t ch = 0; ch < 3; ++ch) {
        uint32_t sum = 0;
        for (uint32_t dy = 0; dy < factor; ++dy)
          for (uint32_t dx = 0; dx < factor; ++dx)
            sum += rgb[3 * ((size_t)(y * factor + dy) * width + (x * factor + dx)) + ch];
        out[3 * ((size_t)y * w + x) + ch] = (uint8_t)((sum + area / 2) / area);
      }
}

void enc_gray(const uint8_t* rgb, uint32_t n, uint8_t* gray) {
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t r = rgb[3 * (size_t)i], g = rgb[3 * (size_t)i + 1], b = rgb[3 * (size_t)i + 2];
    gray[i] = (uint8_t)((4899u * r + 9617u * g + 1868u * b + 8192u) >> 14);
  }
}

static uint32_t clampi(int64_t v, uint32_t n) {
  if (v < 0) return 0;
  if (v >= (int64_t)n) return n - 1;
  return (uint32_t)v;
}

void enc_threshold(const uint8_t* gray, uint32_t w, uint32_t h, uint32_t block, int32_t offset,
                   uint8_t* on) {
  /* binomial weights: row b - 1 of Pascal's triangle */
  uint64_t wt[16];
  wt[0] = 1;
  for (uint32_t i = 1; i < block; ++i) wt[i] = wt[i - 1] * (block - i) / i;
  const int64_t r = (int64_t)block / 2;
  const uint32_t shift = 2 * (block - 1); /* log2 of the total weight */
  for (uint32_t y = 0; y < h; ++y)
    for (uint32_t x = 0; x < w; ++x) {
      uint64_t sum = 0;
      for (uint32_t i = 0; i < block; ++i)
        for (uint32_t j = 0; j < block; ++j) {
          const uint32_t yy = clampi((int64_t)y + (int64_t)i - r, h);
          const uint32_t xx = clampi((int64_t)x + (int64_t)j - r, w);
          sum += wt[i] * wt[j] * gray[(size_t)yy * w + xx];
        }
      const int64_t mean = (int64_t)((sum + (1ull << (shift - 1))) >> shift);
      on[(size_t)y * w + x] = (int64_t)gray[(size_t)y * w + x] > mean - offset ? 1 : 0;
    }
}

void enc_pack(const uint8_t* on, uint32_t n, uint32_t* words) {
  memset(words, 0, sizeof(uint32_t) * (((size_t)n + 31) / 32));
  for (uint32_t p = 0; p < n; ++p)
    if (on[p]) words[p >> 5] |= 1u << (p & 31);
}

int enc_frames(const enc_config* cfg, const uint8_t* rgb, uint32_t frames, uint32_t* words) {
  if (!cfg || cfg->factor < 1 || cfg->block < 3 || cfg->block > 11 || cfg->block % 2 == 0)
    return -1;
  const uint32_t w = cfg->width / cfg->factor, h = cfg->height / cfg->factor;
  if (w == 0 || h == 0) return -1;
  const size_t n = (size_t)w * h, nw = (n + 31) / 32;
  uint8_t* small = (uint8_t*)malloc(3 * n);
  uint8_t* gray = (uint8_t*)malloc(n);
  uint8_t* on = (uint8_t*)malloc(n);
  if (!small || !gray || !on) {
    free(small);
    free(gray);
    free(on);
    return -1;
  }
  for (uint32_t f = 0; f < frames; ++f) {
    const uint8_t* src = rgb + (size_t)f * cfg->width * cfg->height * 3;
    enc_reduce(src, cfg->width, cfg->height, cfg->factor, small);
    enc_gray(small, (uint32_t)n, gray);
    enc_threshold(gray, w, h, cfg->block, cfg->offset, on);
    enc_pack(on, (uint32_t)n, words + (size_t)f * nw);
  }
  free(small);
  free(gray);
  free(on);
  return 0;
}
