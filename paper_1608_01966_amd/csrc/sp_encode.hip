// Adaptive video encoder (Section 3.1.2): a colour frame, optionally reduced
// in size, turned to grayscale and binarised with an adaptive threshold whose
// value at each pixel is a Gaussian-weighted sum of its neighbourhood, into
// the spatial pooler's packed input.
//
// Exact integer arithmetic throughout (so the output is bit-for-bit
// defined): block means rounded half up, BT.601 luma in 14-bit fixed point,
// the binomial window C(b-1, i) as the Gaussian (total weight 4^(b-1)),
// edge pixels repeated outside the image, mean rounded half up, on iff
// gray > mean - offset; pixel p = y w + x at bit p & 31 of word p >> 5.
//
// One workgroup per (frame, band of kBandRows output rows, strip of
// 256 - 2r output columns).  Each thread owns one column of the strip plus
// its r halo columns on either side and walks down the band: it computes
// the gray value of each input row it needs straight from the RGB frame,
// keeps the last b of them in registers and forms the vertical window sum;
// one LDS row of vertical sums per output row then gives every thread its
// horizontal window sum.  Threads of halo columns outside the image read the
// nearest edge column, so border repetition needs no special case.  When
// the output width is a multiple of 32 (rows start on word boundaries), a
// strip's output width is a multiple of 32 too (512 threads: 480 columns at
// the largest window, two strips for a 960-wide frame): two output rows
// share each barrier, every wave leaves its ballots of both in LDS and,
// after the next barrier, a thread per output word assembles and stores
// each word once, so each word is written by one store and nothing is
// cleared first.  Other widths OR each wave's
// 64-lane ballot into the (zeroed) output words it covers, which makes any
// width and strip boundary correct.  Bands of one frame share an XCD (block
// ids equal modulo 8), so the halo rows two bands both read come from L2.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

using namespace dev;

constexpr uint32_t kEncThreads = 256;       // strips OR-ed into zeroed words
constexpr uint32_t kEncWordThreads = 512;   // strips of whole words
constexpr uint32_t kBandRows = 64;

// Output columns per strip: THREADS less the halo on each side, rounded
// down to whole 32-bit words when WORDS.
template <int B, int THREADS, bool WORDS>
constexpr uint32_t strip_width() {
  return WORDS ? (uint32_t)((THREADS - 2 * (B / 2)) & ~31) : (uint32_t)(THREADS - 2 * (B / 2));
}

__global__ __launch_bounds__(256) void k_zero(uint32_t* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = 0u;
}

// ONE: no reduction (factor 1), the rows' loads issued ahead.  WORDS: the
// output width is a multiple of 32 and every word is stored whole (see
// above).
template <int B, bool ONE, int THREADS, bool WORDS>
__global__ __launch_bounds__(THREADS) void k_encode(const uint8_t* __restrict__ rgb,
                                                    uint32_t F, EncShape e,
                                                    uint32_t* __restrict__ out) {
  constexpr int R = B / 2;
  constexpr uint32_t TW = strip_width<B, THREADS, WORDS>();  // output columns per strip
  constexpr uint32_t kWaves = THREADS / kWave;
  // Output rows per barrier: two where every word is stored whole (their
  // vertical sums and ballots side by side in LDS), one where waves OR
  // their ballots into the output.
  constexpr int RPB = WORDS ? 2 : 1;
  __shared__ uint32_t vrow[2][RPB][THREADS];
  __shared__ uint64_t bal[2][RPB][WORDS ? kWaves : 1];
  const uint32_t strips = (e.w + TW - 1) / TW;
  const uint32_t bands = (e.h + kBandRows - 1) / kBandRows;
  const uint32_t per = 8 * strips * bands;
  const uint32_t f = (blockIdx.x / per) * 8 + blockIdx.x % 8;
  const uint32_t local = (blockIdx.x % per) / 8;
  if (f >= F) return;  // whole workgroup
  const uint32_t band = local / strips, strip = local % strips;
  const uint32_t tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int x = (int)(strip * TW) - R + (int)tid;  // this thread's column
  const uint32_t xc = (uint32_t)min(max(x, 0), (int)e.w - 1);
  const bool out_col = tid >= (uint32_t)R && tid < (uint32_t)R + TW && x < (int)e.w;
  const uint32_t y0 = band * kBandRows, y1 = min(y0 + kBandRows, e.h);

  // binomial weights, row B - 1 of Pascal's triangle
  uint32_t wt[B];
  wt[0] = 1;
#pragma unroll
  for (int i = 1; i < B; ++i) wt[i] = wt[i - 1] * (B - i) / i;
  constexpr uint32_t kShift = 2 * (B - 1);

  const uint8_t* src = rgb + (size_t)f * e.W * e.H * 3;
  const uint32_t fa = e.factor;
  auto gray = [&](uint32_t gy) {
    uint32_t r = 0, g = 0, b = 0;
    if (fa == 1) {
      const uint8_t* px = src + 3 * ((size_t)gy * e.W + xc);
      r = px[0];
      g = px[1];
      b = px[2];
    } else {
      for (uint32_t dy = 0; dy < fa; ++dy) {
        const uint8_t* row = src + 3 * ((size_t)(gy * fa + dy) * e.W + xc * fa);
        for (uint32_t dx = 0; dx < fa; ++dx) {
          r += row[3 * dx];
          g += row[3 * dx + 1];
          b += row[3 * dx + 2];
        }
      }
      // block means rounded half up; floor(n / area) as a high multiply
      // (exact for n < 256 area, area <= 1024)
      const uint32_t half = e.area / 2;
      r = __umulhi(r + half, e.area_magic);
      g = __umulhi(g + half, e.area_magic);
      b = __umulhi(b + half, e.area_magic);
    }
    return (4899u * r + 9617u * g + 1868u * b + 8192u) >> 14;
  };

  uint32_t win[B];  // gray values of rows y - R .. y + R of this column
#pragma unroll
  for (int i = 0; i < B - 1; ++i) win[i + 1] = gray((uint32_t)min(max((int)y0 - R + i, 0), (int)e.h - 1));
  uint32_t* dst = out + (size_t)f * e.words;
  uint32_t buf = 0;
  // WORDS: word j of output row `row` of this strip from the ballots in
  // bal[b][r] (bit t of the concatenated ballots is thread t's column).
  auto flush = [&](uint32_t row, uint32_t b, int r) {
    if constexpr (WORDS) {
      const uint32_t j = tid;
      if (row < y1 && j < TW / 32 && strip * TW + 32 * j < e.w) {
        const uint32_t start = (uint32_t)R + 32 * j, q = start >> 6, o = start & 63u;
        uint64_t v = bal[b][r][q] >> o;
        if (o > 32) v |= bal[b][r][q + 1] << (64 - o);
        dst[((size_t)row * e.w + strip * TW) / 32 + j] = (uint32_t)v;
      }
    }
  };
  // Without reduction, the RGB bytes of the row entering the window are
  // loaded kAhead rows before they are needed, into a ring indexed by the
  // unrolled row (so that no register with a load in flight is copied);
  // loads past the band's last needed row read that row again.
  constexpr int kAhead = 8;
  uint32_t pr[kAhead], pg[kAhead], pb[kAhead];
  const uint32_t last_row = min(y1 - 1 + R, e.h - 1);
  auto issue = [&](int k, uint32_t gy) {
    const uint8_t* px = src + 3 * ((size_t)min(gy, last_row) * e.W + xc);
    pr[k] = px[0];
    pg[k] = px[1];
    pb[k] = px[2];
  };
  if constexpr (ONE) {
#pragma unroll
    for (int k = 0; k < kAhead; ++k) issue(k, y0 + R + k);
  }
  for (uint32_t yb = y0; yb < y1; yb += kAhead) {
#pragma unroll
  for (int k0 = 0; k0 < kAhead; k0 += RPB) {
    uint32_t cen[RPB];  // each row's own gray value
#pragma unroll
    for (int r = 0; r < RPB; ++r) {
      const int k = k0 + r;
      const uint32_t y = yb + k;
#pragma unroll
      for (int i = 0; i < B - 1; ++i) win[i] = win[i + 1];
      if constexpr (ONE) {
        win[B - 1] = (4899u * pr[k] + 9617u * pg[k] + 1868u * pb[k] + 8192u) >> 14;
        issue(k, y + R + kAhead);
      } else {
        win[B - 1] = gray((uint32_t)min((int)y + R, (int)e.h - 1));
      }
      uint32_t v = 0;
#pragma unroll
      for (int i = 0; i < B; ++i) v += wt[i] * win[i];
      vrow[buf][r][tid] = v;
      cen[r] = win[R];
    }
    // The rows of vertical sums (and the previous rows' ballots) are the
    // only thing the barrier orders: wait for LDS only, so the row loads
    // issued ahead stay in flight across it.
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (yb + k0 > y0) {
#pragma unroll
      for (int r = 0; r < RPB; ++r) flush(yb + k0 - RPB + r, buf ^ 1u, r);
    }
#pragma unroll
    for (int r = 0; r < RPB; ++r) {
    const uint32_t y = yb + k0 + r;
    bool on = false;
    if (out_col && y < y1) {
      const uint32_t* vr = &vrow[buf][r][tid - R];
      uint32_t s = 0;
#pragma unroll
      for (int j = 0; j < B; ++j) s += wt[j] * vr[j];
      const int mean = (int)((s + (1u << (kShift - 1))) >> kShift);
      on = (int)cen[r] > mean - e.offset;
    }
    uint64_t bits = __ballot(on);
    if constexpr (WORDS) {
      if (lane == 0) bal[buf][r][wave] = bits;
      continue;
    }
    // the wave's 64 columns start at xs; output bit y * w + xs + lane
    int xs = (int)(strip * TW) - R + (int)(kWave * wave);
    if (xs < 0) {  // first strip: its left halo lanes carry no output
      bits >>= (uint32_t)(-xs);
      xs = 0;
    }
    if (bits) {
      const uint64_t base = (uint64_t)y * e.w + (uint32_t)xs;
      const uint32_t wi = (uint32_t)(base >> 5), o = (uint32_t)(base & 31u);
      uint32_t part = 0;
      if (lane == 0) part = (uint32_t)(bits << o);
      if (lane == 1) part = (uint32_t)(bits >> (32 - o));
      if (lane == 2 && o) part = (uint32_t)(bits >> (64 - o));
      if (part && wi + lane < e.words) atomicOr(&dst[wi + lane], part);
    }
    }
    buf ^= 1u;
  }
  }
  if constexpr (WORDS) {
    // the band's last rows: their ballots are in bal[buf ^ 1]
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    const uint32_t rows = (y1 - y0 + kAhead - 1) / kAhead * kAhead;
#pragma unroll
    for (int r = 0; r < RPB; ++r) flush(y0 + rows - RPB + r, buf ^ 1u, r);
  }
}

}  // namespace

hipError_t launch_encode(const uint8_t* rgb, uint32_t F, const EncShape& e, uint32_t* out,
                         hipStream_t s) {
  if (F == 0) return hipSuccess;
  const bool words = e.w % 32 == 0;
  if (!words) {
    const size_t n = (size_t)F * e.words;
    size_t zb = (n + 255) / 256;
    if (zb > 4096) zb = 4096;
    hipLaunchKernelGGL(k_zero, dim3((uint32_t)zb), dim3(256), 0, s, out, n);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  const uint32_t bands = (e.h + kBandRows - 1) / kBandRows;
  auto blocks = [&](uint32_t tw) { return (F + 7) / 8 * 8 * ((e.w + tw - 1) / tw) * bands; };
#define HTMSP_ENC_GO(B, ONE, T, WD)                                                            \
  hipLaunchKernelGGL((k_encode<B, ONE, T, WD>), dim3(blocks(strip_width<B, T, WD>())), dim3(T), \
                     0, s, rgb, F, e, out)
#define HTMSP_ENC(B)                                                                  \
  case B:                                                                             \
    if (words) {                                                                      \
      if (e.factor == 1) HTMSP_ENC_GO(B, true, kEncWordThreads, true);                \
      else HTMSP_ENC_GO(B, false, kEncWordThreads, true);                             \
    } else {                                                                          \
      if (e.factor == 1) HTMSP_ENC_GO(B, true, kEncThreads, false);                   \
      else HTMSP_ENC_GO(B, false, kEncThreads, false);                                \
    }                                                                                 \
    break;
  switch (e.block) {
    HTMSP_ENC(3) HTMSP_ENC(5) HTMSP_ENC(7) HTMSP_ENC(9) HTMSP_ENC(11)
    default:
      return hipErrorInvalidValue;
  }
#undef HTMSP_ENC
#undef HTMSP_ENC_GO
  return hipGetLastError();
}

}  // namespace htmsp
