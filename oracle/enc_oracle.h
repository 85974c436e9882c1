/*
 * Oracle for the adaptive video encoder -- TEST INFRASTRUCTURE ONLY.
 *
 * Section 3.1.2 of Wielgosz & Pietron (arXiv 1608.01966) turns each video
 * frame into the spatial pooler's binary input: the colour frame may first
 * be reduced in size, is converted to grayscale, and is binarised with an
 * adaptive threshold whose value at each pixel is a Gaussian-weighted sum of
 * the pixel's neighbourhood (OpenCV's Gaussian adaptive method).  The paper
 * names the steps only; this oracle fixes each one as an exact integer
 * operation (readings E1-E6, also listed in the design notes):
 *   E1  input: 8-bit RGB, pixel (y, x) at bytes 3 (y W + x) + {0, 1, 2};
 *   E2  reduction by an integer factor f: each output pixel is the mean of
 *       its f x f input block per channel, rounded half up; the output is
 *       floor(W / f) x floor(H / f) (a trailing partial block is dropped);
 *   E3  grayscale: BT.601 luma weights 0.299, 0.587, 0.114 in 14-bit fixed
 *       point, Y = (4899 R + 9617 G + 1868 B + 8192) >> 14;
 *   E4  Gaussian window: the binomial weights C(b - 1, i), i < b, for an odd
 *       block size b (the discrete Gaussian; 3 <= b <= 11), in both
 *       directions; pixels outside the image repeat the nearest edge pixel;
 *   E5  threshold: the weighted mean is the window sum over 4^(b-1),
 *       rounded half up; a pixel is on iff Y > mean - offset;
 *   E6  output: the SP input layout, pixel p = y w + x at bit p & 31 of word
 *       p >> 5, least significant bit first, trailing bits zero.
 * It shares no code with the GPU library.
 */
#ifndef ENC_ORACLE_H
#define ENC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct enc_config {
  uint32_t width, height; /* input frame size in pixels            */
  uint32_t factor;        /* integer reduction factor, 1 = none    */
  uint32_t block;         /* odd neighbourhood size b, 3..11       */
  int32_t offset;         /* constant subtracted from the mean     */
} enc_config;

/* E2 on one channel-interleaved RGB frame: out is [H/f][W/f][3]. */
void enc_reduce(const uint8_t* rgb, uint32_t width, uint32_t height, uint32_t factor,
                uint8_t* out);

/* E3 per pixel: gray[i] from rgb[3 i .. 3 i + 2], n pixels. */
void enc_gray(const uint8_t* rgb, uint32_t n, uint8_t* gray);

/* E4-E5 on a w x h grayscale image: on[y w + x] is 0 or 1.  The window sum
 * is taken directly over the b x b neighbourhood. */
void enc_threshold(const uint8_t* gray, uint32_t w, uint32_t h, uint32_t block, int32_t offset,
                   uint8_t* on);

/* E6: n 0/1 values into ceil(n / 32) words. */
void enc_pack(const uint8_t* on, uint32_t n, uint32_t* words);

/* The whole encoder on `frames` frames ([F][H][W][3] bytes) into
 * [F][ceil(w h / 32)] words, w = W / f, h = H / f.  Returns 0, or -1 on a
 * bad configuration. */
int enc_frames(const enc_config* cfg, const uint8_t* rgb, uint32_t frames, uint32_t* words);

#ifdef __cplusplus
}
#endif

#endif
