// Internal interface between the C-ABI host code (sp_api.hip) and the
// kernels (sp_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace htmsp {

// Shape and learning parameters shared by every kernel, permanences in
// 1/256 units.
struct Shape {
  uint32_t N, C, S, W;      // input bits, columns, synapses per column, words per frame
  uint32_t m, k;            // min_overlap, winners_set_size
  uint32_t theta, inc, dec; // connected threshold, increment, decrement (x256)
};

// Persistent multi-frame step: one workgroup (one wave) per group of `cpw`
// consecutive columns, each column spread over `rpc` rows of 64 synapses.
struct PersistArgs {
  const uint32_t* idx;
  float* perm;
  const uint32_t* frames;
  int32_t* ov_out;    // [F][C] or null
  int32_t* win_out;   // [F][k]
  uint32_t* xchg;     // [2][C] tagged overlaps
  uint32_t* err;      // set to non-zero when a wave gives up waiting
  uint32_t F, learn, frame_base, cpw, rpc, spin_limit;
  Shape sh;
};

// Rows of 64 synapses one workgroup of the persistent kernel may hold.
constexpr int kPersistMaxRows = 64;
// Largest C the persistent kernel exchanges through LDS (uint16 per column).
constexpr uint32_t kPersistMaxColumns = 16384;

size_t persistent_lds_bytes(const Shape& sh);
// The kernel instance for `rows` (rounded up to a power of two <= 64).
const void* persistent_kernel(uint32_t rows);

hipError_t launch_check_state(const uint32_t* idx, const float* perm, size_t n, uint32_t N,
                              uint32_t* out4, hipStream_t s);
hipError_t launch_overlap_plain(const uint32_t* idx, const float* perm, const uint32_t* frame,
                                int32_t* ov, const Shape& sh, hipStream_t s);
hipError_t launch_topk_plain(const int32_t* ov, int32_t* winners, const Shape& sh, hipStream_t s);
hipError_t launch_learn_plain(const uint32_t* idx, float* perm, const uint32_t* frame,
                              const int32_t* winners, const Shape& sh, hipStream_t s);

}  // namespace htmsp
