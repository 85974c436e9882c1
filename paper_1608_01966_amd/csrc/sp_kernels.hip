// HIP kernels for the HTM spatial pooler step on gfx950 (wave64).
//
// Section 1.1 of Wielgosz & Pietron (arXiv 1608.01966) splits a step into
// overlap (Algorithm 1), inhibition (Algorithm 2) and learning.  Two
// executions are provided:
//   * plain: three kernels per frame (overlap, global top-k, learning), the
//     state read from and written to HBM every frame;
//   * persistent: one cooperative launch for F frames.  Each workgroup keeps
//     the synapses of its columns in registers for the whole launch, gathers
//     the input bits of the next frame while it waits, exchanges per-frame
//     overlaps with all other workgroups through a tagged device buffer, and
//     resolves the global top-k redundantly so that every workgroup knows
//     which of its own columns learn, with no second exchange.
// Permanences are handled as integers q = 256 * permanence (0..256), so
// every comparison and update is exact.
#include "sp_internal.h"

namespace htmsp {

namespace {

constexpr uint32_t kWave = 64;

__device__ __forceinline__ uint32_t perm_to_q(float p) {
  int q = (int)(p * 256.0f);
  return (uint32_t)min(max(q, 0), 256);
}

__device__ __forceinline__ float q_to_perm(uint32_t q) { return (float)q * (1.0f / 256.0f); }

__device__ __forceinline__ uint32_t input_bit(uint32_t word, uint32_t i) {
  return (word >> (i & 31u)) & 1u;
}

__device__ __forceinline__ uint32_t learn_q(uint32_t q, uint32_t bit, const Shape& sh) {
  return bit ? min(q + sh.inc, 256u) : (uint32_t)max((int)q - (int)sh.dec, 0);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ uint64_t lanemask_lt(uint32_t lane) { return (1ull << lane) - 1ull; }

__device__ __forceinline__ uint32_t load_tagged(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_tagged(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// State validation: counts indices >= N and permanences off the 1/256 grid,
// remembering the first offending position of each kind.
__global__ __launch_bounds__(256) void k_check_state(const uint32_t* __restrict__ idx,
                                                     const float* __restrict__ perm, size_t n,
                                                     uint32_t N, uint32_t* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    if (idx[i] >= N) {
      atomicAdd(&out[0], 1u);
      atomicMin(&out[2], (uint32_t)i);
    }
    const float q = perm[i] * 256.0f;
    if (!(q >= 0.0f && q <= 256.0f && q == rintf(q))) {
      atomicAdd(&out[1], 1u);
      atomicMin(&out[3], (uint32_t)i);
    }
  }
}

// ---------------------------------------------------------------------------
// Plain overlap (Algorithm 1): one wave per column, 64 synapses per ballot.
__global__ __launch_bounds__(256) void k_overlap_plain(const uint32_t* __restrict__ idx,
                                                       const float* __restrict__ perm,
                                                       const uint32_t* __restrict__ frame,
                                                       int32_t* __restrict__ ov, Shape sh) {
  const uint32_t lane = threadIdx.x % kWave;
  const uint32_t c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (c >= sh.C) return;
  const uint32_t* ci = idx + (size_t)c * sh.S;
  const float* cp = perm + (size_t)c * sh.S;
  uint32_t raw = 0;
  for (uint32_t s0 = 0; s0 < sh.S; s0 += kWave) {
    const uint32_t s = s0 + lane;
    bool hit = false;
    if (s < sh.S) {
      const uint32_t i = min(ci[s], sh.N - 1);
      if (perm_to_q(cp[s]) >= sh.theta) hit = input_bit(frame[i >> 5], i);
    }
    raw += (uint32_t)__popcll(__ballot(hit));
  }
  if (lane == 0) ov[c] = raw >= sh.m ? (int32_t)raw : 0;
}

// ---------------------------------------------------------------------------
// Plain global top-k (Algorithm 2, global form) in one workgroup of 1024.
// T = the largest value x >= 1 with #(overlap >= x) >= k (0 if fewer than k
// overlaps are positive) is found by binary search on block-wide counts;
// then every column above T wins, and the lowest-index columns equal to T
// fill the remaining k - #(overlap > T) slots.  Winners are compacted in
// column order with ballot prefix counts.
constexpr uint32_t kTopkThreads = 1024;

__device__ uint32_t block_count(uint32_t flag_count, uint32_t* red) {
  const uint32_t lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const uint32_t w = wave_sum(flag_count);
  __syncthreads();
  if (lane == 0) red[wave] = w;
  __syncthreads();
  uint32_t tot = 0;
  for (uint32_t i = 0; i < blockDim.x / kWave; ++i) tot += red[i];
  return tot;
}

// Exclusive prefix of a 0/1 flag over the block in thread order; *total gets
// the block total.
__device__ uint32_t block_excl_scan(bool flag, uint32_t* red, uint32_t* total) {
  const uint32_t lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const uint64_t b = __ballot(flag);
  __syncthreads();
  if (lane == 0) red[wave] = (uint32_t)__popcll(b);
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (uint32_t i = 0; i < blockDim.x / kWave; ++i) {
    if (i < wave) before += red[i];
    tot += red[i];
  }
  *total = tot;
  return before + (uint32_t)__popcll(b & lanemask_lt(lane));
}

__global__ __launch_bounds__(kTopkThreads) void k_topk_plain(const int32_t* __restrict__ ov,
                                                            int32_t* __restrict__ winners,
                                                            Shape sh) {
  __shared__ uint32_t red[kTopkThreads / kWave];
  const uint32_t tid = threadIdx.x;
  auto count_ge = [&](int32_t x) {
    uint32_t n = 0;
    for (uint32_t c = tid; c < sh.C; c += blockDim.x) n += ov[c] >= x;
    return block_count(n, red);
  };
  int32_t T = 0;
  uint32_t need = 0;
  if (count_ge(1) >= sh.k) {
    int32_t lo = 1, hi = (int32_t)sh.S;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) / 2;
      if (count_ge(mid) >= sh.k) lo = mid; else hi = mid - 1;
    }
    T = lo;
    need = sh.k - count_ge(T + 1);
  }
  uint32_t eq_base = 0, sel_base = 0;
  for (uint32_t c0 = 0; c0 < sh.C; c0 += blockDim.x) {
    const uint32_t c = c0 + tid;
    const int32_t v = c < sh.C ? ov[c] : 0;
    const bool gt = v > T && v > 0;
    const bool eq = T > 0 && v == T;
    uint32_t eq_tot, sel_tot;
    const uint32_t eq_pre = eq_base + block_excl_scan(eq, red, &eq_tot);
    const bool sel = gt || (eq && eq_pre < need);
    const uint32_t pos = sel_base + block_excl_scan(sel, red, &sel_tot);
    if (sel) winners[pos] = (int32_t)c;
    eq_base += eq_tot;
    sel_base += sel_tot;
  }
  for (uint32_t i = sel_base + tid; i < sh.k; i += blockDim.x) winners[i] = -1;
}

// ---------------------------------------------------------------------------
// Plain learning: one workgroup per winner slot.
__global__ __launch_bounds__(256) void k_learn_plain(const uint32_t* __restrict__ idx,
                                                     float* __restrict__ perm,
                                                     const uint32_t* __restrict__ frame,
                                                     const int32_t* __restrict__ winners,
                                                     Shape sh) {
  const int32_t c = winners[blockIdx.x];
  if (c < 0) return;
  const uint32_t* ci = idx + (size_t)c * sh.S;
  float* cp = perm + (size_t)c * sh.S;
  for (uint32_t s = threadIdx.x; s < sh.S; s += blockDim.x) {
    const uint32_t i = min(ci[s], sh.N - 1);
    cp[s] = q_to_perm(learn_q(perm_to_q(cp[s]), input_bit(frame[i >> 5], i), sh));
  }
}

// ---------------------------------------------------------------------------
// Persistent multi-frame step.  Workgroup g (one wave) owns columns
// [g*cpw, g*cpw + ncols); row r of its register state holds synapses
// (r % rpc)*64 + lane of local column r / rpc, packed as idx << 9 | q.
constexpr uint32_t kPollBatch = 16;

template <int ROWS>
__global__ __launch_bounds__(64) void k_sp_persistent(PersistArgs a) {
  extern __shared__ uint32_t lds[];
  const Shape sh = a.sh;
  uint16_t* ovs = reinterpret_cast<uint16_t*>(lds);  // [C] overlaps of the frame
  uint32_t* hist = lds + ((sh.C + 1) / 2);            // [S + 1] overlap histogram
  const uint32_t lane = threadIdx.x;
  const uint32_t c_begin = blockIdx.x * a.cpw;
  const uint32_t ncols = min(a.cpw, sh.C - c_begin);
  const uint32_t nrows = ncols * a.rpc;

  // Invalid slots (past S, or past the workgroup's last column) load from
  // offset 0 and are masked out by `valid`, so no load depends on a branch.
  uint32_t st[ROWS], wc[ROWS], wn[ROWS];
  uint64_t valid = 0;  // bit r: this lane holds a synapse in row r
  {
    uint32_t j = 0, rr = 0;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const uint32_t s = rr * kWave + lane;
      const bool ok = (uint32_t)r < nrows && s < sh.S;
      const size_t off = ok ? (size_t)(c_begin + j) * sh.S + s : 0;
      const uint32_t i = min(a.idx[off], sh.N - 1);
      const uint32_t packed = (i << 9) | perm_to_q(a.perm[off]);
      st[r] = ok ? packed : 0u;
      valid |= (uint64_t)ok << r;
      if (++rr == a.rpc) { rr = 0; ++j; }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      wc[r] = a.frames[(st[r] >> 9) >> 5];
      wn[r] = 0;
    }
  }
  for (uint32_t v = lane; v <= sh.S; v += kWave) hist[v] = 0;
  __syncthreads();

  bool abort = false;
  for (uint32_t t = 0; t < a.F && !abort; ++t) {
    // Overlap of the own columns (Algorithm 1): lane j accumulates column j.
    uint32_t myraw = 0;
    {
      uint32_t j = 0, rr = 0;
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        const uint32_t i = st[r] >> 9, q = st[r] & 511u;
        const bool hit = ((valid >> r) & 1ull) && q >= sh.theta && input_bit(wc[r], i);
        const uint32_t pc = (uint32_t)__popcll(__ballot(hit));
        myraw += lane == j ? pc : 0u;
        if (++rr == a.rpc) { rr = 0; ++j; }
      }
    }
    const bool mine = lane < ncols;
    const uint32_t my_ov = (mine && myraw >= sh.m) ? myraw : 0u;

    // Publish, tagged with the frame's global sequence number.
    const uint32_t g = a.frame_base + t;
    const uint32_t tag = (g + 1u) & 0xFFFFu;
    uint32_t* xs = a.xchg + (size_t)(g & 1u) * sh.C;
    if (mine) store_tagged(xs + c_begin + lane, (tag << 16) | my_ov);

    // Gather the next frame's input words while the others publish.
    if (t + 1 < a.F) {
      const uint32_t* fr = a.frames + (size_t)(t + 1) * sh.W;
#pragma unroll
      for (int r = 0; r < ROWS; ++r) wn[r] = fr[(st[r] >> 9) >> 5];
    }

    // Collect every column's overlap and histogram the positive ones.
    uint32_t spins = 0;
    for (uint32_t base = 0; base < sh.C && !abort; base += kWave * kPollBatch) {
      uint32_t v[kPollBatch];
#pragma unroll
      for (uint32_t u = 0; u < kPollBatch; ++u) {
        const uint32_t c = base + u * kWave + lane;
        v[u] = c < sh.C ? load_tagged(xs + c) : (tag << 16);
      }
      while (true) {
        bool ok = true;
#pragma unroll
        for (uint32_t u = 0; u < kPollBatch; ++u) ok = ok && (v[u] >> 16) == tag;
        if (__all(ok)) break;
        if (++spins > a.spin_limit || ((spins & 63u) == 0 && load_tagged(a.err) != 0)) {
          abort = true;
          break;
        }
#pragma unroll
        for (uint32_t u = 0; u < kPollBatch; ++u) {
          const uint32_t c = base + u * kWave + lane;
          if ((v[u] >> 16) != tag) v[u] = load_tagged(xs + c);
        }
      }
      if (abort) break;
#pragma unroll
      for (uint32_t u = 0; u < kPollBatch; ++u) {
        const uint32_t c = base + u * kWave + lane;
        const uint32_t val = v[u] & 0xFFFFu;
        if (c < sh.C) {
          ovs[c] = (uint16_t)val;
          if (val) atomicAdd(&hist[val], 1u);
        }
      }
    }
    if (abort) break;
    __syncthreads();

    // Threshold T: the largest x >= 1 with #(overlap >= x) >= k, else 0.
    // Lane l sums the bins of values [1 + l*B, (l+1)*B]; a suffix scan over
    // lanes gives #(overlap >= 1 + l*B).
    const uint32_t B = (sh.S + kWave - 1) / kWave;
    const uint32_t vlo = 1 + lane * B, vhi = min(sh.S, (lane + 1) * B);
    uint32_t suf = 0;
    for (uint32_t x = vlo; x <= vhi; ++x) suf += hist[x];
#pragma unroll
    for (uint32_t off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_down(suf, off);
      if (lane + off < kWave) suf += y;
    }
    const uint32_t npos = __shfl(suf, 0);
    const uint64_t reach = __ballot(suf >= sh.k);
    uint32_t T = 0, cnt_gt = npos;
    if (reach) {
      const uint32_t L = 63u - (uint32_t)__clzll(reach);
      const uint32_t above_l = __shfl(suf, (int)min(L + 1, 63u));
      uint32_t acc = (L == 63u) ? 0u : above_l;
      const uint32_t lo = 1 + L * B, hi = min(sh.S, (L + 1) * B);
      for (uint32_t x = hi; x >= lo; --x) {
        const uint32_t h = hist[x];
        if (acc + h >= sh.k) {
          T = x;
          cnt_gt = acc;
          break;
        }
        acc += h;
      }
    }
    const uint32_t need = T ? sh.k - cnt_gt : 0u;
    const uint32_t nsel = T ? sh.k : npos;

    // Rank of the own columns among the winners, in column order.
    uint32_t gtb = 0, eqb = 0;
    for (uint32_t c = lane; c < c_begin; c += kWave) {
      const uint32_t v = ovs[c];
      gtb += v > T;
      eqb += (T != 0) & (v == T);
    }
    gtb = wave_sum(gtb);
    eqb = wave_sum(eqb);
    const bool gt = mine && my_ov > T;
    const bool eq = mine && T != 0 && my_ov == T;
    const uint32_t gt_pre = gtb + (uint32_t)__popcll(__ballot(gt) & lanemask_lt(lane));
    const uint32_t eq_pre = eqb + (uint32_t)__popcll(__ballot(eq) & lanemask_lt(lane));
    const bool sel = gt || (eq && eq_pre < need);
    int32_t* wrow = a.win_out + (size_t)t * sh.k;
    if (sel) wrow[gt_pre + min(eq_pre, need)] = (int32_t)(c_begin + lane);
    if (blockIdx.x == 0)
      for (uint32_t i = nsel + lane; i < sh.k; i += kWave) wrow[i] = -1;
    if (a.ov_out && mine) a.ov_out[(size_t)t * sh.C + c_begin + lane] = (int32_t)my_ov;

    // Learning on the own winning columns, with the bits of this frame.
    if (a.learn) {
      const uint64_t selm = __ballot(sel);
      uint32_t j = 0, rr = 0;
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        const bool upd = ((selm >> j) & 1ull) && ((valid >> r) & 1ull);
        const uint32_t i = st[r] >> 9, q = st[r] & 511u;
        st[r] = upd ? (i << 9) | learn_q(q, input_bit(wc[r], i), sh) : st[r];
        if (++rr == a.rpc) { rr = 0; ++j; }
      }
    }
    __syncthreads();
    for (uint32_t v = lane; v <= sh.S; v += kWave) hist[v] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROWS; ++r) wc[r] = wn[r];
  }

  if (abort) {
    if (lane == 0) store_tagged(a.err, 1u);
    return;
  }
  if (a.learn) {
    uint32_t j = 0, rr = 0;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      if ((valid >> r) & 1ull)
        a.perm[(size_t)(c_begin + j) * sh.S + rr * kWave + lane] = q_to_perm(st[r] & 511u);
      if (++rr == a.rpc) { rr = 0; ++j; }
    }
  }
}

}  // namespace

size_t persistent_lds_bytes(const Shape& sh) {
  return sizeof(uint32_t) * (((size_t)sh.C + 1) / 2 + (size_t)sh.S + 1);
}

const void* persistent_kernel(uint32_t rows) {
  if (rows <= 1) return reinterpret_cast<const void*>(&k_sp_persistent<1>);
  if (rows <= 2) return reinterpret_cast<const void*>(&k_sp_persistent<2>);
  if (rows <= 4) return reinterpret_cast<const void*>(&k_sp_persistent<4>);
  if (rows <= 8) return reinterpret_cast<const void*>(&k_sp_persistent<8>);
  if (rows <= 16) return reinterpret_cast<const void*>(&k_sp_persistent<16>);
  if (rows <= 32) return reinterpret_cast<const void*>(&k_sp_persistent<32>);
  if (rows <= 64) return reinterpret_cast<const void*>(&k_sp_persistent<64>);
  return nullptr;
}

hipError_t launch_check_state(const uint32_t* idx, const float* perm, size_t n, uint32_t N,
                              uint32_t* out4, hipStream_t s) {
  const uint32_t init[4] = {0u, 0u, 0xFFFFFFFFu, 0xFFFFFFFFu};
  hipError_t e = hipMemcpyAsync(out4, init, sizeof(init), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_check_state, dim3((uint32_t)blocks), dim3(256), 0, s, idx, perm, n, N, out4);
  return hipGetLastError();
}

hipError_t launch_overlap_plain(const uint32_t* idx, const float* perm, const uint32_t* frame,
                                int32_t* ov, const Shape& sh, hipStream_t s) {
  const uint32_t waves_per_block = 4;
  const uint32_t blocks = (sh.C + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(k_overlap_plain, dim3(blocks), dim3(waves_per_block * kWave), 0, s, idx,
                     perm, frame, ov, sh);
  return hipGetLastError();
}

hipError_t launch_topk_plain(const int32_t* ov, int32_t* winners, const Shape& sh,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_topk_plain, dim3(1), dim3(kTopkThreads), 0, s, ov, winners, sh);
  return hipGetLastError();
}

hipError_t launch_learn_plain(const uint32_t* idx, float* perm, const uint32_t* frame,
                              const int32_t* winners, const Shape& sh, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_plain, dim3(sh.k), dim3(256), 0, s, idx, perm, frame, winners, sh);
  return hipGetLastError();
}

}  // namespace htmsp
