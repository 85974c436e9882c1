// Many independent spatial pooler instances stepped by one persistent
// launch (Section 3.1's 'Multiple HTMs' setup runs one pooler per category;
// serving runs one per video stream).  Each instance still follows Section
// 1.1 frame by frame -- overlap, global inhibition, learning -- so its frames
// are sequential, but the instances are independent: while one waits for its
// inhibition, the GPU works on the others.
//
// Work is split into tasks, assigned statically to the workgroups of a
// cooperative grid (in each workgroup, tile tasks before top-k tasks):
//   tile task (instance, columns [c0, c1)), at most kTileSynapses synapses,
//     the whole workgroup: for step t it applies learning of frame t-1 to its
//     winning columns, then computes the overlaps of frame t and publishes
//     them.  Each thread owns up to 32 synapses of the tile's flat
//     [column][synapse] range and issues all their state loads before the
//     wait for the previous decision, then both input gathers at once;
//     per-column counts are summed in LDS, and each tile keeps its last
//     published overlaps in LDS to decide its winners.
//   top-k task (instance), wave 0: for step t it collects the instance's
//     overlaps, resolves the global top-k, writes the frame's outputs (and
//     adds the winners to the instance's histogram, if it has one) and
//     publishes a decision word from which every tile derives which of its
//     columns won.
// Synapse state is read from and written to device memory every step (the
// instances' state does not fit on chip together).  Every cross-workgroup
// value carries its step's tag (overlap entries [tag:16 | overlap:16],
// decision [tag:16 | T:16 | last tied winner + 1:32]) and is written and read
// with agent-scope atomics, so no fence is needed; a tag never matches a
// value left by an earlier step, and an instance's buffers are rewritten only
// after their readers are done with them (tiles wait for the previous
// decision, which the top-k task publishes after reading every overlap).
// Aborts (spin limit, error word) are made uniform over the workgroup before
// its next barrier, so a failing launch still drains.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

using namespace dev;

constexpr uint32_t kPerThread = kTileSynapses / kManyThreads;  // 32

__device__ __forceinline__ uint64_t load_word(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_word64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until the instance's decision word carries `tag`; false on abort.
__device__ bool wait_decision(const ManyInst& in, uint32_t tag, const ManyArgs& a,
                              uint64_t* out) {
  uint32_t spins = 0;
  while (true) {
    const uint64_t d = load_word(in.dec);
    if ((uint32_t)(d >> 48) == tag) {
      *out = d;
      return true;
    }
    if (++spins > a.spin_limit || ((spins & 63u) == 0 && load_tagged(a.err) != 0)) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

// floor(p / S) for p < 2^24 from a float reciprocal, corrected to exact.
__device__ __forceinline__ uint32_t div_s(uint32_t p, uint32_t S, float invS) {
  uint32_t q = (uint32_t)((float)p * invS);
  if (q * S > p) --q;
  else if ((q + 1) * S <= p) ++q;
  return q;
}

struct TileLds {
  uint32_t cnt[kTileColumns];                 // raw overlap counts of the step
  uint16_t prev[kMaxTileSlots][kTileColumns];  // each tile's published overlaps of the last step
  uint32_t bc[3];                             // ok, T, last tied winner + 1
};

// Tile task `slot` of this workgroup, whole workgroup.  Returns false
// (uniformly) on abort.
__device__ bool tile_step(const ManyArgs& a, const ManyInst& in, uint32_t c0, uint32_t c1,
                          uint32_t t, uint32_t slot, TileLds& L) {
  const Shape& sh = in.sh;
  const uint32_t tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const uint32_t tag_prev = (in.step_base + t) & 0xFFFFu;  // tag of step t - 1
  const uint32_t tag = (in.step_base + t + 1) & 0xFFFFu;
  const uint32_t ncol = c1 - c0, nsyn = ncol * sh.S;
  const bool learn_now = a.learn && t > 0;
  const bool overlap_now = t < in.F;

  // The state does not depend on the decision: its loads are in flight
  // while thread 0 waits.
  const size_t p0 = (size_t)c0 * sh.S;
  const uint32_t* gidx = in.idx + p0;
  float* gperm = in.perm + p0;
  const float invS = 1.0f / (float)sh.S;
  uint32_t ix[kPerThread], q[kPerThread];
#pragma unroll
  for (uint32_t j = 0; j < kPerThread; ++j) {
    const uint32_t p = tid + kManyThreads * j;
    const bool v = p < nsyn;
    ix[j] = v ? min(gidx[p], sh.N - 1) : 0u;
    q[j] = v ? perm_to_q(gperm[p]) : 0u;
  }
  if (tid == 0) {
    uint64_t d = 0;
    const bool ok = t == 0 || wait_decision(in, tag_prev, a, &d);
    L.bc[0] = ok;
    L.bc[1] = (uint32_t)(d >> 32) & 0xFFFFu;
    L.bc[2] = (uint32_t)d;
  }
  __syncthreads();
  if (!L.bc[0]) return false;
  const uint32_t T = L.bc[1], clast1 = L.bc[2];

  // Which synapses belong to a column that won frame t - 1 (its overlap of
  // that frame is the one this tile published last step), then both input
  // gathers in one round: frame t - 1 for learning, frame t for every
  // synapse that can be connected after learning.
  const uint32_t* fprev = in.frames + (size_t)(learn_now ? t - 1 : 0) * sh.W;
  const uint32_t* fcur = in.frames + (size_t)(overlap_now ? t : 0) * sh.W;
  uint32_t won = 0;  // bit j: synapse j belongs to a winner
  uint32_t wp[kPerThread], wc[kPerThread];
#pragma unroll
  for (uint32_t j = 0; j < kPerThread; ++j) {
    const uint32_t p = tid + kManyThreads * j;
    bool wj = false;
    if (learn_now && p < nsyn) {
      const uint32_t cl = div_s(p, sh.S, invS);
      const uint32_t prev = L.prev[slot][cl];
      wj = prev > T || (T != 0 && prev == T && c0 + cl + 1 <= clast1);
    }
    won |= (uint32_t)wj << j;
    wp[j] = wj ? fprev[ix[j] >> 5] : 0u;
    const bool maybe = overlap_now && p < nsyn && (wj ? q[j] + sh.inc : q[j]) >= sh.theta;
    wc[j] = maybe ? fcur[ix[j] >> 5] : 0u;
  }
  if (won) {
#pragma unroll
    for (uint32_t j = 0; j < kPerThread; ++j) {
      if (won & (1u << j)) {
        q[j] = learn_q(q[j], input_bit(wp[j], ix[j]), sh);
        gperm[tid + kManyThreads * j] = q_to_perm(q[j]);
      }
    }
  }
  if (overlap_now) {
#pragma unroll
    for (uint32_t j = 0; j < kPerThread; ++j) {
      const uint32_t pb = kManyThreads * j + kWave * wave;  // first flat position of the chunk
      const bool hit = (pb + lane < nsyn) && q[j] >= sh.theta && input_bit(wc[j], ix[j]);
      const uint64_t mask = __ballot(hit);
      if (pb < nsyn && mask) {
        // columns that meet the chunk [pb, pb + 64): lane l counts column clA + l
        const uint32_t clA = div_s(pb, sh.S, invS);
        const uint32_t clB = div_s(min(pb + kWave, nsyn) - 1, sh.S, invS);
        const uint32_t cl = clA + lane;
        if (cl <= clB) {
          const uint32_t lo = max(cl * sh.S, pb) - pb;
          const uint32_t hi = min((cl + 1) * sh.S, pb + kWave) - pb;
          const uint64_t bits = hi - lo == 64 ? mask : (mask >> lo) & ((1ull << (hi - lo)) - 1);
          const uint32_t n = (uint32_t)__popcll(bits);
          if (n) atomicAdd(&L.cnt[cl], n);
        }
      }
    }
  }
  __syncthreads();
  if (overlap_now) {
    for (uint32_t cl = tid; cl < ncol; cl += kManyThreads) {
      const uint32_t raw = L.cnt[cl];
      L.cnt[cl] = 0;
      const uint32_t ov = raw >= sh.m ? raw : 0u;
      L.prev[slot][cl] = (uint16_t)ov;
      store_tagged(in.ovx + c0 + cl, (tag << 16) | ov);
    }
  }
  return true;
}

// Top-k task, one wave: collects the instance's overlaps of step t, resolves
// the global top-k, writes the outputs and publishes the decision.  Lane l
// holds columns u * 256 + 4l + q (q < 4) as the 16-bit fields of ev[u].
__device__ bool topk_step(const ManyArgs& a, ManyInst& in, uint32_t t, uint32_t lane) {
  const Shape& sh = in.sh;
  const uint32_t tag = (in.step_base + t + 1) & 0xFFFFu;
  const uint32_t nv = (sh.C + 4 * kWave - 1) / (4 * kWave);
  const uint64_t* src = reinterpret_cast<const uint64_t*>(in.ovx);
  // two 64-bit loads (columns c, c + 1 and c + 2, c + 3) per word, all in
  // flight at once; stale pairs are loaded again until every tag matches
  uint64_t raw[2 * kManyNV];
#pragma unroll
  for (uint32_t i = 0; i < 2 * kManyNV; ++i) {
    const uint32_t c = (i / 2) * 4 * kWave + 4 * lane + 2 * (i % 2);
    raw[i] = (i / 2 < nv && c < sh.C) ? load_word(src + c / 2) : 0ull;
  }
  uint32_t spins = 0;
  bool bad = false;
  while (true) {
    uint32_t stale = 0;
#pragma unroll
    for (uint32_t i = 0; i < 2 * kManyNV; ++i) {
      const uint32_t c = (i / 2) * 4 * kWave + 4 * lane + 2 * (i % 2);
      if (i / 2 < nv && c < sh.C) {
        const bool ok0 = (uint32_t)(raw[i] >> 16) % 65536u == tag;
        const bool ok1 = c + 1 >= sh.C || (uint32_t)(raw[i] >> 48) == tag;
        stale |= (uint32_t)!(ok0 && ok1) << i;
      }
    }
    if (!__any(stale != 0)) break;
    if (++spins > a.spin_limit || ((spins & 63u) == 0 && load_tagged(a.err) != 0)) {
      bad = true;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (uint32_t i = 0; i < 2 * kManyNV; ++i)
      if (stale & (1u << i)) {
        const uint32_t c = (i / 2) * 4 * kWave + 4 * lane + 2 * (i % 2);
        raw[i] = load_word(src + c / 2);
      }
  }
  if (bad) return false;
  uint64_t ev[kManyNV];
#pragma unroll
  for (uint32_t u = 0; u < kManyNV; ++u) {
    uint64_t v = 0;
    if (u < nv) {
      const uint32_t c = u * 4 * kWave + 4 * lane;
      const uint64_t r0 = raw[2 * u], r1 = raw[2 * u + 1];
      v = (r0 & 0xFFFFull) | (c + 1 < sh.C ? ((r0 >> 32) & 0xFFFFull) << 16 : 0ull) |
          (c + 2 < sh.C ? (r1 & 0xFFFFull) << 32 : 0ull) |
          (c + 3 < sh.C ? ((r1 >> 32) & 0xFFFFull) << 48 : 0ull);
      if (c >= sh.C) v = 0;
    }
    ev[u] = v;
  }
  uint32_t c_hi;
  const uint32_t T = topk_threshold(ev, sh.S, sh.k, in.guess, &c_hi);
  const uint32_t need = T ? sh.k - c_hi : 0u;
  const uint32_t nsel = T ? sh.k : c_hi;
  if (T) in.guess = T;
  uint64_t fm[kManyNV];
  select_all(ev, T, need, lane, fm);

  int32_t* wrow = in.win_out + (size_t)t * sh.k;
  uint32_t base = 0, clast1 = 0;
  const uint64_t k_ge = (uint64_t)(0x8000u - (T ? T : 1u)) * kOnes16;
  const uint64_t k_gt = (uint64_t)(0x8000u - (T + 1)) * kOnes16;
#pragma unroll
  for (uint32_t u = 0; u < kManyNV; ++u) {
    if (u < nv) {
      const uint64_t sel = fm[u] & kHighBits;
      const uint64_t eq =
          T ? (((ev[u] + k_ge) & kHighBits) & ~((ev[u] + k_gt) & kHighBits)) & sel : 0ull;
      const uint32_t n = (uint32_t)__popcll(sel);
      uint32_t pos = base + wave_prefix<3>(n, lane);
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t c = u * 4 * kWave + 4 * lane + q;
        if (sel & (0x8000ull << (16 * q))) {
          wrow[pos] = (int32_t)c;
          ++pos;
          // this wave is the instance's only histogram writer in the launch
          if (in.hist) in.hist[c] += 1u;
        }
        if (eq & (0x8000ull << (16 * q))) clast1 = max(clast1, c + 1);
        if (in.ov_out && c < sh.C)
          in.ov_out[(size_t)t * sh.C + c] = (int32_t)((ev[u] >> (16 * q)) & 0xFFFFu);
      }
      base += wave_count<3>(n);
    }
  }
  for (uint32_t i = nsel + lane; i < sh.k; i += kWave) wrow[i] = -1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) clast1 = max(clast1, (uint32_t)__shfl_xor(clast1, off));
  if (lane == 0)
    store_word64(in.dec, ((uint64_t)tag << 48) | ((uint64_t)T << 32) | (uint64_t)clast1);
  return true;
}

// Two waves per SIMD (at most 256 registers): two tiles in flight per CU
// already keep more bytes in flight than device memory needs to stream.
__global__ __launch_bounds__(kManyThreads, 2) void k_sp_many(ManyArgs a) {
  __shared__ TileLds L;
  // per-step abort flags, alternating so that a flag is never written while
  // a slower thread may still read the previous step's one
  __shared__ uint32_t s_ok[2];
  const uint32_t wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  for (uint32_t i = threadIdx.x; i < kTileColumns; i += kManyThreads) L.cnt[i] = 0;
  if (threadIdx.x == 0) s_ok[0] = s_ok[1] = 1;
  __syncthreads();
  const uint32_t t0 = a.task_off[blockIdx.x], t1 = a.task_off[blockIdx.x + 1];
  bool ok = true;
  for (uint32_t t = 0; t <= a.Fmax && ok; ++t) {
    for (uint32_t j = t0; j < t1 && ok; ++j) {
      const ManyTask task = a.tasks[j];
      ManyInst& in = a.insts[task.inst];
      if (t > in.F) continue;
      if (task.kind == 0) {
        // the host deals at most kMaxTileSlots tiles, first, to a workgroup
        ok = j - t0 < kMaxTileSlots && tile_step(a, in, task.c0, task.c1, t, j - t0, L);
      } else if (t < in.F && wave == 0) {
        ok = topk_step(a, in, t, lane);
      }
    }
    // a failed top-k task (wave 0 only) ends the whole workgroup
    if (!ok) s_ok[t & 1] = 0;
    __syncthreads();
    ok = s_ok[t & 1] != 0;
  }
  if (!ok && threadIdx.x == 0) store_tagged(a.err, 1u);
}

}  // namespace

uint32_t many_tile_columns(uint32_t S) {
  return std::min(kTileColumns, std::max(1u, kTileSynapses / S));
}

hipError_t launch_many(const ManyArgs& a, uint32_t grid, hipStream_t s) {
  ManyArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_sp_many), dim3(grid),
                                    dim3(kManyThreads), args, 0, s);
}

int many_max_blocks(int device) {
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&k_sp_many), kManyThreads, 0) != hipSuccess)
    return 0;
  return cus * per_cu;
}

}  // namespace htmsp
