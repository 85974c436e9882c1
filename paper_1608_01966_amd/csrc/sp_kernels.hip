// HIP kernels for the HTM spatial pooler step on gfx950 (wave64).
//
// Section 1.1 of Wielgosz & Pietron (arXiv 1608.01966) splits a step into
// overlap (Algorithm 1), inhibition (Algorithm 2) and learning.  Two
// executions are provided:
//   * plain: three kernels per frame (overlap, global top-k, learning), the
//     state read from and written to HBM every frame;
//   * persistent: one cooperative launch for F frames.  The synapses of
//     every column stay in registers for the whole launch; the input bits of
//     the next frames are gathered while the exchange is in flight;
//     per-frame overlaps go to all other workgroups through a tagged device
//     buffer, and the global top-k is resolved redundantly so that every
//     wave knows which of its own columns learn, with no second exchange
//     (k_sp_persistent_w: a column group per wave, one workgroup per CU).
// Permanences are handled as integers q = 256 * permanence (0..256), so
// every comparison and update is exact.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

using namespace dev;

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
// Plain overlap (Algorithm 1): one wave per column, 64 synapses per ballot;
// with `boost` (1/256 units per column) the gated overlap is multiplied by it.
__global__ __launch_bounds__(256) void k_overlap_plain(const uint32_t* __restrict__ idx,
                                                       const float* __restrict__ perm,
                                                       const uint32_t* __restrict__ frame,
                                                       int32_t* __restrict__ ov, Shape sh,
                                                       const uint32_t* __restrict__ boost) {
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
  const uint32_t gated = raw >= sh.m ? raw : 0u;
  if (lane == 0) ov[c] = (int32_t)(boost ? gated * boost[c] : gated);
}

// ---------------------------------------------------------------------------
// Plain global top-k (Algorithm 2, global form) in one workgroup of 1024.
// Overlaps lie in [0, vmax] (S, or S times the largest boost).
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
                                                            Shape sh, uint32_t vmax) {
  __shared__ uint32_t red[kTopkThreads / kWave];
  ov += (size_t)blockIdx.x * sh.C;  // one frame per workgroup
  winners += (size_t)blockIdx.x * sh.k;
  const uint32_t tid = threadIdx.x;
  auto count_ge = [&](int32_t x) {
    uint32_t n = 0;
    for (uint32_t c = tid; c < sh.C; c += blockDim.x) n += ov[c] >= x;
    return block_count(n, red);
  };
  int32_t T = 0;
  uint32_t need = 0;
  if (count_ge(1) >= sh.k) {
    int32_t lo = 1, hi = (int32_t)vmax;
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

// Frames 2p and min(2p + 1, F - 1) side by side, one 64-bit entry per input
// word: both frames read and the pair written once, coalesced.  Block
// (x, y): words 1024 x ... 1024 x + 1023 of pair y.
__global__ __launch_bounds__(256) void k_pair_frames(const uint32_t* __restrict__ frames,
                                                     uint32_t F, uint32_t W, uint32_t p0,
                                                     uint64_t* __restrict__ out) {
  const uint32_t p = p0 + blockIdx.y;
  const uint32_t* f0 = frames + (size_t)(2 * p) * W;
  const uint32_t* f1 = frames + (size_t)min(2 * p + 1, F - 1) * W;
  uint64_t* o = out + (size_t)p * W;
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j) {
    const uint32_t i = blockIdx.x * 1024 + j * 256 + threadIdx.x;
    if (i < W) o[i] = f0[i] | ((uint64_t)f1[i] << 32);
  }
}

// ---------------------------------------------------------------------------
// Persistent multi-frame step.
//
// Exchange: one 16-bit entry [tag:2 | overlap:14] per column, written as
// whole 64-bit words (four columns) with agent-scope stores into each of
// `replicas` copies and read with agent-scope 64-bit loads from the copy of
// the reader's XCD.  Exchange g of the handle uses slot g & 1 and tag
// (g + 1) & 3; the slot's previous content belongs to exchange g - 2 with tag
// (g - 1) & 3 (or is the zeroed initial state), so a stale entry is never
// taken for a fresh one, and a slot is rewritten only after every workgroup
// has finished reading it.

// Whether this lane's own column (overlap v, lane < ncols) wins: above T, or
// equal to T and among the first `need` such columns in column order.
template <int NV>
__device__ __forceinline__ bool own_wins(const uint64_t (&ev)[NV], uint32_t v, bool mine,
                                         uint32_t T, uint32_t need, uint32_t lane,
                                         uint32_t c_begin) {
  const bool gt = mine && v > T;
  const bool eq = mine && T != 0 && v == T;
  const uint64_t eqm = __ballot(eq);
  if (eqm == 0ull) return gt;
  // one count of the tied columns before c_begin; at 16 words per lane (the
  // register ceiling) the difference of two counts runs faster
  const uint32_t eqb = NV <= 8 ? count_eq_before(ev, T, lane, c_begin)
                               : count_ge_before(ev, T, lane, c_begin) -
                                     count_ge_before(ev, T + 1, lane, c_begin);
  return gt || (eq && eqb + (uint32_t)__popcll(eqm & lanemask_lt(lane)) < need);
}

// Whether column c_begin + lane is selected in the field masks fm of
// select_all.  A wave's CPW columns start at a multiple of CPW (<= 16), so
// they lie in one 256-column block (one word index u for the wave); up to
// four of them share one lane's word, which is then read as a scalar.
template <int NV, uint32_t CPW>
__device__ __forceinline__ bool own_selected(const uint64_t (&fm)[NV], uint32_t lane,
                                             uint32_t c_begin) {
  const uint32_t ub = __builtin_amdgcn_readfirstlane(c_begin >> 8);
  uint64_t w = fm[0];
#pragma unroll
  for (int u = 1; u < NV; ++u) w = (uint32_t)u == ub ? fm[u] : w;
  const uint32_t c = c_begin + lane;
  uint32_t lo, hi;
  if constexpr (CPW <= 4) {
    const uint32_t src = __builtin_amdgcn_readfirstlane((c_begin >> 2) & 63u);
    lo = __builtin_amdgcn_readlane((uint32_t)w, src);
    hi = __builtin_amdgcn_readlane((uint32_t)(w >> 32), src);
  } else {
    const int src = (int)((c >> 2) & 63u);
    lo = (uint32_t)__shfl((int)(uint32_t)w, src);
    hi = (uint32_t)__shfl((int)(uint32_t)(w >> 32), src);
  }
  const uint64_t x = ((uint64_t)hi << 32) | lo;
  return ((x >> (16 * (c & 3u))) & 1ull) != 0ull;
}

// What one frame leaves for its deferred outputs.
struct FrameResult {
  uint32_t T, need, nsel, ov;
  bool sel;
};

// Outputs of frame tt: overlaps of the own columns, the own winners at their
// rank in column order, and (group 0) the -1 padding.
template <int NV>
__device__ __forceinline__ void write_frame(const PersistArgs& a, const uint64_t (&ev)[NV],
                                            const FrameResult& r, uint32_t tt, uint32_t lane,
                                            bool mine, uint32_t c_begin, bool pad) {
  const Shape& sh = a.sh;
  if (a.ov_out && mine) a.ov_out[(size_t)tt * sh.C + c_begin + lane] = (int32_t)r.ov;
  int32_t* wrow = a.win_out + (size_t)tt * sh.k;
  if (pad)
    for (uint32_t i = r.nsel + lane; i < sh.k; i += kWave) wrow[i] = -1;
  if (__ballot(r.sel) != 0ull) {
    const uint32_t gtb = count_ge_before(ev, r.T + 1, lane, c_begin);
    const uint32_t eqb = r.T ? count_ge_before(ev, r.T, lane, c_begin) - gtb : 0u;
    const uint32_t gt_pre =
        gtb + (uint32_t)__popcll(__ballot(mine && r.ov > r.T) & lanemask_lt(lane));
    const uint32_t eq_pre =
        eqb + (uint32_t)__popcll(__ballot(mine && r.T != 0 && r.ov == r.T) & lanemask_lt(lane));
    if (r.sel) wrow[gt_pre + min(eq_pre, r.need)] = (int32_t)(c_begin + lane);
  }
}

// Persistent multi-frame step, two frames per exchange.  Learning makes
// frame t + 1 depend on which columns win frame t, but only through the
// winners' own synapses; so each wave publishes, with its frame-t overlaps,
// the frame-(t+1) overlaps its columns will have if they lose frame t and if
// they win it.  Every wave resolves frame t's winners, picks each column's
// frame-(t+1) overlap accordingly and resolves frame t + 1 as well, so one
// exchange round trip serves two frames; the results are exactly those of
// stepping the frames one by one.  The next pair's products are computed
// while the exchange is in flight.  Each workgroup holds kPersistWaves
// waves and each wave owns CPW = RW / RPC consecutive
// columns (row r of the wave holds synapses (r % RPC) * 64 + lane of its
// local column r / RPC), so the per-pair work that depends on a wave's
// columns (products, learning, outputs) is split four ways, and the wave
// that learns most in a pair, which every workgroup waits for at the next
// exchange, has at most CPW columns to redo.
//   * Each wave gathers its own input words for the next pair at the start
//     of a pair, into registers; they arrive during the exchange.
//   * Wave 0 (the poller) reads the exchange and hands it to the other waves
//     through LDS (two buffers by pair parity; `seen` counts the pairs
//     handed over), so the exchange has one reader per workgroup.
//   * The workgroup's entries are staged in LDS and, after a barrier, waves
//     1..3 publish one array each as whole 64-bit words.
//   * Only wave 0 decides to abort (kSeenAbort in `seen`), so every wave
//     leaves the loop at the same point and no barrier is left waiting.
// The pair loop is instantiated once for the poller and once for the other
// waves, so that neither copy's memory waits are widened by the other's
// accesses.
template <bool B>
struct PollRole {
  static constexpr bool value = B;
};

// Instances (RPC, NV, RW) whose wave 0 issues a pair's gathers only after
// the workgroup's publish stores (PF below).  Each instance was timed both
// ways over 1000 learning frames of the 960x540 input at one C x S that
// lands on it: faster by 2-14 % at these, slower by up to 12 % or level at
// every other one.  Whether the exchange reads wait for entries still on
// their way or come back late depends on how the publish stores and the
// gathers share the workgroup's memory pipeline, which the instance sets;
// the results are the same either way.
constexpr bool publish_first(int rpc, int nv, int rw) {
  return (rpc == 2 && nv == 4 && rw == 4) || (rpc == 4 && nv == 4 && rw == 8) ||
         (rpc == 1 && nv == 8 && rw == 4) || (rpc == 2 && nv == 8 && rw == 8) ||
         (rpc == 8 && nv == 2 && rw == 8) || (rpc == 16 && nv == 4 && rw == 16) ||
         (rpc == 1 && nv == 16 && rw == 8) || (rpc == 2 && nv == 16 && rw == 16) ||
         (rpc == 4 && nv == 16 && rw == 16);
}

template <int RPC, int NV, int RW, bool PF = publish_first(RPC, NV, RW)>
__global__ __launch_bounds__(kPersistWaves * kWave) void k_sp_persistent_w(PersistArgs a) {
  constexpr uint32_t CPW = RW / RPC;
  constexpr uint32_t CPAD = NV * 4 * kWave;        // entries per exchange array
  constexpr uint32_t NARR = 3;                     // frame t, frame t+1 if lost, if won
  constexpr uint32_t WGC = kPersistWaves * CPW;    // columns per workgroup
  constexpr uint32_t kSeenAbort = 0xFFFFFFFFu;
  static_assert(kPersistWaves == NARR + 1, "waves 1..3 publish the three arrays");
  __shared__ uint64_t xl[2][NARR][NV][kWave];
  __shared__ uint32_t pub[NARR][WGC];
  __shared__ uint32_t seen;
  __shared__ uint32_t pubd[NARR];  // pairs each publishing wave has issued
  const Shape sh = a.sh;
  const uint32_t lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const uint32_t gw = blockIdx.x * kPersistWaves + wave;
  const uint32_t c_begin = gw * CPW;
  const uint32_t wg_begin = blockIdx.x * WGC;
  const uint32_t ncols = c_begin < sh.C ? min(CPW, sh.C - c_begin) : 0u;
  if (threadIdx.x < NARR) pubd[threadIdx.x] = 0;
  if (threadIdx.x == 0) seen = 0;

  // State: idx << 9 | q, and the mask of the input bit while connected;
  // wi: the frame word each row reads (word 0 for rows without a synapse).
  uint32_t st[RW], msk[RW], wi[RW];
  uint32_t row_ok = 0;
#pragma unroll
  for (uint32_t r = 0; r < RW; ++r) {
    const uint32_t j = r / RPC, s = (r % RPC) * kWave + lane;
    const bool ok = j < ncols && s < sh.S;
    const size_t off = ok ? (size_t)(c_begin + j) * sh.S + s : 0;
    const uint32_t i = min(a.idx[off], sh.N - 1);
    const uint32_t q = perm_to_q(a.perm[off]);
    st[r] = ok ? (i << 9) | q : 0u;
    msk[r] = (ok && q >= sh.theta) ? (1u << (i & 31u)) : 0u;
    wi[r] = ok ? i >> 5 : 0u;
    row_ok |= ok ? 1u << r : 0u;
  }

  uint64_t* x64w = reinterpret_cast<uint64_t*>(a.xchg);
  const uint32_t rep = xcc_id() % a.replicas;
  const bool mine = lane < ncols;
  uint64_t ev0[NV], ev1[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    ev0[u] = 0;
    ev1[u] = 0;
  }
  uint32_t guess = 1 + sh.S / 16;
  FrameResult r0 = {0, 0, 0, 0, false}, r1 = {0, 0, 0, 0, false};
  bool abort = false;
  uint32_t prev_t = 0;
  bool prev_two = false;

  // This wave's entries of the three arrays, into the workgroup's staging.
  auto stage = [&](const uint32_t(&o0)[CPW], const uint32_t(&oL)[CPW], const uint32_t(&oW)[CPW]) {
    if (lane < CPW) {
      pub[0][wave * CPW + lane] = lane_value(o0, lane);
      pub[1][wave * CPW + lane] = lane_value(oL, lane);
      pub[2][wave * CPW + lane] = lane_value(oW, lane);
    }
  };

  // Input words of frames t and t + 1 (t even), one 64-bit load per row
  // from their pair, clamped to the last pair (a gather past the end is never
  // used; issuing it unconditionally keeps the loads free of copies that
  // would wait for them).  Random gathers cost the workgroup's L1 one tag
  // lookup per distinct line per load; pairing halves the loads.
  auto gather = [&](uint32_t t, uint32_t (&x0)[RW], uint32_t (&x1)[RW]) {
    const uint64_t* fp = a.fpair + (size_t)min(t / 2, (a.F - 1) / 2) * sh.W;
#pragma unroll
    for (uint32_t r = 0; r < RW; ++r) {
      const uint64_t v = fp[wi[r]];
      x0[r] = (uint32_t)v;
      x1[r] = (uint32_t)(v >> 32);
    }
  };

  // What a pair publishes, for the columns in `cols`: frame t's overlap, the
  // state after learning frame t, and frame t + 1's overlap if the column
  // loses frame t (same state) and if it wins it.
  auto products = [&](uint32_t cols, const uint32_t (&x0)[RW], const uint32_t (&x1)[RW],
                      uint32_t (&o0)[CPW], uint32_t (&oL)[CPW], uint32_t (&oW)[CPW],
                      uint32_t (&sW)[RW], uint32_t (&mW)[RW]) {
#pragma unroll
    for (uint32_t j = 0; j < CPW; ++j) {
      if ((cols >> j) & 1u) {
        uint32_t c0 = 0, cL = 0, cW = 0;
#pragma unroll
        for (uint32_t rr = 0; rr < RPC; ++rr) {
          const uint32_t r = j * RPC + rr;
          const uint32_t i = st[r] >> 9;
          const uint32_t q = learn_q(st[r] & 511u, input_bit(x0[r], i), sh);
          const bool ok = a.learn && ((row_ok >> r) & 1u);
          sW[r] = ok ? (i << 9) | q : st[r];
          mW[r] = ok ? (q >= sh.theta ? 1u << (i & 31u) : 0u) : msk[r];
          c0 += (uint32_t)__popcll(__ballot((x0[r] & msk[r]) != 0u));
          cL += (uint32_t)__popcll(__ballot((x1[r] & msk[r]) != 0u));
          cW += (uint32_t)__popcll(__ballot((x1[r] & mW[r]) != 0u));
        }
        const bool live = j < ncols;
        o0[j] = (live && c0 >= sh.m) ? c0 : 0u;
        oL[j] = (live && cL >= sh.m) ? cL : 0u;
        oW[j] = (live && cW >= sh.m) ? cW : 0u;
      }
    }
  };

  constexpr uint32_t kAllCols = (1u << CPW) - 1u;
  auto run = [&](auto role) {
    constexpr bool POLL = decltype(role)::value;
    uint32_t w0[RW], w1[RW];  // this pair's input words
    uint32_t ov0[CPW], ovL[CPW], ovW[CPW];
    uint32_t stW[RW], mskW[RW];
    gather(0, w0, w1);
    products(kAllCols, w0, w1, ov0, ovL, ovW, stW, mskW);
    stage(ov0, ovL, ovW);
    __syncthreads();
    for (uint32_t t = 0; t < a.F; t += 2) {
      const bool two = t + 1 < a.F;
      const uint32_t pair = t / 2;
      const uint32_t g = a.frame_base + pair;
      const uint32_t slot = g & 1u;
      const uint32_t tg = ((g + 1u) & 3u) << kTagShift;
      const uint64_t* xs = x64w + (size_t)(rep * 2 + slot) * NARR * (CPAD / 4);

      // Wave 1 + q publishes array q of the workgroup as whole 64-bit words
      // (entries past C land in the padding that readers skip).
      if constexpr (!POLL) {
        const uint32_t arr = wave - 1;
        if (lane < WGC / 4) {
          const uint64_t word = (uint64_t)(tg | pub[arr][4 * lane]) |
                                ((uint64_t)(tg | pub[arr][4 * lane + 1]) << 16) |
                                ((uint64_t)(tg | pub[arr][4 * lane + 2]) << 32) |
                                ((uint64_t)(tg | pub[arr][4 * lane + 3]) << 48);
          for (uint32_t rr = 0; rr < a.replicas; ++rr)
            store_word(x64w + (((size_t)(rr * 2 + slot) * NARR + arr) * CPAD + wg_begin) / 4 + lane,
                       word);
        }
        if constexpr (PF) lds_release(&pubd[arr], pair + 1);
      } else if constexpr (PF) {
        // Wave 0 issues its gathers only after the workgroup's publish
        // stores, which then reach the other workgroups sooner; its first
        // read of the exchange moves later with them.  Waves 1..3 publish
        // at the top of every pair they enter, so this wait always ends.
        while (lds_acquire(&pubd[0]) <= pair || lds_acquire(&pubd[1]) <= pair ||
               lds_acquire(&pubd[2]) <= pair)
          __builtin_amdgcn_s_sleep(0);
      }
      // The next pair's input words, which arrive while the exchange is in flight.
      const uint32_t tn = t + 2;
      const bool has_next = tn < a.F;
      uint32_t n0[RW], n1[RW];
      gather(tn, n0, n1);
      uint64_t v0[NV], vL[NV], vW[NV];
      if (t > 0) {
        write_frame(a, ev0, r0, prev_t, lane, mine, c_begin, gw == 0);
        if (prev_two) write_frame(a, ev1, r1, prev_t + 1, lane, mine, c_begin, gw == 0);
      }

      // The next pair's products with the current state, while the exchange
      // is in flight; redone below for the columns that learn in this pair.
      uint32_t sov0[CPW], sovL[CPW], sovW[CPW];
      uint32_t sstW[RW], smskW[RW];
      if (has_next) products(kAllCols, n0, n1, sov0, sovL, sovW, sstW, smskW);

      if constexpr (POLL) {
        // First read of the exchange after the outputs and the speculation
        // (a read that comes back stale costs a whole further round trip).
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          v0[u] = load_entries(xs + u * kWave + lane);
          vL[u] = load_entries(xs + CPAD / 4 + u * kWave + lane);
          vW[u] = load_entries(xs + 2 * (CPAD / 4) + u * kWave + lane);
        }
        // (a.stall != 0 only in tests of the failure path)
        const uint64_t tagw = (uint64_t)((((g + 1u + a.stall) & 3u) << kTagShift)) * kOnes16;
        uint32_t spins = 0;
        while (true) {
          bool ok = true;
#pragma unroll
          for (int u = 0; u < NV; ++u) {
            const uint64_t tm = tag_mask(u, lane, sh.C);
            ok = ok && ((v0[u] ^ tagw) & tm) == 0ull && ((vL[u] ^ tagw) & tm) == 0ull &&
                 ((vW[u] ^ tagw) & tm) == 0ull;
          }
          if (__all(ok)) break;
          if (++spins > a.spin_limit || ((spins & 63u) == 0 && load_tagged(a.err) != 0)) {
            abort = true;
            break;
          }
#pragma unroll
          for (int u = 0; u < NV; ++u) {
            const uint64_t tm = tag_mask(u, lane, sh.C);
            if (((v0[u] ^ tagw) & tm) != 0ull) v0[u] = load_entries(xs + u * kWave + lane);
            if (((vL[u] ^ tagw) & tm) != 0ull) vL[u] = load_entries(xs + CPAD / 4 + u * kWave + lane);
            if (((vW[u] ^ tagw) & tm) != 0ull)
              vW[u] = load_entries(xs + 2 * (CPAD / 4) + u * kWave + lane);
          }
        }
        if (abort) {
          lds_release(&seen, kSeenAbort);
          break;
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          xl[pair & 1][0][u][lane] = v0[u];
          xl[pair & 1][1][u][lane] = vL[u];
          xl[pair & 1][2][u][lane] = vW[u];
        }
        lds_release(&seen, pair + 1);
      } else {
        // Bounded by wave 0, which sets `seen` within its own spin limit.
        uint32_t sv;
        while ((sv = lds_acquire(&seen)) <= pair) __builtin_amdgcn_s_sleep(0);
        if (sv == kSeenAbort) {
          abort = true;
          break;
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          v0[u] = xl[pair & 1][0][u][lane];
          vL[u] = xl[pair & 1][1][u][lane];
          vW[u] = xl[pair & 1][2][u][lane];
        }
      }

      // Frame t: threshold, and which own columns win.
      const uint32_t my0 = lane_value(ov0, lane);
#pragma unroll
      for (int u = 0; u < NV; ++u) ev0[u] = v0[u] & kFieldBits;
      uint32_t c_hi;
      const uint32_t T0 = topk_threshold(ev0, sh.S, sh.k, guess, &c_hi);
      r0.T = T0;
      r0.need = T0 ? sh.k - c_hi : 0u;
      r0.nsel = T0 ? sh.k : c_hi;
      r0.ov = my0;
      if (T0) guess = T0;

      // Frame t + 1: every column's overlap given frame t's winners (whose
      // field masks also give the own columns' frame-t result).
      if (!two) r0.sel = own_wins(ev0, my0, mine, T0, r0.need, lane, c_begin);
      if (two) {
        uint64_t fm[NV];
        select_all(ev0, T0, r0.need, lane, fm);
        // (read in every lane: the word it reads lives in another lane)
        const bool own0 = own_selected<NV, CPW>(fm, lane, c_begin);
        r0.sel = mine && own0;
#pragma unroll
        for (int u = 0; u < NV; ++u)
          ev1[u] = ((vL[u] & ~fm[u]) | (vW[u] & fm[u])) & kFieldBits;
        const uint32_t my1 = r0.sel ? lane_value(ovW, lane) : lane_value(ovL, lane);
        const uint32_t T1 = topk_threshold(ev1, sh.S, sh.k, guess, &c_hi);
        r1.T = T1;
        r1.need = T1 ? sh.k - c_hi : 0u;
        r1.nsel = T1 ? sh.k : c_hi;
        r1.ov = my1;
        r1.sel = own_wins(ev1, my1, mine, T1, r1.need, lane, c_begin);
        if (T1) guess = T1;
      }

      // Learning on the own columns that won (frame t's state, then frame t+1).
      uint32_t changed = 0;
      if (a.learn) {
        const uint32_t sel0 = (uint32_t)__ballot(r0.sel) & kAllCols;
        const uint32_t sel1 = two ? (uint32_t)__ballot(r1.sel) & kAllCols : 0u;
        changed = sel0 | sel1;
#pragma unroll
        for (uint32_t j = 0; j < CPW; ++j) {
          if ((changed >> j) & 1u) {
#pragma unroll
            for (uint32_t rr = 0; rr < RPC; ++rr) {
              const uint32_t r = j * RPC + rr;
              if ((sel0 >> j) & 1u) {
                st[r] = stW[r];
                msk[r] = mskW[r];
              }
              if ((sel1 >> j) & 1u) {
                const uint32_t i = st[r] >> 9;
                const uint32_t q = learn_q(st[r] & 511u, input_bit(w1[r], i), sh);
                const bool ok = (row_ok >> r) & 1u;
                st[r] = ok ? (i << 9) | q : st[r];
                msk[r] = ok ? (q >= sh.theta ? 1u << (i & 31u) : 0u) : msk[r];
              }
            }
          }
        }
      }
      prev_t = t;
      prev_two = two;

      if (has_next) {
        if (changed) products(changed, n0, n1, sov0, sovL, sovW, sstW, smskW);
#pragma unroll
        for (uint32_t r = 0; r < RW; ++r) {
          w0[r] = n0[r];
          w1[r] = n1[r];
          stW[r] = sstW[r];
          mskW[r] = smskW[r];
        }
#pragma unroll
        for (uint32_t j = 0; j < CPW; ++j) {
          ov0[j] = sov0[j];
          ovL[j] = sovL[j];
          ovW[j] = sovW[j];
        }
        stage(ov0, ovL, ovW);
      }
      __syncthreads();
    }
  };
  if (a.F > 0) {
    if (wave == 0)
      run(PollRole<true>{});
    else
      run(PollRole<false>{});
  }

  if (abort) {
    if (wave == 0 && lane == 0) store_tagged(a.err, 1u);
    return;
  }
  if (a.F > 0) {
    write_frame(a, ev0, r0, prev_t, lane, mine, c_begin, gw == 0);
    if (prev_two) write_frame(a, ev1, r1, prev_t + 1, lane, mine, c_begin, gw == 0);
  }
  if (a.learn) {
#pragma unroll
    for (uint32_t r = 0; r < RW; ++r) {
      const uint32_t j = r / RPC, s = (r % RPC) * kWave + lane;
      if ((row_ok >> r) & 1u) a.perm[(size_t)(c_begin + j) * sh.S + s] = q_to_perm(st[r] & 511u);
    }
  }
}

}  // namespace

uint32_t persistent_exchange_arrays() { return 3; }

uint32_t persistent_exchange_entries(uint32_t C) {
  uint32_t nv = 1;
  while (nv * 4 * kWave < C) nv <<= 1;
  return nv * 4 * kWave;
}

const void* persistent_wave_kernel(uint32_t rpc, uint32_t nv, uint32_t rw) {
#define HTMSP_PW(P, V, R)                              \
  if (rpc == P && nv == V && rw == R)                  \
    return reinterpret_cast<const void*>(&k_sp_persistent_w<P, V, R>);
  // The shapes persistent_wave_rows gives on a 256-CU device.
  HTMSP_PW(1, 1, 4) HTMSP_PW(1, 2, 4) HTMSP_PW(1, 4, 4) HTMSP_PW(1, 8, 4) HTMSP_PW(1, 16, 8)
  HTMSP_PW(2, 1, 4) HTMSP_PW(2, 2, 4) HTMSP_PW(2, 4, 4) HTMSP_PW(2, 8, 8) HTMSP_PW(2, 16, 16)
  HTMSP_PW(4, 1, 4) HTMSP_PW(4, 2, 4) HTMSP_PW(4, 4, 8) HTMSP_PW(4, 8, 16) HTMSP_PW(4, 16, 16)
  HTMSP_PW(8, 1, 8) HTMSP_PW(8, 2, 8) HTMSP_PW(8, 4, 16) HTMSP_PW(8, 8, 16) HTMSP_PW(16, 1, 16)
  HTMSP_PW(16, 2, 16) HTMSP_PW(16, 4, 16)
#undef HTMSP_PW
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
                                int32_t* ov, const Shape& sh, hipStream_t s,
                                const uint32_t* boost) {
  const uint32_t waves_per_block = 4;
  const uint32_t blocks = (sh.C + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(k_overlap_plain, dim3(blocks), dim3(waves_per_block * kWave), 0, s, idx,
                     perm, frame, ov, sh, boost);
  return hipGetLastError();
}

hipError_t launch_topk_plain(const int32_t* ov, int32_t* winners, const Shape& sh,
                             hipStream_t s, uint32_t frames, uint32_t vmax) {
  hipLaunchKernelGGL(k_topk_plain, dim3(frames), dim3(kTopkThreads), 0, s, ov, winners, sh,
                     vmax ? vmax : sh.S);
  return hipGetLastError();
}

hipError_t launch_learn_plain(const uint32_t* idx, float* perm, const uint32_t* frame,
                              const int32_t* winners, const Shape& sh, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_plain, dim3(sh.k), dim3(256), 0, s, idx, perm, frame, winners, sh);
  return hipGetLastError();
}

hipError_t launch_pair_frames(const uint32_t* frames, uint32_t F, uint32_t W, uint64_t* out,
                              hipStream_t s) {
  const uint32_t P = (F + 1) / 2, bx = (W + 1023) / 1024;
  constexpr uint32_t kMaxY = 65535;
  for (uint32_t p0 = 0; p0 < P; p0 += kMaxY) {
    hipLaunchKernelGGL(k_pair_frames, dim3(bx, std::min(kMaxY, P - p0)), dim3(256), 0, s, frames,
                       F, W, p0, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace htmsp
