// Local inhibition: Algorithm 2 as printed, each column competing within a
// neighbourhood given by an inhibition radius (the form Section 3.2.2
// describes), and the learning step built on it.
//
// Columns sit on a row-major grid of grid_w columns per row.  The
// neighbourhood of c is every other column within `radius` in both grid
// coordinates (no wrap-around); with v the n-th largest neighbour overlap
// (0 when there are fewer than n neighbours), c is active iff its overlap is
// greater than max(v, 1).  Equivalently -- and that is what the kernel
// counts -- c is active iff its overlap is at least 2 and fewer than n
// neighbours have an overlap at least as large; a thread stops counting as
// soon as n are found, so most columns (low overlaps) finish early.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

using namespace dev;

constexpr uint32_t kLocalThreads = 256;
constexpr uint32_t kLocalLdsColumns = 16384;  // a frame's overlaps fit LDS up to this C

// Block (frame f, columns [b * 256, b * 256 + 256)).  LDS: the whole frame's
// overlaps when they fit, else reads from device memory.
// `radius_dev`, when set, holds the radius instead of `radius` (the
// adaptive step keeps it in device memory), and block 0 then records it in
// `radius_out`, when set.
template <bool LDS>
__global__ __launch_bounds__(kLocalThreads) void k_inhibit_local(
    const int32_t* __restrict__ ov, uint32_t C, uint32_t grid_w, uint32_t radius, uint32_t n,
    uint32_t col_blocks, uint8_t* __restrict__ active, const uint32_t* __restrict__ radius_dev,
    uint32_t* __restrict__ radius_out) {
  __shared__ int32_t s_ov[LDS ? kLocalLdsColumns : 1];
  if (radius_dev) {
    radius = *radius_dev;
    if (radius_out && blockIdx.x == 0 && threadIdx.x == 0) *radius_out = radius;
  }
  const uint32_t f = blockIdx.x / col_blocks;
  const uint32_t c = (blockIdx.x % col_blocks) * kLocalThreads + threadIdx.x;
  const int32_t* o = ov + (size_t)f * C;
  if constexpr (LDS) {
    for (uint32_t i = threadIdx.x; i < C; i += kLocalThreads) s_ov[i] = o[i];
    __syncthreads();
  }
  if (c >= C) return;
  const int32_t* src = LDS ? s_ov : o;
  const int32_t v = src[c];
  uint8_t on = 0;
  if (v >= 2) {
    const uint32_t rows = (C + grid_w - 1) / grid_w;
    const uint32_t cx = c % grid_w, cy = c / grid_w;
    const uint32_t y0 = cy >= radius ? cy - radius : 0u;
    const uint32_t y1 = min(cy + radius, rows - 1);
    const uint32_t x0 = cx >= radius ? cx - radius : 0u;
    const uint32_t x1 = min(cx + radius, grid_w - 1);
    uint32_t k = 0;
    for (uint32_t y = y0; y <= y1 && k < n; ++y) {
      const uint32_t base = y * grid_w;
      for (uint32_t x = x0; x <= x1; ++x) {
        const uint32_t d = base + x;
        if (d >= C) break;  // the last grid row may be partly empty
        k += (d != c && src[d] >= v) ? 1u : 0u;
      }
    }
    on = k < n ? 1 : 0;
  }
  active[(size_t)f * C + c] = on;
}

// Learning on the active columns of one frame: one wave per column, idle
// for inactive ones.
__global__ __launch_bounds__(256) void k_learn_active(const uint32_t* __restrict__ idx,
                                                      float* __restrict__ perm,
                                                      const uint32_t* __restrict__ frame,
                                                      const uint8_t* __restrict__ active,
                                                      Shape sh) {
  const uint32_t c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  if (c >= sh.C || !active[c]) return;
  const uint32_t* ci = idx + (size_t)c * sh.S;
  float* cp = perm + (size_t)c * sh.S;
  for (uint32_t s = lane; s < sh.S; s += kWave) {
    const uint32_t i = min(ci[s], sh.N - 1);
    cp[s] = q_to_perm(learn_q(perm_to_q(cp[s]), input_bit(frame[i >> 5], i), sh));
  }
}

// Inhibition radius adaptation (after a learning frame, the average
// connected receptive field of the columns carried to the column grid; the
// rule is stated with sp_step_local_adaptive in include/sp.h).  One wave per
// column: the extent of its connected inputs on the input image, then one
// add of span_x + span_y and one count per column into acc = {A, n}.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, (uint32_t)__shfl_xor(v, off));
  return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor(v, off));
  return v;
}

__global__ __launch_bounds__(256) void k_radius_span(const uint32_t* __restrict__ idx,
                                                     const float* __restrict__ perm, Shape sh,
                                                     uint32_t in_w,
                                                     unsigned long long* __restrict__ acc) {
  const uint32_t c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  if (c >= sh.C) return;  // whole wave
  uint32_t x0 = 0xFFFFFFFFu, y0 = 0xFFFFFFFFu, x1 = 0, y1 = 0;
  for (uint32_t s = lane; s < sh.S; s += kWave) {
    const size_t off = (size_t)c * sh.S + s;
    if (perm_to_q(perm[off]) < sh.theta) continue;
    const uint32_t p = min(idx[off], sh.N - 1);
    const uint32_t y = p / in_w, x = p - y * in_w;
    x0 = min(x0, x);
    x1 = max(x1, x);
    y0 = min(y0, y);
    y1 = max(y1, y);
  }
  x0 = wave_min(x0);
  y0 = wave_min(y0);
  x1 = wave_max(x1);
  y1 = wave_max(y1);
  if (lane == 0 && x0 != 0xFFFFFFFFu) {
    atomicAdd(&acc[0], (unsigned long long)(x1 - x0 + 1) + (y1 - y0 + 1));
    atomicAdd(&acc[1], 1ull);
  }
}

// One thread: the new radius from acc (unchanged when no column has a
// connected synapse), floor(A B / D) with the 128-bit product divided by
// shifts and subtractions; then acc is cleared for the next frame.
__global__ void k_radius_update(unsigned long long* __restrict__ acc, uint32_t* __restrict__ radius,
                                uint64_t B, uint64_t in_area8, uint32_t reset_only) {
  const unsigned long long A = acc[0], n = acc[1];
  acc[0] = 0;
  acc[1] = 0;
  if (reset_only || n == 0) return;
  const unsigned __int128 num = (unsigned __int128)A * B;
  const unsigned __int128 den = (unsigned __int128)in_area8 * n;
  unsigned __int128 rem = 0;
  uint64_t q = 0;
  for (int bit = 127; bit >= 0; --bit) {
    rem = (rem << 1) | (unsigned __int128)((num >> bit) & 1u);
    if (rem >= den) {
      rem -= den;
      if (bit < 64) q |= 1ull << bit;
      else q = 0xFFFFFFFFFFFFFFFFull;  // cannot happen for valid shapes; saturate
    }
  }
  *radius = q < 1 ? 1u : (q > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)q);
}

// Persistent learning step with local inhibition: F frames in one
// cooperative launch.  Columns are split as in the global persistent kernel
// (kPersistWaves waves per workgroup, a group of CPW = RW / RPC consecutive
// columns per wave, synapse state in registers for the whole launch).  Per
// frame every wave publishes its columns' overlaps through a tagged exchange
// (one 16-bit entry [tag:2 | overlap:14] per column; frame g of the handle's
// local sequence uses slot g & 1 and tag (g + 1) & 3), wave 0 of each
// workgroup reads every column's entry into LDS, and each wave then decides
// its own columns by scanning their neighbourhoods in LDS, learns on the
// active ones and computes its next overlaps (speculatively before the
// exchange wait, redone for the columns that learned).  Only wave 0 decides
// to abort, through the LDS pair counter, so no barrier is left waiting.
template <bool B>
struct LocalRole {
  static constexpr bool value = B;
};

template <int RPC, int NV, int RW>
__global__ __launch_bounds__(kPersistWaves * kWave) void k_sp_persistent_local(LocalArgs a) {
  constexpr uint32_t CPW = RW / RPC;
  constexpr uint32_t WGC = kPersistWaves * CPW;  // columns per workgroup
  constexpr uint32_t kSeenAbort = 0xFFFFFFFFu;
  // Every column's overlap of one frame (two buffers by frame parity): the
  // exchange words hold columns u * 256 + 4 * lane + q, so word u * 64 + lane
  // of the copy is columns 4 * (u * 64 + lane) + q and the copy indexes by
  // column as 16-bit entries.
  __shared__ uint64_t xl[2][NV * kWave];
  __shared__ uint32_t pub[WGC];
  __shared__ uint32_t seen;
  const Shape sh = a.sh;
  const uint32_t lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const uint32_t gw = blockIdx.x * kPersistWaves + wave;
  const uint32_t c_begin = gw * CPW;
  const uint32_t wg_begin = blockIdx.x * WGC;
  const uint32_t ncols = c_begin < sh.C ? min(CPW, sh.C - c_begin) : 0u;
  const uint32_t rows = (sh.C + a.grid_w - 1) / a.grid_w;
  if (threadIdx.x == 0) seen = 0;

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
  const uint32_t rep = xcc_id() % a.replicas;
  bool abort = false;

  // Input words of frame t (clamped to the last frame: unconditional loads).
  auto gather = [&](uint32_t t, uint32_t (&x)[RW]) {
    const uint32_t* f = a.frames + (size_t)min(t, a.F - 1) * sh.W;
#pragma unroll
    for (uint32_t r = 0; r < RW; ++r) x[r] = f[wi[r]];
  };
  // Gated overlaps (Algorithm 1) of the columns in `cols` with the current state.
  auto overlaps = [&](uint32_t cols, const uint32_t (&x)[RW], uint32_t (&o)[CPW]) {
#pragma unroll
    for (uint32_t j = 0; j < CPW; ++j) {
      if ((cols >> j) & 1u) {
        uint32_t c = 0;
#pragma unroll
        for (uint32_t rr = 0; rr < RPC; ++rr) {
          const uint32_t r = j * RPC + rr;
          c += (uint32_t)__popcll(__ballot((x[r] & msk[r]) != 0u));
        }
        o[j] = (j < ncols && c >= sh.m) ? c : 0u;
      }
    }
  };
  // Algorithm 2 for column c with overlap v against the frame's copy: active
  // iff v >= 2 and fewer than n other columns of its neighbourhood have an
  // overlap >= v (lanes split each row of the window; stops at n).
  auto decide = [&](uint32_t c, uint32_t v, const uint16_t* ov) {
    if (v < 2) return false;
    const uint32_t cx = c % a.grid_w, cy = c / a.grid_w;
    const uint32_t y0 = cy >= a.radius ? cy - a.radius : 0u;
    const uint32_t y1 = min(cy + a.radius, rows - 1);
    const uint32_t x0 = cx >= a.radius ? cx - a.radius : 0u;
    const uint32_t x1 = min(cx + a.radius, a.grid_w - 1);
    uint32_t k = 0;
    for (uint32_t y = y0; y <= y1 && k < sh.k; ++y) {
      for (uint32_t xb = x0; xb <= x1 && k < sh.k; xb += kWave) {
        const uint32_t x = xb + lane, d = y * a.grid_w + x;
        const bool hit = x <= x1 && d < sh.C && d != c && (ov[d] & 0x3FFFu) >= v;
        k += (uint32_t)__popcll(__ballot(hit));
      }
    }
    return k < sh.k;
  };

  auto run = [&](auto role) {
    constexpr bool POLL = decltype(role)::value;
    uint32_t w[RW], o[CPW];
    gather(0, w);
    overlaps((1u << CPW) - 1u, w, o);
    if (lane < CPW) pub[wave * CPW + lane] = lane_value(o, lane);
    __syncthreads();
    for (uint32_t t = 0; t < a.F; ++t) {
      const uint32_t g = a.frame_base + t;
      const uint32_t slot = g & 1u;
      const uint32_t tg = ((g + 1u) & 3u) << kTagShift;
      uint64_t* xs = a.xchg + (size_t)(rep * 2 + slot) * NV * kWave;
      // Wave 1 publishes the workgroup's entries as whole 64-bit words.
      if (!POLL && wave == 1 && lane < WGC / 4) {
        const uint64_t word = (uint64_t)(tg | pub[4 * lane]) |
                              ((uint64_t)(tg | pub[4 * lane + 1]) << 16) |
                              ((uint64_t)(tg | pub[4 * lane + 2]) << 32) |
                              ((uint64_t)(tg | pub[4 * lane + 3]) << 48);
        for (uint32_t rr = 0; rr < a.replicas; ++rr)
          store_word(a.xchg + (size_t)(rr * 2 + slot) * NV * kWave + wg_begin / 4 + lane, word);
      }
      uint32_t nx[RW], on[CPW];
      gather(t + 1, nx);
      overlaps((1u << CPW) - 1u, nx, on);  // speculation: no own column learns

      if constexpr (POLL) {
        uint64_t v[NV];
#pragma unroll
        for (int u = 0; u < NV; ++u) v[u] = load_entries(xs + u * kWave + lane);
        // (a.stall != 0 only in tests of the failure path)
        const uint64_t tagw = (uint64_t)((((g + 1u + a.stall) & 3u) << kTagShift)) * kOnes16;
        uint32_t spins = 0;
        while (true) {
          bool ok = true;
#pragma unroll
          for (int u = 0; u < NV; ++u) ok = ok && ((v[u] ^ tagw) & tag_mask(u, lane, sh.C)) == 0ull;
          if (__all(ok)) break;
          if (++spins > a.spin_limit || ((spins & 63u) == 0 && load_tagged(a.err) != 0)) {
            abort = true;
            break;
          }
#pragma unroll
          for (int u = 0; u < NV; ++u)
            if (((v[u] ^ tagw) & tag_mask(u, lane, sh.C)) != 0ull)
              v[u] = load_entries(xs + u * kWave + lane);
        }
        if (abort) {
          lds_release(&seen, kSeenAbort);
          break;
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) xl[t & 1][u * kWave + lane] = v[u];
        lds_release(&seen, t + 1);
      } else {
        // Bounded by wave 0, which sets `seen` within its own spin limit.
        uint32_t sv;
        while ((sv = lds_acquire(&seen)) <= t) __builtin_amdgcn_s_sleep(0);
        if (sv == kSeenAbort) {
          abort = true;
          break;
        }
      }

      // Own columns: decision, outputs, learning on the active ones.
      const uint16_t* ov16 = reinterpret_cast<const uint16_t*>(xl[t & 1]);
      uint32_t act = 0;
#pragma unroll
      for (uint32_t j = 0; j < CPW; ++j)
        if (j < ncols && decide(c_begin + j, o[j], ov16)) act |= 1u << j;
      if (lane < ncols) {
        a.active_out[(size_t)t * sh.C + c_begin + lane] = (uint8_t)((act >> lane) & 1u);
        if (a.ov_out) a.ov_out[(size_t)t * sh.C + c_begin + lane] = (int32_t)lane_value(o, lane);
      }
      if (a.learn && act) {
#pragma unroll
        for (uint32_t r = 0; r < RW; ++r) {
          if ((act >> (r / RPC)) & (row_ok >> r) & 1u) {
            const uint32_t i = st[r] >> 9;
            const uint32_t q = learn_q(st[r] & 511u, input_bit(w[r], i), sh);
            st[r] = (i << 9) | q;
            msk[r] = q >= sh.theta ? 1u << (i & 31u) : 0u;
          }
        }
        overlaps(act, nx, on);
      }
#pragma unroll
      for (uint32_t r = 0; r < RW; ++r) w[r] = nx[r];
#pragma unroll
      for (uint32_t j = 0; j < CPW; ++j) o[j] = on[j];
      if (lane < CPW) pub[wave * CPW + lane] = lane_value(o, lane);
      __syncthreads();
    }
  };
  if (a.F > 0) {
    if (wave == 0)
      run(LocalRole<true>{});
    else
      run(LocalRole<false>{});
  }
  if (abort) {
    if (wave == 0 && lane == 0) store_tagged(a.err, 1u);
    return;
  }
  if (a.learn) {
#pragma unroll
    for (uint32_t r = 0; r < RW; ++r) {
      const uint32_t j = r / RPC, s = (r % RPC) * kWave + lane;
      if ((row_ok >> r) & 1u) a.perm[(size_t)(c_begin + j) * sh.S + s] = q_to_perm(st[r] & 511u);
    }
  }
}

// Algorithm 2 for column d = (dx, dy) with overlap v in one thread, against
// one frame's copy of every column's overlap (word i holds columns 4i..4i+3
// as 16-bit fields, tag bits cleared): active iff v >= 2 and fewer than n
// other columns of its neighbourhood have an overlap >= v.  Counts four
// columns a word with the field compare of the top-k: the end words of each
// window row under a mask, the words between in runs of eight loads (the
// last run's loads past the row read zero words, which count nothing); d
// itself (overlap v) is counted once, so the count stops at n + 1.
__device__ __forceinline__ bool local_active(uint32_t dx, uint32_t dy, uint32_t v,
                                             const uint64_t* w64, uint32_t C, uint32_t grid_w,
                                             uint32_t rows, uint32_t radius, uint32_t n) {
  if (v < 2) return false;
  const uint32_t y0 = dy >= radius ? dy - radius : 0u, y1 = min(dy + radius, rows - 1);
  const uint32_t x0 = dx >= radius ? dx - radius : 0u, x1 = min(dx + radius, grid_w - 1);
  const uint32_t add = 0x8000u - v, lim = n + 1;
  auto cnt = [&](uint64_t w) { return (uint32_t)__popcll(field_add(w, add) & kHighBits); };
  uint32_t k = 0;
  for (uint32_t y = y0; y <= y1; ++y) {
    const uint32_t lo = y * grid_w + x0;
    if (lo >= C) break;  // the ragged last row ends before this segment
    const uint32_t hi = min(y * grid_w + x1, C - 1);
    const uint32_t i0 = lo >> 2, i1 = hi >> 2;
    const uint64_t m0 = kHighBits & (~0ull << (16 * (lo & 3u)));
    const uint64_t m1 = kHighBits & (~0ull >> (16 * (3u - (hi & 3u))));
    if (i0 == i1) {
      k += (uint32_t)__popcll(field_add(w64[i0], add) & m0 & m1);
    } else {
      k += (uint32_t)__popcll(field_add(w64[i0], add) & m0) +
           (uint32_t)__popcll(field_add(w64[i1], add) & m1);
      uint32_t i = i0 + 1;
      for (; i + 8 <= i1 && k < lim; i += 8) {
        uint64_t wv[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) wv[u] = w64[i + u];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) k += cnt(wv[u]);
      }
      if (i < i1 && k < lim) {
        uint64_t wv[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) {
          const uint64_t x = w64[min(i + u, i1)];
          wv[u] = i + u < i1 ? x : 0ull;
        }
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) k += cnt(wv[u]);
      }
    }
    if (k >= lim) return false;
  }
  return true;
}

// Persistent learning step with local inhibition, two frames per exchange
// (the lookahead of the global step's k_sp_persistent_w): learning couples
// frame t + 1 to frame t only through each column's own synapses, so every
// wave publishes, with its columns' frame-t overlaps, their frame-(t+1)
// overlaps if they stay inactive in frame t and if they are active.  A
// workgroup then decides frame t for every column of its halo -- the
// bounding box of its columns' neighbourhoods, one column per thread,
// local_active on the frame-t copy -- and writes each halo column's
// frame-(t+1) overlap, picked by that decision, into LDS; each wave decides
// its own columns' frame t + 1 from there (lanes across a window row, as
// the one-frame kernel does), learns on the columns active in either frame,
// and computes the next pair's overlaps (speculatively while the exchange
// is in flight, redone for the columns that learned).  The results are
// exactly those of stepping the frames one by one.  Exchange layout, tags,
// poller, publishers and abort are those of the global two-frame kernel, in
// the local pair region of the workspace with its own exchange counter.
// Instances of the two-frame local step whose wave 0 gathers only after the
// workgroup's publish stores (as publish_first for the global step).  Timed
// both ways over 1000 learning frames of the 960x540 input (1-D grid, radius
// 80) at 256 x 32, 1024 x 64, 1024 x 256, 512 x 512, 2048 x 128 and
// 4096 x 64: faster by 3-12 % wherever a lane holds two or more exchange
// words, 8 % slower at one.
constexpr bool local2_publish_first(int, int nv, int) { return nv >= 2; }

template <int RPC, int NV, int RW, bool PF = local2_publish_first(RPC, NV, RW)>
__global__ __launch_bounds__(kPersistWaves * kWave) void k_sp_persistent_local2(LocalArgs a) {
  constexpr uint32_t CPW = RW / RPC;
  constexpr uint32_t CPAD = NV * 4 * kWave;      // entries per exchange array
  constexpr uint32_t NARR = 3;                   // frame t, frame t+1 if inactive, if active
  constexpr uint32_t WGC = kPersistWaves * CPW;  // columns per workgroup
  constexpr uint32_t kSeenAbort = 0xFFFFFFFFu;
  static_assert(kPersistWaves == NARR + 1, "waves 1..3 publish the three arrays");
  __shared__ uint64_t xl[2][NARR][NV * kWave];  // the exchange, word i = columns 4i..4i+3
  __shared__ uint64_t e1w[NV * kWave];          // frame t+1 overlaps of the halo columns
  __shared__ uint8_t a0[CPAD];                  // frame-t decisions of the halo columns
  __shared__ uint32_t hcell[kLocal2MaxHalo];    // halo cells: x | y << 16 (y * grid_w + x < C)
  __shared__ uint32_t nhalo;
  __shared__ uint32_t pub[NARR][WGC];
  __shared__ uint32_t seen;
  __shared__ uint32_t pubd[NARR];  // pairs each publishing wave has issued
  const Shape sh = a.sh;
  const uint32_t lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const uint32_t gw = blockIdx.x * kPersistWaves + wave;
  const uint32_t c_begin = gw * CPW;
  const uint32_t wg_begin = blockIdx.x * WGC;
  const uint32_t ncols = c_begin < sh.C ? min(CPW, sh.C - c_begin) : 0u;
  const uint32_t rows = (sh.C + a.grid_w - 1) / a.grid_w;
  const bool mine = lane < ncols;
  if (threadIdx.x < NARR) pubd[threadIdx.x] = 0;
  if (threadIdx.x == 0) seen = 0;

  // The halo box (rows hy0..hy0+bh-1, grid columns hx0..hx0+bw-1): the
  // neighbourhoods of the workgroup's columns; empty past C.
  // The halo box's cells that are columns (< C), listed once in LDS.
  if (threadIdx.x == 0) nhalo = 0;
  __syncthreads();
  if (wg_begin < sh.C) {
    const uint32_t wg_last = min(wg_begin + WGC, sh.C) - 1;
    const uint32_t yf = wg_begin / a.grid_w, yl = wg_last / a.grid_w;
    const uint32_t xf = yf == yl ? wg_begin % a.grid_w : 0u;
    const uint32_t xl_ = yf == yl ? wg_last % a.grid_w : a.grid_w - 1;
    const uint32_t hy0 = yf >= a.radius ? yf - a.radius : 0u;
    const uint32_t hx0 = xf >= a.radius ? xf - a.radius : 0u;
    const uint32_t bh = min(yl + a.radius, rows - 1) - hy0 + 1;
    const uint32_t bw = min(xl_ + a.radius, a.grid_w - 1) - hx0 + 1;
    for (uint32_t i = threadIdx.x; i < bh * bw; i += kPersistWaves * kWave) {
      const uint32_t y = hy0 + i / bw, x = hx0 + i % bw;
      if (y * a.grid_w + x < sh.C) hcell[atomicAdd(&nhalo, 1u)] = x | (y << 16);
    }
  }

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
  const uint32_t rep = xcc_id() % a.replicas;
  bool abort = false;

  auto stage = [&](const uint32_t(&o0)[CPW], const uint32_t(&oL)[CPW], const uint32_t(&oW)[CPW]) {
    if (lane < CPW) {
      pub[0][wave * CPW + lane] = lane_value(o0, lane);
      pub[1][wave * CPW + lane] = lane_value(oL, lane);
      pub[2][wave * CPW + lane] = lane_value(oW, lane);
    }
  };
  // Input words of frames t and t + 1 (t even), one 64-bit load per row
  // from their pair (clamped to the last pair).
  auto gather = [&](uint32_t t, uint32_t (&x0)[RW], uint32_t (&x1)[RW]) {
    const uint64_t* fp = a.fpair + (size_t)min(t / 2, (a.F - 1) / 2) * sh.W;
#pragma unroll
    for (uint32_t r = 0; r < RW; ++r) {
      const uint64_t v = fp[wi[r]];
      x0[r] = (uint32_t)v;
      x1[r] = (uint32_t)(v >> 32);
    }
  };
  // Frame t's overlap, the state after learning frame t, and frame t + 1's
  // overlap with the current state and with that state.
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
  // Algorithm 2 for own column c with overlap v against a copy by column
  // (lanes split each row of the window, four 64-column chunks a step, all
  // four reads in flight; stops at n).
  auto decide = [&](uint32_t c, uint32_t v, const uint16_t* ov) {
    if (v < 2) return false;
    const uint32_t cx = c % a.grid_w, cy = c / a.grid_w;
    const uint32_t y0 = cy >= a.radius ? cy - a.radius : 0u;
    const uint32_t y1 = min(cy + a.radius, rows - 1);
    const uint32_t x0 = cx >= a.radius ? cx - a.radius : 0u;
    const uint32_t x1 = min(cx + a.radius, a.grid_w - 1);
    uint32_t k = 0;
    for (uint32_t y = y0; y <= y1 && k < sh.k; ++y) {
      for (uint32_t xb = x0; xb <= x1 && k < sh.k; xb += 4 * kWave) {
        uint32_t o[4];
        bool in[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
          const uint32_t x = xb + u * kWave + lane, d = y * a.grid_w + x;
          in[u] = x <= x1 && d < sh.C && d != c;
          o[u] = ov[in[u] ? d : c];
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u)
          k += (uint32_t)__popcll(__ballot(in[u] && (o[u] & 0x3FFFu) >= v));
      }
    }
    return k < sh.k;
  };

  constexpr uint32_t kAllCols = (1u << CPW) - 1u;
  uint64_t* x64w = a.xchg;
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
        // (waves 1..3 publish at the top of every pair they enter)
        while (lds_acquire(&pubd[0]) <= pair || lds_acquire(&pubd[1]) <= pair ||
               lds_acquire(&pubd[2]) <= pair)
          __builtin_amdgcn_s_sleep(0);
      }
      const uint32_t tn = t + 2;
      const bool has_next = tn < a.F;
      uint32_t n0[RW], n1[RW];
      gather(tn, n0, n1);
      uint32_t sov0[CPW], sovL[CPW], sovW[CPW];
      uint32_t sstW[RW], smskW[RW];
      if (has_next) products(kAllCols, n0, n1, sov0, sovL, sovW, sstW, smskW);

      if constexpr (POLL) {
        uint64_t v0[NV], vL[NV], vW[NV];
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
        // (tags cleared: the halo pass compares whole words)
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          xl[pair & 1][0][u * kWave + lane] = v0[u] & kFieldBits;
          xl[pair & 1][1][u * kWave + lane] = vL[u] & kFieldBits;
          xl[pair & 1][2][u * kWave + lane] = vW[u] & kFieldBits;
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
      }

      // Frame t for every halo column, and its frame-(t+1) overlap.
      const uint64_t* x0w = xl[pair & 1][0];
      const uint16_t* xL16 = reinterpret_cast<const uint16_t*>(xl[pair & 1][1]);
      const uint16_t* xW16 = reinterpret_cast<const uint16_t*>(xl[pair & 1][2]);
      const uint16_t* x016 = reinterpret_cast<const uint16_t*>(x0w);
      uint16_t* e1 = reinterpret_cast<uint16_t*>(e1w);
      for (uint32_t i = threadIdx.x; i < nhalo; i += kPersistWaves * kWave) {
        const uint32_t xy = hcell[i], dx = xy & 0xFFFFu, dy = xy >> 16;
        const uint32_t d = dy * a.grid_w + dx;
        const bool act =
            local_active(dx, dy, x016[d], x0w, sh.C, a.grid_w, rows, a.radius, sh.k);
        a0[d] = act ? 1u : 0u;
        e1[d] = act ? xW16[d] : xL16[d];
      }
      __syncthreads();

      // Own columns: frame t from the halo pass, frame t + 1 against it.
      uint32_t sel0 = 0, sel1 = 0;
#pragma unroll
      for (uint32_t j = 0; j < CPW; ++j)
        if (j < ncols && a0[c_begin + j]) sel0 |= 1u << j;
      uint32_t my1[CPW];
#pragma unroll
      for (uint32_t j = 0; j < CPW; ++j) my1[j] = ((sel0 >> j) & 1u) ? ovW[j] : ovL[j];
      if (two) {
#pragma unroll
        for (uint32_t j = 0; j < CPW; ++j)
          if (j < ncols && decide(c_begin + j, my1[j], e1)) sel1 |= 1u << j;
      }
      if (mine) {
        const size_t o = (size_t)t * sh.C + c_begin + lane;
        a.active_out[o] = (uint8_t)((sel0 >> lane) & 1u);
        if (a.ov_out) a.ov_out[o] = (int32_t)lane_value(ov0, lane);
        if (two) {
          a.active_out[o + sh.C] = (uint8_t)((sel1 >> lane) & 1u);
          if (a.ov_out) a.ov_out[o + sh.C] = (int32_t)lane_value(my1, lane);
        }
      }

      // Learning on the own columns active in frame t (its state), then t + 1.
      uint32_t changed = 0;
      if (a.learn) {
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
      run(LocalRole<true>{});
    else
      run(LocalRole<false>{});
  }
  if (abort) {
    if (wave == 0 && lane == 0) store_tagged(a.err, 1u);
    return;
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

hipError_t launch_inhibit_local(const int32_t* ov, uint32_t F, uint32_t C, uint32_t grid_w,
                                uint32_t radius, uint32_t n, uint8_t* active, hipStream_t s,
                                const uint32_t* radius_dev, uint32_t* radius_out) {
  if (F == 0) return hipSuccess;
  const uint32_t col_blocks = (C + kLocalThreads - 1) / kLocalThreads;
  const dim3 grid(F * col_blocks);
  if (C <= kLocalLdsColumns)
    hipLaunchKernelGGL(k_inhibit_local<true>, grid, dim3(kLocalThreads), 0, s, ov, C, grid_w,
                       radius, n, col_blocks, active, radius_dev, radius_out);
  else
    hipLaunchKernelGGL(k_inhibit_local<false>, grid, dim3(kLocalThreads), 0, s, ov, C, grid_w,
                       radius, n, col_blocks, active, radius_dev, radius_out);
  return hipGetLastError();
}

hipError_t launch_radius_adapt(const uint32_t* idx, const float* perm, const Shape& sh,
                               uint32_t in_w, uint32_t grid_w, uint64_t* acc, uint32_t* radius,
                               hipStream_t s, bool reset_only) {
  const uint64_t in_h = ((uint64_t)sh.N + in_w - 1) / in_w;
  const uint64_t grid_h = ((uint64_t)sh.C + grid_w - 1) / grid_w;
  const uint64_t B = (uint64_t)grid_w * in_h + grid_h * in_w;
  const uint64_t area8 = 8ull * in_w * in_h;
  unsigned long long* a = reinterpret_cast<unsigned long long*>(acc);
  if (!reset_only) {
    hipLaunchKernelGGL(k_radius_span, dim3((sh.C + 3) / 4), dim3(256), 0, s, idx, perm, sh, in_w,
                       a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_radius_update, dim3(1), dim3(1), 0, s, a, radius, B, area8,
                     reset_only ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_learn_active(const uint32_t* idx, float* perm, const uint32_t* frame,
                               const uint8_t* active, const Shape& sh, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_active, dim3((sh.C + 3) / 4), dim3(256), 0, s, idx, perm, frame,
                     active, sh);
  return hipGetLastError();
}

const void* persistent_local_kernel(uint32_t rpc, uint32_t nv, uint32_t rw) {
#define HTMSP_PL(P, V, R)                              \
  if (rpc == P && nv == V && rw == R)                  \
    return reinterpret_cast<const void*>(&k_sp_persistent_local<P, V, R>);
  // The shapes persistent_wave_rows gives on a 256-CU device.
  HTMSP_PL(1, 1, 4) HTMSP_PL(1, 2, 4) HTMSP_PL(1, 4, 4) HTMSP_PL(1, 8, 4) HTMSP_PL(1, 16, 8)
  HTMSP_PL(2, 1, 4) HTMSP_PL(2, 2, 4) HTMSP_PL(2, 4, 4) HTMSP_PL(2, 8, 8) HTMSP_PL(2, 16, 16)
  HTMSP_PL(4, 1, 4) HTMSP_PL(4, 2, 4) HTMSP_PL(4, 4, 8) HTMSP_PL(4, 8, 16) HTMSP_PL(4, 16, 16)
  HTMSP_PL(8, 1, 8) HTMSP_PL(8, 2, 8) HTMSP_PL(8, 4, 16) HTMSP_PL(8, 8, 16) HTMSP_PL(16, 1, 16)
  HTMSP_PL(16, 2, 16) HTMSP_PL(16, 4, 16)
#undef HTMSP_PL
  return nullptr;
}

size_t persistent_local_exchange_bytes(uint32_t C) {
  return (size_t)2 * kPersistMaxReplicas * persistent_exchange_entries(C) * sizeof(uint16_t);
}

const void* persistent_local2_kernel(uint32_t rpc, uint32_t nv, uint32_t rw) {
#define HTMSP_PL2(P, V, R)                             \
  if (rpc == P && nv == V && rw == R)                  \
    return reinterpret_cast<const void*>(&k_sp_persistent_local2<P, V, R>);
  HTMSP_PL2(1, 1, 4) HTMSP_PL2(1, 2, 4) HTMSP_PL2(1, 4, 4) HTMSP_PL2(1, 8, 4) HTMSP_PL2(1, 16, 8)
  HTMSP_PL2(2, 1, 4) HTMSP_PL2(2, 2, 4) HTMSP_PL2(2, 4, 4) HTMSP_PL2(2, 8, 8) HTMSP_PL2(2, 16, 16)
  HTMSP_PL2(4, 1, 4) HTMSP_PL2(4, 2, 4) HTMSP_PL2(4, 4, 8) HTMSP_PL2(4, 8, 16) HTMSP_PL2(4, 16, 16)
  HTMSP_PL2(8, 1, 8) HTMSP_PL2(8, 2, 8) HTMSP_PL2(8, 4, 16) HTMSP_PL2(8, 8, 16) HTMSP_PL2(16, 1, 16)
  HTMSP_PL2(16, 2, 16) HTMSP_PL2(16, 4, 16)
#undef HTMSP_PL2
  return nullptr;
}

size_t persistent_local2_exchange_bytes(uint32_t C) {
  return (size_t)2 * kPersistReplicas * 3 * persistent_exchange_entries(C) * sizeof(uint16_t);
}

bool persistent_local2_fits(uint32_t C, uint32_t wgc, uint32_t grid_w, uint32_t radius) {
  if (grid_w < 1 || grid_w > C || wgc < 1) return false;
  const uint64_t rows = (C + grid_w - 1) / grid_w;
  const uint64_t win = std::min<uint64_t>(rows, 2ull * radius + 1) *
                       std::min<uint64_t>(grid_w, 2ull * radius + 1);
  if (win > kLocal2MaxWindow) return false;
  // every workgroup's halo box, as the kernel computes it
  for (uint64_t b = 0; b * wgc < C; ++b) {
    const uint64_t first = b * wgc, last = std::min<uint64_t>(first + wgc, C) - 1;
    const uint64_t yf = first / grid_w, yl = last / grid_w;
    const uint64_t xf = yf == yl ? first % grid_w : 0, xl = yf == yl ? last % grid_w : grid_w - 1;
    const uint64_t y0 = yf >= radius ? yf - radius : 0, x0 = xf >= radius ? xf - radius : 0;
    const uint64_t bh = std::min<uint64_t>(yl + radius, rows - 1) - y0 + 1;
    const uint64_t bw = std::min<uint64_t>(xl + radius, grid_w - 1) - x0 + 1;
    if (bh * bw > kLocal2MaxHalo) return false;
  }
  return true;
}

}  // namespace htmsp
