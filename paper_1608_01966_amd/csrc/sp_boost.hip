// Boosting and duty cycles: Algorithm 1 multiplies each column's gated
// overlap by its boost (Section 3.2.2 computes it in the kernel); the boost
// and the permanence raise follow the whitepaper's spatial pooler phase 3.
// Exact fixed point: boosts in 1/256, duty cycles in 1/65536, updated after
// each learning frame as d <- floor((d (P - 1) + 65536 e) / P) with
// P = 2^period_log2; the minimum duty cycle is a fraction (in 1/65536) of the
// largest active duty cycle; below it the boost rises linearly to
// max_boost_q8 at duty 0; a column whose overlap duty cycle is below it has
// every permanence raised by bump_q8 / 256, clipped at 1.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

using namespace dev;

constexpr uint32_t kBoostThreads = 1024;
constexpr uint32_t kBoostMaxColumns = 65536;  // the library's column limit

// One workgroup: duty cycles, minimum, boosts and raise flags of one frame.
// ov: the frame's boosted overlaps (positive iff the gated overlap is);
// winners: the frame's winners (-1 padded).
__global__ __launch_bounds__(kBoostThreads) void k_boost_update(
    const int32_t* __restrict__ ov, const int32_t* __restrict__ winners, Shape sh,
    BoostParams b, uint32_t* __restrict__ adc, uint32_t* __restrict__ odc,
    uint32_t* __restrict__ boost, uint8_t* __restrict__ raise) {
  __shared__ uint32_t won[kBoostMaxColumns / 32];
  __shared__ uint32_t red[kBoostThreads / kWave];
  const uint32_t tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const uint32_t nwords = (sh.C + 31) / 32;
  for (uint32_t i = tid; i < nwords; i += kBoostThreads) won[i] = 0;
  __syncthreads();
  for (uint32_t i = tid; i < sh.k; i += kBoostThreads) {
    const int32_t c = winners[i];
    if (c >= 0 && (uint32_t)c < sh.C) atomicOr(&won[c >> 5], 1u << (c & 31));
  }
  __syncthreads();
  const uint64_t P = 1ull << b.period_log2;
  uint32_t mx = 0;
  for (uint32_t c = tid; c < sh.C; c += kBoostThreads) {
    const uint32_t a = (won[c >> 5] >> (c & 31)) & 1u;
    const uint32_t na = (uint32_t)(((uint64_t)adc[c] * (P - 1) + (a ? 65536u : 0u)) >> b.period_log2);
    const uint32_t no = (uint32_t)(((uint64_t)odc[c] * (P - 1) + (ov[c] > 0 ? 65536u : 0u)) >>
                                   b.period_log2);
    adc[c] = na;
    odc[c] = no;
    mx = max(mx, na);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, off));
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  mx = 0;
  for (uint32_t i = 0; i < kBoostThreads / kWave; ++i) mx = max(mx, red[i]);
  const uint32_t mn = (uint32_t)(((uint64_t)mx * b.min_pct_q16) >> 16);
  for (uint32_t c = tid; c < sh.C; c += kBoostThreads) {
    const uint32_t a = adc[c];
    boost[c] = (mn == 0 || a >= mn)
                   ? 256u
                   : 256u + (uint32_t)(((uint64_t)(b.max_boost_q8 - 256u) * (mn - a)) / mn);
    raise[c] = odc[c] < mn ? 1 : 0;
  }
}

// One wave per column: the permanence raise of flagged columns.
__global__ __launch_bounds__(256) void k_boost_raise(float* __restrict__ perm,
                                                     const uint8_t* __restrict__ raise,
                                                     Shape sh, uint32_t bump_q8) {
  const uint32_t c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  if (c >= sh.C || !raise[c]) return;
  float* cp = perm + (size_t)c * sh.S;
  for (uint32_t s = lane; s < sh.S; s += kWave)
    cp[s] = q_to_perm(min(perm_to_q(cp[s]) + bump_q8, 256u));
}

__global__ __launch_bounds__(256) void k_boost_init(uint32_t* __restrict__ adc,
                                                    uint32_t* __restrict__ odc,
                                                    uint32_t* __restrict__ boost, uint32_t C) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  adc[c] = 0;
  odc[c] = 0;
  boost[c] = 256;
}

// Persistent boosted learning step, the order of a frame as in the launch
// sequence above: boosted overlaps with the current boosts, global top-k of
// the boosted values (ties to the lower index), learning on the winners, duty
// cycles, minimum, boosts, permanence raise.  Columns are split as in the
// other persistent kernels (kPersistWaves waves per workgroup, a column
// group per wave, synapses in registers).  Per frame every wave publishes
// its columns' gated overlaps through a tagged exchange; wave 0 of each
// workgroup reads all of them into LDS; then every wave holds, for the
// columns u * 256 + 4 * lane + q of its lane (u < NV, q < 4), their gated
// overlap, duty cycles and boost, resolves the top-k of the boosted values
// and updates every column's duty cycles and boost itself, so that no second
// exchange is needed for the maximum duty cycle.  Global wave 0 writes the
// frame's winners and boosted overlaps and, at the end, the duty cycles and
// boosts.
template <bool B>
struct BoostRole {
  static constexpr bool value = B;
};

// Columns of the lane whose boosted value is >= x, summed over the wave.
template <int N>
__device__ __forceinline__ uint32_t count_ge32(const uint32_t (&bv)[N], uint32_t x) {
  uint32_t n = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) n += bv[i] >= x ? 1u : 0u;
  return wave_count<ilog2(N) + 1>(n);
}

// T = the largest x >= 1 with #(value >= x) >= k (0 when fewer than k
// values are positive), *c_hi = #(value >= T + 1).  Boosted values are
// overlaps times a boost in 1/256 units, and those near the threshold are
// often whole multiples of 256 (unboosted columns), so the search runs in two
// stages: the coarse threshold y (largest y with #(value >= 256 y) >= k) by
// a gallop from guess / 256 and a binary search, then one count at 256 y + 1,
// which settles T = 256 y whenever no value lies strictly between 256 y and
// 256 (y + 1); only otherwise a binary search of the 255 values between.
template <int N>
__device__ __forceinline__ uint32_t topk_threshold32(const uint32_t (&bv)[N], uint32_t vmax,
                                                     uint32_t k, uint32_t guess,
                                                     uint32_t* c_hi_out) {
  // Stage 1 over y, counting values >= y << 8; c_hi = #(value >= (hi + 1) << 8).
  const uint32_t ymax = vmax >> 8;
  uint32_t lo = 0, hi = ymax, c_hi = 0;
  if (ymax > 0) {
    const uint32_t g0 = min(max(guess >> 8, 1u), ymax);
    const uint32_t c0 = count_ge32(bv, g0 << 8);
    if (c0 >= k) {
      lo = g0;
      for (uint32_t step = 1; lo < hi; step <<= 1) {
        const uint32_t y = hi - lo > step ? lo + step : hi;
        const uint32_t cy = count_ge32(bv, y << 8);
        if (cy >= k) {
          lo = y;
        } else {
          hi = y - 1;
          c_hi = cy;
          break;
        }
      }
    } else {
      hi = g0 - 1;
      c_hi = c0;
      for (uint32_t step = 1; hi > 0; step <<= 1) {
        const uint32_t y = hi >= step ? hi - step + 1 : 1u;
        const uint32_t cy = count_ge32(bv, y << 8);
        if (cy >= k) {
          lo = y;
          break;
        }
        hi = y - 1;
        c_hi = cy;
      }
    }
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo + 1) / 2;
      const uint32_t c = count_ge32(bv, mid << 8);
      if (c >= k) {
        lo = mid;
      } else {
        hi = mid - 1;
        c_hi = c;
      }
    }
  }  // (ymax == 0: every value is below 256 = (hi + 1) << 8, so c_hi = 0)
  // Stage 2 in [base, base + 255]: #(value >= base) >= k (base >= 1) and
  // #(value >= base + 256) = c_hi < k.
  const uint32_t base = lo << 8;
  const uint32_t c1 = count_ge32(bv, base + 1u);
  if (c1 < k) {
    *c_hi_out = c1;
    return base;
  }
  uint32_t flo = base + 1u, fhi = min(base + 255u, vmax), fc = c_hi;
  while (flo < fhi) {
    const uint32_t mid = flo + (fhi - flo + 1) / 2;
    const uint32_t c = count_ge32(bv, mid);
    if (c >= k) {
      flo = mid;
    } else {
      fhi = mid - 1;
      fc = c;
    }
  }
  *c_hi_out = fc;
  return flo;
}

template <int RPC, int NV, int RW>
__global__ __launch_bounds__(kPersistWaves * kWave) void k_sp_persistent_boost(BoostArgs a) {
  constexpr uint32_t CPW = RW / RPC;
  constexpr uint32_t WGC = kPersistWaves * CPW;
  constexpr uint32_t NC = 4 * NV;  // columns per lane
  constexpr uint32_t kSeenAbort = 0xFFFFFFFFu;
  __shared__ uint64_t xl[2][NV * kWave];
  __shared__ uint32_t pub[WGC];
  __shared__ uint32_t seen;
  const Shape sh = a.sh;
  const BoostParams b = a.b;
  const uint32_t lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const uint32_t gw = blockIdx.x * kPersistWaves + wave;
  const uint32_t c_begin = gw * CPW;
  const uint32_t wg_begin = blockIdx.x * WGC;
  const uint32_t ncols = c_begin < sh.C ? min(CPW, sh.C - c_begin) : 0u;
  const uint32_t vmax = sh.S * b.max_boost_q8;
  const uint64_t P1 = (1ull << b.period_log2) - 1ull;
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
  // Every column's duty cycles and boost, in the exchange's column order.
  uint32_t adc[NC], odc[NC], bst[NC];
#pragma unroll
  for (uint32_t i = 0; i < NC; ++i) {
    const uint32_t c = (i / 4) * 4 * kWave + 4 * lane + i % 4;
    adc[i] = c < sh.C ? a.adc[c] : 0u;
    odc[i] = c < sh.C ? a.odc[c] : 0u;
    bst[i] = c < sh.C ? a.boost[c] : 256u;
  }
  const uint32_t rep = xcc_id() % a.replicas;
  uint32_t guess = 1 + vmax / 16;
  bool abort = false;

  auto gather = [&](uint32_t t, uint32_t (&x)[RW]) {
    const uint32_t* f = a.frames + (size_t)min(t, a.F - 1) * sh.W;
#pragma unroll
    for (uint32_t r = 0; r < RW; ++r) x[r] = f[wi[r]];
  };
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
  // Bits of the own columns (bit j: column c_begin + j) in the masks `m`
  // whose bit 4u + q in lane l stands for column u * 256 + 4l + q.  A wave's
  // CPW columns start at a multiple of CPW (<= 16), so up to four of them
  // share one lane, whose mask is then read as a scalar.  Every lane calls it.
  auto own_bits = [&](uint32_t m) {
    uint32_t r = 0;
    if constexpr (CPW <= 4) {
      const uint32_t src = __builtin_amdgcn_readfirstlane((c_begin % (4 * kWave)) / 4);
      const uint32_t ms = __builtin_amdgcn_readlane(m, src);
#pragma unroll
      for (uint32_t j = 0; j < CPW; ++j) {
        const uint32_t c = c_begin + j;
        r |= (j < ncols && ((ms >> ((c / (4 * kWave)) * 4 + c % 4)) & 1u)) ? 1u << j : 0u;
      }
    } else {
#pragma unroll
      for (uint32_t j = 0; j < CPW; ++j) {
        const uint32_t c = c_begin + j;
        const uint32_t ms = (uint32_t)__shfl((int)m, (int)((c % (4 * kWave)) / 4));
        r |= (j < ncols && ((ms >> ((c / (4 * kWave)) * 4 + c % 4)) & 1u)) ? 1u << j : 0u;
      }
    }
    return r;
  };

  // Frame wt's winners in column order from their bits (bit 4u + q of lane
  // l: column u * 256 + 4l + q) and count, then the -1 padding; global wave 0
  // writes them while the next frame's exchange is in flight.
  auto write_winners = [&](uint32_t ws, uint32_t wn, uint32_t wt) {
    int32_t* wr = a.win_out + (size_t)wt * sh.k;
    uint32_t before = 0;
#pragma unroll
    for (uint32_t u = 0; u < NV; ++u) {
      const uint32_t su = (ws >> (4 * u)) & 15u;
      uint32_t pos = before + wave_prefix<3>((uint32_t)__popc(su), lane);
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q)
        if ((su >> q) & 1u) wr[pos++] = (int32_t)(u * 4 * kWave + 4 * lane + q);
      before += wave_count<3>((uint32_t)__popc(su));
    }
    for (uint32_t i = wn + lane; i < sh.k; i += kWave) wr[i] = -1;
  };

  auto run = [&](auto role) {
    constexpr bool POLL = decltype(role)::value;
    uint32_t w[RW], o[CPW];
    uint32_t wsel = 0, wnsel = 0, wt = 0;  // global wave 0: winners not yet written
    bool wpend = false;
    gather(0, w);
    overlaps((1u << CPW) - 1u, w, o);
    if (lane < CPW) pub[wave * CPW + lane] = lane_value(o, lane);
    __syncthreads();
    for (uint32_t t = 0; t < a.F; ++t) {
      const uint32_t g = a.frame_base + t;
      const uint32_t slot = g & 1u;
      const uint32_t tg = ((g + 1u) & 3u) << kTagShift;
      uint64_t* xs = a.xchg + (size_t)(rep * 2 + slot) * NV * kWave;
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
      overlaps((1u << CPW) - 1u, nx, on);  // speculation: no own column changes
      if (gw == 0 && wpend) write_winners(wsel, wnsel, wt);

      uint64_t v[NV];
      if constexpr (POLL) {
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
#pragma unroll
        for (int u = 0; u < NV; ++u) v[u] = xl[t & 1][u * kWave + lane];
      }

      // Boosted values and the frame's top-k.
      uint32_t gv[NC], bv[NC];
#pragma unroll
      for (uint32_t i = 0; i < NC; ++i) {
        const uint32_t c = (i / 4) * 4 * kWave + 4 * lane + i % 4;
        gv[i] = c < sh.C ? (uint32_t)(v[i / 4] >> (16 * (i % 4))) & 0x3FFFu : 0u;
        bv[i] = gv[i] * bst[i];
      }
      uint32_t c_hi;
      const uint32_t T = topk_threshold32(bv, vmax, sh.k, guess, &c_hi);
      if (T) guess = T;
      const uint32_t need = T ? sh.k - c_hi : 0u;
      const uint32_t nsel = T ? sh.k : c_hi;
      // Winners in column order: every value above T, then the first `need`
      // equal to T; `sel` holds bit 4u + q for column u * 256 + 4 * lane + q.
      // Ties are ranked in the one word where the `need` quota runs out:
      // earlier words take all their ties, later ones none.
      uint32_t sel = 0, eq_before = 0;
#pragma unroll
      for (uint32_t u = 0; u < NV; ++u) {
        uint32_t gt = 0, eq = 0;
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
          gt |= bv[4 * u + q] > T ? 1u << q : 0u;
          eq |= (T != 0 && bv[4 * u + q] == T) ? 1u << q : 0u;
        }
        uint32_t take = 0;
        if (eq_before < need) {
          const uint32_t neq = (uint32_t)__popc(eq);
          const uint32_t tot = wave_count<3>(neq);
          if (eq_before + tot <= need) {
            take = eq;
          } else {
            const uint32_t pre = eq_before + wave_prefix<3>(neq, lane);
            uint32_t keep = need > pre ? need - pre : 0u;
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q) {
              const bool use = ((eq >> q) & 1u) && keep > 0;
              take |= use ? 1u << q : 0u;
              keep -= use ? 1u : 0u;
            }
          }
          eq_before += tot;
        }
        sel |= (gt | take) << (4 * u);
      }
      if (gw == 0) {
        wsel = sel;
        wnsel = nsel;
        wt = t;
        wpend = true;
        if (a.ov_out) {
#pragma unroll
          for (uint32_t i = 0; i < NC; ++i) {
            const uint32_t c = (i / 4) * 4 * kWave + 4 * lane + i % 4;
            if (c < sh.C) a.ov_out[(size_t)t * sh.C + c] = (int32_t)bv[i];
          }
        }
      }

      uint32_t changed = 0;
      if (a.learn) {
        // Learning on the own columns that won, with frame t.
        const uint32_t won = own_bits(sel);
#pragma unroll
        for (uint32_t r = 0; r < RW; ++r) {
          if ((won >> (r / RPC)) & (row_ok >> r) & 1u) {
            const uint32_t i = st[r] >> 9;
            const uint32_t q = learn_q(st[r] & 511u, input_bit(w[r], i), sh);
            st[r] = (i << 9) | q;
            msk[r] = q >= sh.theta ? 1u << (i & 31u) : 0u;
          }
        }
        // Duty cycles of every column, their maximum (17 bits, one ballot a
        // bit from the top), the minimum, boosts.
        uint32_t mx = 0;
#pragma unroll
        for (uint32_t i = 0; i < NC; ++i) {
          adc[i] = (uint32_t)(((uint64_t)adc[i] * P1 + (((sel >> i) & 1u) ? 65536u : 0u)) >>
                              b.period_log2);
          odc[i] = (uint32_t)(((uint64_t)odc[i] * P1 + (gv[i] > 0 ? 65536u : 0u)) >>
                              b.period_log2);
          mx = max(mx, adc[i]);
        }
        uint32_t wmx = 0;
#pragma unroll
        for (int bit = 16; bit >= 0; --bit) {
          const uint32_t cand = wmx | (1u << bit);
          if (__ballot(mx >= cand) != 0ull) wmx = cand;
        }
        const uint32_t mn = (uint32_t)(((uint64_t)wmx * b.min_pct_q16) >> 16);
        // (max_boost - 256)(mn - a) / mn exactly, as (num * mg) >> (28 + l)
        // with l = ceil(log2 mn) and mg = ceil(2^(28 + l) / mn): exact for
        // numerators below 2^28 (the error term stays below 1 / mn), and num
        // <= 3840 * 65536.
        const uint32_t l = mn > 1 ? 32u - (uint32_t)__clz(mn - 1u) : 0u;
        const uint64_t p2 = 1ull << (28 + l);
        uint64_t mg = 0;
        if (mn) {
          // a double estimate of the ceiling, then the two integer checks
          mg = (uint64_t)((double)p2 / (double)mn);
          mg = mg * mn < p2 ? mg + 1u : mg;
          mg = (mg - 1u) * mn >= p2 ? mg - 1u : mg;
        }
        uint32_t raise = 0;
#pragma unroll
        for (uint32_t i = 0; i < NC; ++i) {
          const uint32_t num = (b.max_boost_q8 - 256u) * (mn - min(adc[i], mn));
          const uint32_t qt = (uint32_t)(((uint64_t)num * mg) >> (28 + l));
          bst[i] = 256u + qt;
          raise |= (odc[i] < mn) ? 1u << i : 0u;
        }
        // Permanence raise of the own columns whose overlap duty is below it.
        if (b.bump_q8) {
          const uint32_t up = own_bits(raise);
#pragma unroll
          for (uint32_t r = 0; r < RW; ++r) {
            if ((up >> (r / RPC)) & (row_ok >> r) & 1u) {
              const uint32_t i = st[r] >> 9;
              const uint32_t q = min((st[r] & 511u) + b.bump_q8, 256u);
              st[r] = (i << 9) | q;
              msk[r] = q >= sh.theta ? 1u << (i & 31u) : 0u;
            }
          }
          changed = won | up;
        } else {
          changed = won;
        }
      }
      if (changed) overlaps(changed, nx, on);
#pragma unroll
      for (uint32_t r = 0; r < RW; ++r) w[r] = nx[r];
#pragma unroll
      for (uint32_t j = 0; j < CPW; ++j) o[j] = on[j];
      if (lane < CPW) pub[wave * CPW + lane] = lane_value(o, lane);
      __syncthreads();
    }
    if (!abort && gw == 0 && wpend) write_winners(wsel, wnsel, wt);
  };
  if (a.F > 0) {
    if (wave == 0)
      run(BoostRole<true>{});
    else
      run(BoostRole<false>{});
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
    if (gw == 0) {
#pragma unroll
      for (uint32_t i = 0; i < NC; ++i) {
        const uint32_t c = (i / 4) * 4 * kWave + 4 * lane + i % 4;
        if (c < sh.C) {
          a.adc[c] = adc[i];
          a.odc[c] = odc[i];
          a.boost[c] = bst[i];
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_boost_update(const int32_t* ov, const int32_t* winners, const Shape& sh,
                               const BoostParams& b, uint32_t* adc, uint32_t* odc,
                               uint32_t* boost, uint8_t* raise, float* perm, hipStream_t s) {
  hipLaunchKernelGGL(k_boost_update, dim3(1), dim3(kBoostThreads), 0, s, ov, winners, sh, b, adc,
                     odc, boost, raise);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || b.bump_q8 == 0) return e;
  hipLaunchKernelGGL(k_boost_raise, dim3((sh.C + 3) / 4), dim3(256), 0, s, perm, raise, sh,
                     b.bump_q8);
  return hipGetLastError();
}

hipError_t launch_boost_init(uint32_t* adc, uint32_t* odc, uint32_t* boost, uint32_t C,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_boost_init, dim3((C + 255) / 256), dim3(256), 0, s, adc, odc, boost, C);
  return hipGetLastError();
}

const void* persistent_boost_kernel(uint32_t rpc, uint32_t nv, uint32_t rw) {
#define HTMSP_PB(P, V, R)                              \
  if (rpc == P && nv == V && rw == R)                  \
    return reinterpret_cast<const void*>(&k_sp_persistent_boost<P, V, R>);
  // The shapes persistent_wave_rows gives on a 256-CU device.
  HTMSP_PB(1, 1, 4) HTMSP_PB(1, 2, 4) HTMSP_PB(1, 4, 4) HTMSP_PB(2, 1, 4) HTMSP_PB(2, 2, 4)
  HTMSP_PB(2, 4, 4) HTMSP_PB(4, 1, 4) HTMSP_PB(4, 2, 4) HTMSP_PB(4, 4, 8) HTMSP_PB(8, 1, 8)
  HTMSP_PB(8, 2, 8) HTMSP_PB(8, 4, 16) HTMSP_PB(16, 1, 16) HTMSP_PB(16, 2, 16)
  HTMSP_PB(16, 4, 16)
#undef HTMSP_PB
  return nullptr;
}

}  // namespace htmsp
