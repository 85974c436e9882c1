// Internal interface between the C-ABI host code (sp_api.hip) and the
// kernels (sp_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace htmsp {

// Shape and learning parameters shared by every kernel, permanences in
// 1/256 units.
struct Shape {
  uint32_t N, C, S, W;      // input bits, columns, synapses per column, words per frame
  uint32_t m, k;            // min_overlap, winners_set_size
  uint32_t theta, inc, dec; // connected threshold, increment, decrement (x256)
};

// Persistent multi-frame step: every column spread over `rpc` rows of 64
// synapses, a group of consecutive columns per wave.
struct PersistArgs {
  const uint32_t* idx;
  float* perm;
  // [ceil(F/2)][W]: word i of frame 2p in the low half of entry p * W + i,
  // of frame min(2p + 1, F - 1) in the high half (launch_pair_frames)
  const uint64_t* fpair;
  int32_t* ov_out;    // [F][C] or null
  int32_t* win_out;   // [F][k]
  uint32_t* xchg;     // [replicas][2][arrays][entries] 16-bit tagged overlaps
  uint32_t* err;      // set to non-zero when a wave gives up waiting
  uint32_t F, learn, frame_base, replicas, spin_limit;  // frame_base counts exchanges
  uint32_t stall;  // 0; a test of the failure path sets 1 (see sp_test_stall)
  Shape sh;
};

// Largest C the persistent kernel exchanges (16 64-bit words per lane).
constexpr uint32_t kPersistMaxColumns = 4096;
// Largest S it holds: 16 rows of 64 synapses per workgroup.
constexpr uint32_t kPersistMaxSynapses = 1024;
// Exchange copies the workspace holds (one per XCD at most), and the number
// used: readers pick the copy of their XCD modulo this.  Measured at
// 960x540, 1024 x 256 with the column-group-per-wave kernels: one copy is
// 2-3 % faster than two and two than four (every copy costs each publisher
// a store; the readers of one copy do not contend measurably).
constexpr uint32_t kPersistMaxReplicas = 8;
constexpr uint32_t kPersistReplicas = 1;

// Exchange arrays per slot (frame t, frame t+1 if lost, frame t+1 if won).
uint32_t persistent_exchange_arrays();
// 16-bit exchange entries per array for C columns: 256 times the power of two
// of 64-bit words per lane that covers C.
uint32_t persistent_exchange_entries(uint32_t C);
// Persistent learning step with local inhibition: F frames in one
// cooperative launch, one frame per exchange of every column's overlap.
struct LocalArgs {
  const uint32_t* idx;
  float* perm;
  const uint32_t* frames;    // the one-frame kernel
  const uint64_t* fpair;     // the two-frame kernel: as PersistArgs::fpair
  int32_t* ov_out;     // [F][C] or null
  uint8_t* active_out; // [F][C]
  uint64_t* xchg;      // [replicas][2][entries / 4] tagged overlaps
  uint32_t* err;
  uint32_t F, learn, frame_base, replicas, spin_limit;
  uint32_t stall;  // 0; a test of the failure path sets 1 (see sp_test_stall)
  uint32_t grid_w, radius;  // the neighbourhood; n = sh.k
  Shape sh;
};
// The persistent local-inhibition instance for `rpc` rows per column, `nv`
// exchange words per lane and `rw` rows per wave (kPersistWaves waves per
// workgroup, one workgroup per CU); nullptr otherwise.
const void* persistent_local_kernel(uint32_t rpc, uint32_t nv, uint32_t rw);
// Exchange bytes of the persistent local step for C columns.
size_t persistent_local_exchange_bytes(uint32_t C);
// The two-frames-per-exchange local instance (same shapes), its exchange
// bytes (three arrays), and whether it serves a neighbourhood: every
// workgroup of `wgc` columns decides a halo of at most kLocal2MaxHalo
// columns per pair, one thread each, each scanning at most kLocal2MaxWindow
// neighbours.
constexpr uint64_t kLocal2MaxHalo = 1024;
constexpr uint64_t kLocal2MaxWindow = 2048;
const void* persistent_local2_kernel(uint32_t rpc, uint32_t nv, uint32_t rw);
size_t persistent_local2_exchange_bytes(uint32_t C);
bool persistent_local2_fits(uint32_t C, uint32_t wgc, uint32_t grid_w, uint32_t radius);

// Waves per workgroup of the one-column-group-per-wave kernel.
constexpr uint32_t kPersistWaves = 4;
// Rows of 64 synapses per wave for the column-group-per-wave kernels (the
// global, local and boosted steps): the fewest of 4, 8 or 16 (at least
// `rpc`, whole columns) that keep the grid to half the CUs, else to all of
// them; 0 if none fits.  *grid gets the workgroups.  Fewer, fuller
// workgroups mean fewer readers of the per-frame exchange against more
// work per wave; measured at 960x540, 1024 x 256: 128 workgroups of 2
// columns per wave ran 2 % (global) and 13 % (local) faster than 256 of 1,
// and 64 of 4 ran 25 % slower.
inline uint32_t persistent_wave_rows(uint32_t C, uint32_t rpc, int cus, uint32_t* grid) {
  const uint32_t limits[2] = {(uint32_t)cus / 2, (uint32_t)cus};
  for (uint32_t limit : limits) {
    for (uint32_t rw = 4; rw <= 16; rw *= 2) {
      if (rw < rpc) continue;
      const uint32_t cols = rw / rpc * kPersistWaves;
      const uint32_t g = (C + cols - 1) / cols;
      if (g <= limit) {
        *grid = g;
        return rw;
      }
    }
  }
  return 0;
}
// The one-column-group-per-wave instance for `rpc` rows per column, `nv`
// exchange words per lane and `rw` rows per wave; nullptr otherwise.
const void* persistent_wave_kernel(uint32_t rpc, uint32_t nv, uint32_t rw);

hipError_t launch_check_state(const uint32_t* idx, const float* perm, size_t n, uint32_t N,
                              uint32_t* out4, hipStream_t s);
// Gated overlaps of one frame; times boost[c] (1/256 units) when boost is set.
hipError_t launch_overlap_plain(const uint32_t* idx, const float* perm, const uint32_t* frame,
                                int32_t* ov, const Shape& sh, hipStream_t s,
                                const uint32_t* boost = nullptr);
// Top-k of `frames` consecutive frames (overlaps [frames][C], winners
// [frames][k]), one workgroup per frame.
// Overlaps lie in [0, vmax] (0: S).
hipError_t launch_topk_plain(const int32_t* ov, int32_t* winners, const Shape& sh, hipStream_t s,
                             uint32_t frames = 1, uint32_t vmax = 0);
// The frames of a step side by side in pairs (the layout of PersistArgs::fpair),
// so that a kernel stepping two frames per exchange reads a synapse's input
// words of both with one 64-bit load.
hipError_t launch_pair_frames(const uint32_t* frames, uint32_t F, uint32_t W, uint64_t* out,
                              hipStream_t s);
// Bytes of paired frames one persistent launch reads at most; longer steps
// run as several launches.
constexpr size_t kPairStageBytes = size_t(64) << 20;
hipError_t launch_learn_plain(const uint32_t* idx, float* perm, const uint32_t* frame,
                              const int32_t* winners, const Shape& sh, hipStream_t s);

// Batched inference (sp_infer.hip).
// Longest connected list the register-resident gather kernel holds.
uint32_t infer_max_list();
// Compacts every column's connected inputs into list [S][C] (slot-major,
// padded with a pixel whose word is zero), counts in cnt [C], max in *maxcnt
// (maxcnt null: not counted, and nothing is cleared).
hipError_t launch_infer_prep(const uint32_t* idx, const float* perm, const Shape& sh,
                             uint32_t* list, uint32_t* cnt, uint32_t* maxcnt, hipStream_t s);
// Overlaps [F][C] of F frames from the compacted lists (maxn <= infer_max_list()).
hipError_t launch_infer_gather(uint32_t maxn, const uint32_t* frames, uint32_t F,
                               const uint32_t* list, const uint32_t* cnt, const Shape& sh,
                               int32_t* ov, uint32_t cus, hipStream_t s);
// Winners [F][k] from overlaps [F][C], one wave per frame (C <= 4096; else
// hipErrorInvalidValue).
hipError_t launch_topk_batch(const int32_t* ov, uint32_t F, const Shape& sh, int32_t* winners,
                             hipStream_t s);

// Batched inference as a dense int8 matrix product (sp_infer_mfma.hip):
// overlaps [F][C] = frames (0/1 per pixel) x connected mask (0/1), widened
// from bits to int8 in registers, int32 accumulation.
// Words per row of the bit mask [C][Wm] for W words per frame.
uint32_t mfma_mask_words(uint32_t W);
// Builds the mask of the connected synapses (zeroing it first) and counts
// in *dup the connected synapses of a column that repeat a pixel.
hipError_t launch_mfma_mask(const uint32_t* idx, const float* perm, const Shape& sh,
                            uint32_t* mask, uint32_t* dup, hipStream_t s);
// Splits of the pixel range for F frames (partial sums [splits][F][C] when
// above 1) on a device of `cus` compute units.
uint32_t mfma_splits(const Shape& sh, uint32_t F, uint32_t cus);
// Gated overlaps [F][C] into ov; `part` holds splits * F * C partial sums
// (unused when splits == 1).  F * W and C * mfma_mask_words(W) must stay
// below 2^31.
hipError_t launch_infer_mfma(const uint32_t* frames, uint32_t F, const uint32_t* mask,
                             const Shape& sh, uint32_t splits, int32_t* part, int32_t* ov,
                             hipStream_t s);

// Adaptive video encoder (sp_encode.hip).  W x H RGB input, w x h output
// (w = W / factor, h = H / factor), `words` per encoded frame; block means
// use area = factor^2 and area_magic = ceil(2^32 / area) (factor <= 32).
struct EncShape {
  uint32_t W, H, factor, block;
  int32_t offset;
  uint32_t w, h, words;
  uint32_t area, area_magic;
};
hipError_t launch_encode(const uint8_t* rgb, uint32_t F, const EncShape& e, uint32_t* out,
                         hipStream_t s);

// Boosting and duty cycles (sp_boost.hip), per learning frame after the
// winners' learning: duty cycles, the minimum, boosts, and the permanence
// raise of columns whose overlap duty cycle is below the minimum.
struct BoostParams {
  uint32_t period_log2, min_pct_q16, max_boost_q8, bump_q8;
};
hipError_t launch_boost_update(const int32_t* ov, const int32_t* winners, const Shape& sh,
                               const BoostParams& b, uint32_t* adc, uint32_t* odc,
                               uint32_t* boost, uint8_t* raise, float* perm, hipStream_t s);
hipError_t launch_boost_init(uint32_t* adc, uint32_t* odc, uint32_t* boost, uint32_t C,
                             hipStream_t s);
// Persistent boosted learning step: F frames in one cooperative launch, one
// exchange of every column's gated overlap per frame (the local step's
// exchange region and tag sequence).
struct BoostArgs {
  const uint32_t* idx;
  float* perm;
  const uint32_t* frames;
  int32_t* ov_out;   // [F][C] boosted overlaps, or null
  int32_t* win_out;  // [F][k]
  uint64_t* xchg;
  uint32_t* err;
  uint32_t* adc;     // [C] active duty cycles (1/65536), updated in place
  uint32_t* odc;     // [C] overlap duty cycles
  uint32_t* boost;   // [C] boosts (1/256)
  uint32_t F, learn, frame_base, replicas, spin_limit;
  uint32_t stall;  // 0; a test of the failure path sets 1 (see sp_test_stall)
  BoostParams b;
  Shape sh;
};
// Largest C of the persistent boosted step (every wave keeps every column's
// duty cycles and boost in registers).
constexpr uint32_t kBoostPersistMaxColumns = 1024;
// The persistent boosted instance for `rpc` rows per column, `nv` exchange
// words per lane and `rw` rows per wave; nullptr otherwise.
const void* persistent_boost_kernel(uint32_t rpc, uint32_t nv, uint32_t rw);

// Local inhibition (sp_local.hip): active [F][C] from overlaps [F][C].
hipError_t launch_inhibit_local(const int32_t* ov, uint32_t F, uint32_t C, uint32_t grid_w,
                                uint32_t radius, uint32_t n, uint8_t* active, hipStream_t s,
                                const uint32_t* radius_dev = nullptr,
                                uint32_t* radius_out = nullptr);
// Inhibition radius adaptation after a learning frame: the connected
// receptive-field extents of every column summed into acc[0..1] (A, n),
// then *radius = max(1, floor(A B / (8 n in_w in_h))) unless n == 0, and
// acc cleared.  reset_only: only clear acc.
hipError_t launch_radius_adapt(const uint32_t* idx, const float* perm, const Shape& sh,
                               uint32_t in_w, uint32_t grid_w, uint64_t* acc, uint32_t* radius,
                               hipStream_t s, bool reset_only = false);
// Learning of one frame on the columns flagged in active[C].
hipError_t launch_learn_active(const uint32_t* idx, float* perm, const uint32_t* frame,
                               const uint8_t* active, const Shape& sh, hipStream_t s);

// Adds 1 to hist[c] for every entry c >= 0 of winners[n] (sp_hist.hip).
// Adds, for every column c, the frames of active [F][C] (0/1) with c active.
hipError_t launch_hist_add_active(const uint8_t* active, uint32_t F, uint32_t C, uint32_t* hist,
                                  hipStream_t s);
hipError_t launch_hist_add(const int32_t* winners, size_t n, uint32_t C, uint32_t* hist,
                           hipStream_t s);

// Many instances in one persistent launch (sp_many.hip).
constexpr uint32_t kManyNV = 16;          // top-k words per lane: C <= 4096
constexpr uint32_t kTileSynapses = 4096;  // synapses per tile task (at most)
constexpr uint32_t kTileColumns = 1024;   // columns per tile task (at most)
constexpr uint32_t kManyThreads = 256;
constexpr uint32_t kMaxTileSlots = 16;    // tile tasks per workgroup (at most)
constexpr uint32_t kMaxTopkSlots = 32;    // top-k tasks per (top-k) workgroup (at most)

// Top-k workgroups of a many-instance launch over `nact` instances and at
// most `maxb` co-resident workgroups: one instance per wave while that keeps
// to an eighth of the grid, more per wave (up to kMaxTopkSlots per
// workgroup) beyond that.
inline uint32_t many_topk_blocks(size_t nact, size_t maxb) {
  const size_t one_per_wave = (nact + 3) / 4, fewest = (nact + kMaxTopkSlots - 1) / kMaxTopkSlots;
  return (uint32_t)std::min(one_per_wave, std::max(fewest, maxb / 8));
}

struct ManyInst {
  const uint32_t* idx;
  float* perm;
  const uint32_t* frames;  // [F][W]
  int32_t* ov_out;         // [F][C] or null
  int32_t* win_out;        // [F][k]
  uint32_t* ovx;           // [C] tagged overlaps
  uint64_t* dec;           // decision word
  uint32_t* hist;          // [C] winner counts to add to, or null
  uint32_t* mir;           // [C][S] launch scratch: min(idx, N - 1) << 9 | q of each synapse
  Shape sh;
  uint32_t F, step_base, guess;
  uint32_t smagic;         // ceil(2^32 / S), 0 for S = 1: floor(p / S) for p < 2^13
  uint32_t* err;           // the handle's error word, set when the launch gives up
  uint32_t stall;          // 0; a test of the failure path sets 1 (see sp_test_stall)
  uint32_t pad;
};

struct ManyTask {
  uint32_t inst, kind, c0, c1;  // kind 0: tile [c0, c1); kind 1: top-k
};

struct ManyArgs {
  ManyInst* insts;
  const ManyTask* tasks;
  const uint32_t* task_off;  // [grid + 1]: tasks of block b are [task_off[b], task_off[b+1])
  uint32_t* err;             // the launch's error word (0 at launch): every wait gives up once set
  uint32_t Fmax, learn, spin_limit, pad;
};

// Columns of one tile task for S synapses per column.
uint32_t many_tile_columns(uint32_t S);
// Co-resident blocks of the many-instance kernel on `device` (0 on error);
// `aligned`: the kernel for launches whose instances all have S % 64 == 0.
int many_max_blocks(int device, bool aligned);
hipError_t launch_many(const ManyArgs& a, uint32_t grid, bool aligned, hipStream_t s);

}  // namespace htmsp
