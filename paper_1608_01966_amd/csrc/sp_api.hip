// Host side of the C ABI declared in include/sp.h: argument checks, the
// per-handle workspace, the choice between the persistent and the plain
// execution, and kernel launches.  No exception crosses the ABI; every entry
// point returns an sp_status and records a message for sp_last_error().
#include <stdarg.h>
#include <stdio.h>

#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sp.h"
#include "sp_internal.h"

using htmsp::Shape;

struct sp_handle {
  sp_config cfg;
  Shape sh;
  uint32_t* idx;  // borrowed [C][S]
  float* perm;    // borrowed [C][S]
  int device;
  void* ws;
  size_t ws_bytes;
  uint32_t* xchg;      // [replicas][2][exchange entries] of 16 bits
  uint32_t* err;       // [1] (padded)
  uint32_t* check;     // [4]
  uint64_t* racc;      // [2] sums of the radius adaptation (zero between frames)
  int32_t* ov_scratch; // [C]
  uint32_t* many_ovx;  // [C] tagged overlaps of the many-instance step
  uint32_t* hist;      // caller's [C] winner counts, or null
  uint32_t* boost_mem; // [3][C] active duty, overlap duty, boost, then [C] raise flags
  uint32_t boost_C;    // columns the boost state was set up for (0: none yet)
  uint64_t* many_dec;  // decision word of the many-instance step
  uint32_t many_steps; // steps this handle has taken through sp_step_many
  uint64_t frames_seen; // learning frames applied to the state (sp_get_state)
  uint64_t xchg_frames;
  // the frames of persistent steps in pairs (PersistArgs::fpair), grown on
  // use up to htmsp::kPairStageBytes
  uint64_t* fpair;
  uint32_t fpair_pairs;
  bool persistent;
  uint32_t grid, block, replicas;
  const void* pkernel;
  // persistent local-inhibition step: instance (null: per-frame launches),
  // grid, its exchange and the count of exchanges it has used
  const void* lkernel;
  uint32_t lgrid;
  // the two-frames-per-exchange local instance (null: none), its columns per
  // workgroup, its exchange region and the count of exchanges it has used
  const void* lkernel2;
  uint32_t lwgc;
  uint64_t* xloc2;
  uint64_t xloc2_pairs;
  const void* bkernel;  // persistent boosted step (null: per-frame launches)
  uint32_t bgrid;
  // sp_test_stall: the next persistent launch waits for entries that are
  // never written, with this spin limit (0: off)
  uint32_t stall_spins;
  uint64_t* xloc;
  uint64_t xloc_frames;
  bool broken;
  int cus;
  // Every learning step and every re-validation changes the state version;
  // batched inference rebuilds its connected lists when the version moved.
  uint64_t state_version;
  uint32_t* infer_list;      // [S][C]
  uint32_t* infer_cnt;       // [C]
  uint32_t* infer_maxcnt;    // [1]
  uint32_t infer_maxn;
  uint64_t infer_version;    // state version the lists were built for (0: none)
  int32_t* infer_ov;         // [capacity][C] overlaps when the caller wants none
  uint32_t infer_ov_frames;
  // int8 matrix-product inference: bit mask [C][Wm] of the connected
  // synapses plus a duplicate counter, the state version it was built for,
  // the duplicates it found, and the partial sums of the pixel splits
  uint32_t* mfma_mask;
  uint64_t mfma_version;
  uint32_t mfma_dups;
  int32_t* mfma_part;
  size_t mfma_part_elems;
  // Completion of the handle's last enqueued work: `idle` is recorded after
  // every call that enqueues work on the handle (except sp_step_many, whose
  // launches are tracked by their sequence number and staging slot), so
  // sp_destroy waits for that work only, not for the whole device.
  hipEvent_t idle;
  bool idle_used;
  uint64_t many_seq;  // sequence number of its last many-instance launch (0: none)
  int many_slot;      // staging slot that launch used
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return SP_OK;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace layout, each part 256-byte aligned.
struct WsLayout {
  size_t xchg, err, check, racc, ov, many_ovx, many_dec, xloc, xloc2, total;
};

WsLayout ws_layout(const sp_config& c) {
  WsLayout l;
  l.xchg = 0;
  l.err = align_up(l.xchg + sizeof(uint16_t) * 2 * htmsp::kPersistReplicas *
                               htmsp::persistent_exchange_arrays() *
                               (size_t)htmsp::persistent_exchange_entries(c.num_columns),
                   256);
  l.check = align_up(l.err + sizeof(uint32_t), 256);
  l.racc = align_up(l.check + 4 * sizeof(uint32_t), 256);
  l.ov = align_up(l.racc + 2 * sizeof(uint64_t), 256);
  l.many_ovx = align_up(l.ov + sizeof(int32_t) * (size_t)c.num_columns, 256);
  // read in pairs of entries by 256-column words
  l.many_dec = align_up(l.many_ovx + sizeof(uint32_t) * align_up(c.num_columns, 256), 256);
  l.xloc = align_up(l.many_dec + sizeof(uint64_t), 256);
  l.xloc2 = align_up(l.xloc + htmsp::persistent_local_exchange_bytes(c.num_columns), 256);
  l.total = align_up(l.xloc2 + htmsp::persistent_local2_exchange_bytes(c.num_columns), 256);
  return l;
}

int check_config(const sp_config* c) {
  if (!c) return fail(SP_EINVAL, "config is NULL");
  if (c->input_bits < 1 || c->input_bits > SP_MAX_INPUT_BITS)
    return fail(SP_EINVAL, "input_bits=%u outside 1..%u", c->input_bits, SP_MAX_INPUT_BITS);
  if (c->num_columns < 1 || c->num_columns > SP_MAX_COLUMNS)
    return fail(SP_EINVAL, "num_columns=%u outside 1..%u", c->num_columns, SP_MAX_COLUMNS);
  if (c->synapses_per_column < 1 || c->synapses_per_column > SP_MAX_SYNAPSES)
    return fail(SP_EINVAL, "synapses_per_column=%u outside 1..%u", c->synapses_per_column,
                SP_MAX_SYNAPSES);
  if (c->winners < 1 || c->winners > c->num_columns)
    return fail(SP_EINVAL, "winners=%u outside 1..num_columns=%u", c->winners, c->num_columns);
  if (c->connected_q8 > 256) return fail(SP_EINVAL, "connected_q8=%u > 256", c->connected_q8);
  if (c->inc_q8 > 256) return fail(SP_EINVAL, "inc_q8=%u > 256", c->inc_q8);
  if (c->dec_q8 > 256) return fail(SP_EINVAL, "dec_q8=%u > 256", c->dec_q8);
  return SP_OK;
}

Shape make_shape(const sp_config& c) {
  Shape s;
  s.N = c.input_bits;
  s.C = c.num_columns;
  s.S = c.synapses_per_column;
  s.W = (c.input_bits + 31) / 32;
  s.m = c.min_overlap;
  s.k = c.winners;
  s.theta = c.connected_q8;
  s.inc = c.inc_q8;
  s.dec = c.dec_q8;
  return s;
}

bool aligned4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

// Makes the handle's device current for the scope of a call.
struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      if (hipSetDevice(dev) != hipSuccess) prev = -1;
    } else {
      prev = -1;
    }
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int check_handle(const sp_handle* h) {
  if (!h) return fail(SP_EINVAL, "handle is NULL");
  if (h->broken) return fail(SP_EBROKEN, "handle saw a device failure; destroy it");
  return SP_OK;
}

// Records, when a call returns, the completion of whatever it enqueued on
// `s` for the handle (also when it fails part-way, so that sp_destroy still
// waits for the launches that did go out).
struct IdleOnExit {
  sp_handle* h;
  hipStream_t s;
  ~IdleOnExit() {
    if (h && hipEventRecord(h->idle, s) == hipSuccess) h->idle_used = true;
  }
};

// A call that learned on F frames changed the state: batched inference
// rebuilds what it derives from it, and the frame count moves on.
void note_learned(sp_handle* h, uint32_t F, int learn) {
  if (!learn || F == 0) return;
  ++h->state_version;
  h->frames_seen += F;
}

int check_step_args(const sp_handle* h, const uint32_t* frames, uint32_t F, int32_t* ov,
                    int32_t* win) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (F == 0) return SP_OK;
  if (!frames) return fail(SP_EINVAL, "frames is NULL with num_frames=%u", F);
  if (!win) return fail(SP_EINVAL, "winners is NULL");
  if (!aligned4(frames) || !aligned4(win) || (ov && !aligned4(ov)))
    return fail(SP_EINVAL, "frames, overlaps and winners must be 4-byte aligned");
  return SP_OK;
}

// Frames one persistent launch of an F-frame step takes (even unless it is
// the whole step), with the handle's paired-frame buffer grown to hold them.
int pair_stage(sp_handle* h, uint32_t F, uint32_t* frames_per_launch) {
  const size_t row = sizeof(uint64_t) * (size_t)h->sh.W;
  const size_t cap = std::max<size_t>(1, htmsp::kPairStageBytes / row);
  const size_t pairs = (size_t)F / 2 + (F & 1u);
  const size_t need = std::min(cap, pairs);
  if (h->fpair_pairs < need) {
    const size_t want = std::min(cap, std::max(need, 2 * (size_t)h->fpair_pairs));
    if (h->fpair) {
      // (hipFree waits for the device, so no launch still reads the buffer)
      const hipError_t e = hipFree(h->fpair);
      h->fpair = nullptr;
      h->fpair_pairs = 0;
      if (e != hipSuccess) return hip_fail(e, "paired-frame buffer free");
    }
    const hipError_t e = hipMalloc(&h->fpair, row * want);
    if (e != hipSuccess) {
      h->fpair = nullptr;
      return fail(SP_ENOMEM, "paired-frame buffer hipMalloc(%zu): %s", row * want,
                  hipGetErrorString(e));
    }
    h->fpair_pairs = (uint32_t)want;
  }
  *frames_per_launch = (uint32_t)std::min<size_t>(2 * need, F);
  return SP_OK;
}

// The winners of a call added to the handle's histogram, if it has one.
int add_histogram(const sp_handle* h, const int32_t* winners, uint32_t F, hipStream_t s) {
  if (!h->hist || F == 0) return ok();
  hipError_t e = htmsp::launch_hist_add(winners, (size_t)F * h->sh.k, h->sh.C, h->hist, s);
  if (e != hipSuccess) return hip_fail(e, "histogram launch");
  return ok();
}

// The active columns of a local-inhibition call added to the histogram.
int add_histogram_active(const sp_handle* h, const uint8_t* active, uint32_t F, hipStream_t s) {
  if (!h->hist || F == 0) return ok();
  hipError_t e = htmsp::launch_hist_add_active(active, F, h->sh.C, h->hist, s);
  if (e != hipSuccess) return hip_fail(e, "histogram launch");
  return ok();
}

// Spin polls one workgroup makes for one frame before it gives up (several
// seconds; a correct launch needs a tiny fraction of it).
constexpr uint32_t kSpinLimit = 1u << 21;

uint32_t next_pow2(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Chooses the persistent kernel instances of the global, local and boosted
// steps: rows of 64 synapses per column rounded up to a power of two,
// exchange words per lane for C, rows per wave by persistent_wave_rows; the
// grid must be co-resident.  Shapes without an instance run the plain path.
void plan_persistent(sp_handle* h) {
  h->persistent = false;
  h->lkernel = nullptr;
  h->lkernel2 = nullptr;
  h->bkernel = nullptr;
  int dev = h->device, cus = 0, coop = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess) return;
  const Shape& sh = h->sh;
  if (!coop || cus <= 0 || sh.C > htmsp::kPersistMaxColumns ||
      sh.S > htmsp::kPersistMaxSynapses)
    return;
  const uint32_t rpc = next_pow2((sh.S + 63) / 64);
  const uint32_t nv = next_pow2(htmsp::persistent_exchange_entries(sh.C) / 256);
  // The column-group-per-wave split shared by the global, local and boosted
  // steps (each needs an instance for it, and a co-resident grid).
  uint32_t wgrid = 0;
  const uint32_t rw = htmsp::persistent_wave_rows(sh.C, rpc, cus, &wgrid);
  auto fits = [&](const void* k) {
    int per_cu = 0;
    return k && hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, htmsp::kPersistWaves * 64,
                                                             0) == hipSuccess &&
           per_cu >= 1;
  };
  // The boosted step: every wave holds every column's duty cycles
  // (C <= kBoostPersistMaxColumns).
  if (rw && sh.C <= htmsp::kBoostPersistMaxColumns) {
    const void* kb = htmsp::persistent_boost_kernel(rpc, nv, rw);
    if (fits(kb)) {
      h->bkernel = kb;
      h->bgrid = wgrid;
    }
  }
  // The local-inhibition step.
  if (rw) {
    const void* kl = htmsp::persistent_local_kernel(rpc, nv, rw);
    if (fits(kl)) {
      h->lkernel = kl;
      h->lgrid = wgrid;
      const void* kl2 = htmsp::persistent_local2_kernel(rpc, nv, rw);
      if (fits(kl2)) {
        h->lkernel2 = kl2;
        h->lwgc = htmsp::kPersistWaves * (rw / rpc);
      }
    }
  }
  // The global step.
  if (rw) {
    const void* kw = htmsp::persistent_wave_kernel(rpc, nv, rw);
    if (fits(kw)) {
      h->grid = wgrid;
      h->block = htmsp::kPersistWaves * 64;
      h->replicas = htmsp::kPersistReplicas;
      h->pkernel = kw;
      h->persistent = true;
    }
  }
}

int run_check_state(sp_handle* h, hipStream_t s) {
  const size_t n = (size_t)h->sh.C * h->sh.S;
  hipError_t e = htmsp::launch_check_state(h->idx, h->perm, n, h->sh.N, h->check, s);
  if (e != hipSuccess) return hip_fail(e, "state check launch");
  uint32_t out[4];
  e = hipMemcpyAsync(out, h->check, sizeof(out), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "state check");
  if (out[0])
    return fail(SP_EINVAL, "%u synapse indices >= input_bits=%u (first at flat position %u)",
                out[0], h->sh.N, out[2]);
  if (out[1])
    return fail(SP_EINVAL,
                "%u permanences off the 1/256 grid or outside [0,1] (first at flat position %u)",
                out[1], out[3]);
  return SP_OK;
}

// Descriptor staging for sp_step_many: two slots of pinned host memory and
// device memory per device, so that a call only waits for the launch two
// calls back before it rewrites a slot.
struct ManySlot {
  void* host = nullptr;
  void* dev = nullptr;
  size_t cap = 0;
  // the launch's packed copy of its instances' synapses (device scratch)
  void* mir = nullptr;
  size_t mir_cap = 0;
  hipEvent_t done = nullptr;
};

struct ManyCtx {
  int device = -1;
  ManySlot slot[2];
  int next = 0;
  // launches enqueued so far; launch n reuses the slot of launch n - 2 only
  // after that launch's completion event, so every launch numbered at most
  // seq - 2 is known to be complete
  uint64_t seq = 0;
};

std::mutex g_many_mu;
ManyCtx g_many[16];

int many_slot(int device, size_t bytes, size_t mir_bytes, ManySlot** out, int* index) {
  if (device < 0 || device >= 16) return fail(SP_EDEVICE, "device %d out of range", device);
  ManyCtx& ctx = g_many[device];
  ctx.device = device;
  *index = ctx.next;
  ManySlot& sl = ctx.slot[ctx.next];
  ctx.next ^= 1;
  hipError_t e = hipSuccess;
  if (sl.done) {
    e = hipEventSynchronize(sl.done);
    if (e != hipSuccess) return hip_fail(e, "many-instance staging");
  } else {
    e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "many-instance event");
  }
  if (sl.cap < bytes) {
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.dev) (void)hipFree(sl.dev);
    sl.host = sl.dev = nullptr;
    sl.cap = 0;
    const size_t cap = std::max<size_t>(bytes, 1 << 16) * 2;
    e = hipHostMalloc(&sl.host, cap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&sl.dev, cap);
    if (e != hipSuccess) {
      if (sl.host) (void)hipHostFree(sl.host);
      sl.host = sl.dev = nullptr;
      return fail(SP_ENOMEM, "many-instance staging allocation (%zu bytes)", cap);
    }
    sl.cap = cap;
  }
  if (sl.mir_cap < mir_bytes) {
    if (sl.mir) (void)hipFree(sl.mir);
    sl.mir = nullptr;
    sl.mir_cap = 0;
    const size_t cap = mir_bytes + mir_bytes / 4;
    e = hipMalloc(&sl.mir, cap);
    if (e != hipSuccess) {
      sl.mir = nullptr;
      return fail(SP_ENOMEM, "many-instance packed state allocation (%zu bytes)", cap);
    }
    sl.mir_cap = cap;
  }
  *out = &sl;
  return SP_OK;
}

// Waits for the handle's last many-instance launch, unless the library has
// already waited for it (two launches later, when its staging slot was
// reused).
hipError_t many_wait(const sp_handle* h) {
  if (!h->many_seq || h->device < 0 || h->device >= 16) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_many_mu);
  const ManyCtx& ctx = g_many[h->device];
  if (h->many_seq + 2 <= ctx.seq) return hipSuccess;
  return hipEventSynchronize(ctx.slot[h->many_slot].done);
}

// Workspaces of destroyed handles, per device, for later sp_create calls: a
// handle's workspace goes back here instead of to hipFree, which would wait
// for every stream of the device (a serving loop that retires a stream must
// not drain the batches in flight).  Pooled buffers are idle (sp_destroy
// waited for their handle's work) and are cleared again on reuse; the pool
// keeps at most kWsPoolMax bytes per device until the process ends.
constexpr size_t kWsPoolMax = size_t(256) << 20;

struct WsPool {
  std::vector<std::pair<size_t, void*>> free;
  size_t bytes = 0;
};

std::mutex g_ws_mu;
WsPool g_ws[16];

// A pooled workspace of at least `bytes` (at most twice that), or null.
void* ws_take(int device, size_t bytes, size_t* got) {
  if (device < 0 || device >= 16) return nullptr;
  std::lock_guard<std::mutex> lock(g_ws_mu);
  WsPool& p = g_ws[device];
  size_t best = p.free.size();
  for (size_t i = 0; i < p.free.size(); ++i)
    if (p.free[i].first >= bytes && p.free[i].first <= 2 * bytes &&
        (best == p.free.size() || p.free[i].first < p.free[best].first))
      best = i;
  if (best == p.free.size()) return nullptr;
  void* ws = p.free[best].second;
  *got = p.free[best].first;
  p.bytes -= *got;
  p.free.erase(p.free.begin() + (ptrdiff_t)best);
  return ws;
}

// Returns an idle workspace to the pool; false if the pool is full (the
// caller frees it).
bool ws_give(int device, void* ws, size_t bytes) {
  if (device < 0 || device >= 16) return false;
  std::lock_guard<std::mutex> lock(g_ws_mu);
  WsPool& p = g_ws[device];
  if (p.bytes + bytes > kWsPoolMax) return false;
  p.free.emplace_back(bytes, ws);
  p.bytes += bytes;
  return true;
}

// One cooperative launch over hs[0..n) (instances with frames; the caller
// holds g_many_mu).  The first workgroups hold tile tasks only, dealt
// round-robin, at most kMaxTileSlots each; the last many_topk_blocks()
// hold the top-k tasks only, also round-robin.
int many_launch(sp_handle* const* hs, uint32_t n, const uint32_t* const* frames_dev,
                const uint32_t* num_frames, int learn, int32_t* const* overlaps_dev,
                int32_t* const* winners_dev, hipStream_t s, int dev, int maxb, bool aligned,
                size_t ntiles, uint32_t nact, uint32_t Fmax) {
  const uint32_t ntasks = (uint32_t)(ntiles + nact);
  const uint32_t kblocks = htmsp::many_topk_blocks(nact, (size_t)maxb);
  const uint32_t tblocks = (uint32_t)std::min<size_t>(ntiles, (size_t)maxb - kblocks);
  const uint32_t grid = tblocks + kblocks;
  // tiles in instance order; tile j goes to workgroup j % tblocks, the top-k
  // task of instance i to workgroup tblocks + i % kblocks
  thread_local std::vector<htmsp::ManyTask> tiles;
  thread_local std::vector<htmsp::ManyInst> insts;
  tiles.clear();
  insts.clear();
  tiles.reserve(ntiles);
  insts.reserve(nact);
  uint32_t spin_limit = kSpinLimit;
  thread_local std::vector<size_t> mir_off;
  mir_off.clear();
  size_t mir_bytes = 0;
  for (uint32_t i = 0; i < n; ++i) {
    sp_handle* h = hs[i];
    if (num_frames[i] == 0) continue;
    mir_off.push_back(mir_bytes);
    mir_bytes = align_up(mir_bytes + sizeof(uint32_t) * (size_t)h->sh.C * h->sh.S, 256);
    const uint32_t id = (uint32_t)insts.size();
    htmsp::ManyInst in = {};
    in.idx = h->idx;
    in.perm = h->perm;
    in.frames = frames_dev[i];
    in.ov_out = overlaps_dev ? overlaps_dev[i] : nullptr;
    in.win_out = winners_dev[i];
    in.ovx = h->many_ovx;
    in.dec = h->many_dec;
    in.hist = h->hist;
    in.sh = h->sh;
    in.F = num_frames[i];
    in.step_base = h->many_steps;
    in.guess = 1 + h->sh.S / 16;
    in.smagic = h->sh.S == 1 ? 0u : (uint32_t)(((1ull << 32) + h->sh.S - 1) / h->sh.S);
    in.err = h->err;
    if (h->stall_spins) {
      in.stall = 1;
      spin_limit = std::min(spin_limit, h->stall_spins);
    }
    insts.push_back(in);
    const uint32_t ct = htmsp::many_tile_columns(h->sh.S);
    for (uint32_t c0 = 0; c0 < h->sh.C; c0 += ct)
      tiles.push_back({id, 0u, c0, std::min(h->sh.C, c0 + ct)});
  }

  // staging layout: the launch's error word (cleared by the upload), the
  // instance descriptors, the tasks, the per-workgroup task offsets
  const size_t b_err = 256;
  const size_t b_insts = align_up(sizeof(htmsp::ManyInst) * insts.size(), 256);
  const size_t b_tasks = align_up(sizeof(htmsp::ManyTask) * ntasks, 256);
  const size_t b_off = sizeof(uint32_t) * (grid + 1);
  ManySlot* sl = nullptr;
  int slot_index = 0;
  int rc = many_slot(dev, b_err + b_insts + b_tasks + b_off, mir_bytes, &sl, &slot_index);
  if (rc) return rc;
  for (size_t i = 0; i < insts.size(); ++i)
    insts[i].mir = reinterpret_cast<uint32_t*>(static_cast<char*>(sl->mir) + mir_off[i]);
  char* hb = static_cast<char*>(sl->host);
  char* db = static_cast<char*>(sl->dev);
  memset(hb, 0, b_err);
  hb += b_err;
  memcpy(hb, insts.data(), sizeof(htmsp::ManyInst) * insts.size());
  htmsp::ManyTask* ht = reinterpret_cast<htmsp::ManyTask*>(hb + b_insts);
  uint32_t* hoff = reinterpret_cast<uint32_t*>(hb + b_insts + b_tasks);
  uint32_t k = 0;
  for (uint32_t b = 0; b < tblocks; ++b) {
    hoff[b] = k;
    for (size_t j = b; j < tiles.size(); j += tblocks) ht[k++] = tiles[j];
  }
  for (uint32_t b = 0; b < kblocks; ++b) {
    hoff[tblocks + b] = k;
    for (uint32_t id = b; id < insts.size(); id += kblocks) ht[k++] = {id, 1u, 0u, 0u};
  }
  hoff[grid] = k;
  hipError_t e = hipMemcpyAsync(db, hb - b_err, b_err + b_insts + b_tasks + b_off,
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "many-instance descriptors");
  htmsp::ManyArgs a = {};
  a.err = reinterpret_cast<uint32_t*>(db);
  db += b_err;
  a.insts = reinterpret_cast<htmsp::ManyInst*>(db);
  a.tasks = reinterpret_cast<const htmsp::ManyTask*>(db + b_insts);
  a.task_off = reinterpret_cast<const uint32_t*>(db + b_insts + b_tasks);
  a.Fmax = Fmax;
  a.learn = learn ? 1u : 0u;
  a.spin_limit = spin_limit;
  e = htmsp::launch_many(a, grid, aligned, s);
  if (e == hipSuccess) e = hipEventRecord(sl->done, s);
  if (e != hipSuccess) return hip_fail(e, "many-instance launch");
  // the launch is enqueued: every instance it holds has moved on
  const uint64_t seq = ++g_many[dev].seq;
  for (uint32_t i = 0; i < n; ++i) {
    if (num_frames[i] == 0) continue;
    hs[i]->many_steps += num_frames[i];
    hs[i]->stall_spins = 0;
    hs[i]->many_seq = seq;
    hs[i]->many_slot = slot_index;
    note_learned(hs[i], num_frames[i], learn);
  }
  return SP_OK;
}

}  // namespace

extern "C" {

int sp_config_check(const sp_config* cfg) {
  int rc = check_config(cfg);
  return rc ? rc : ok();
}

size_t sp_frame_words(const sp_config* cfg) {
  if (check_config(cfg)) return 0;
  return ((size_t)cfg->input_bits + 31) / 32;
}

size_t sp_workspace_bytes(const sp_config* cfg) {
  if (check_config(cfg)) return 0;
  return ws_layout(*cfg).total;
}

int sp_check_state_host(const sp_config* cfg, const uint32_t* idx, const float* perm) {
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!idx || !perm) return fail(SP_EINVAL, "idx or perm is NULL");
  const size_t n = (size_t)cfg->num_columns * cfg->synapses_per_column;
  for (size_t i = 0; i < n; ++i) {
    if (idx[i] >= cfg->input_bits)
      return fail(SP_EINVAL, "idx[%zu]=%u >= input_bits=%u", i, idx[i], cfg->input_bits);
    const float q = perm[i] * 256.0f;
    if (!(q >= 0.0f && q <= 256.0f && q == (float)(int)q))
      return fail(SP_EINVAL, "perm[%zu]=%.9g is off the 1/256 grid or outside [0,1]", i,
                  (double)perm[i]);
  }
  return ok();
}

int sp_create(const sp_config* cfg, uint32_t* idx_dev, float* perm_dev, void* stream,
              sp_handle** out) {
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!out) return fail(SP_EINVAL, "out is NULL");
  if (!idx_dev || !perm_dev) return fail(SP_EINVAL, "idx or perm is NULL");
  if (!aligned4(idx_dev) || !aligned4(perm_dev))
    return fail(SP_EINVAL, "idx and perm must be 4-byte aligned");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);

  sp_handle* h = new (std::nothrow) sp_handle();
  if (!h) return fail(SP_ENOMEM, "host allocation failed");
  h->cfg = *cfg;
  h->sh = make_shape(*cfg);
  h->idx = idx_dev;
  h->perm = perm_dev;
  h->device = dev;
  const WsLayout l = ws_layout(*cfg);
  h->ws_bytes = l.total;
  h->ws = ws_take(dev, l.total, &h->ws_bytes);
  if (!h->ws) {
    h->ws_bytes = l.total;
    e = hipMalloc(&h->ws, l.total);
    if (e != hipSuccess) {
      delete h;
      return fail(SP_ENOMEM, "workspace hipMalloc(%zu): %s", l.total, hipGetErrorString(e));
    }
  }
  e = hipEventCreateWithFlags(&h->idle, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (!ws_give(dev, h->ws, h->ws_bytes)) (void)hipFree(h->ws);
    delete h;
    return hip_fail(e, "completion event");
  }
  char* base = static_cast<char*>(h->ws);
  h->xchg = reinterpret_cast<uint32_t*>(base + l.xchg);
  h->err = reinterpret_cast<uint32_t*>(base + l.err);
  h->check = reinterpret_cast<uint32_t*>(base + l.check);
  h->racc = reinterpret_cast<uint64_t*>(base + l.racc);
  h->ov_scratch = reinterpret_cast<int32_t*>(base + l.ov);
  h->many_ovx = reinterpret_cast<uint32_t*>(base + l.many_ovx);
  h->many_dec = reinterpret_cast<uint64_t*>(base + l.many_dec);
  h->xloc = reinterpret_cast<uint64_t*>(base + l.xloc);
  h->xloc2 = reinterpret_cast<uint64_t*>(base + l.xloc2);
  // (run_check_state synchronises `s`, so the workspace is clear and idle
  // when it goes back to the pool on a failure)
  e = hipMemsetAsync(h->ws, 0, h->ws_bytes, s);
  rc = e != hipSuccess ? hip_fail(e, "workspace clear") : run_check_state(h, s);
  if (rc) {
    if (e != hipSuccess || !ws_give(dev, h->ws, h->ws_bytes)) (void)hipFree(h->ws);
    (void)hipEventDestroy(h->idle);
    delete h;
    return rc;
  }
  (void)hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (h->cus <= 0) h->cus = 1;
  h->state_version = 1;
  plan_persistent(h);
  *out = h;
  return ok();
}

int sp_check_state(sp_handle* h, void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  DeviceScope ds(h->device);
  rc = run_check_state(h, static_cast<hipStream_t>(stream));
  ++h->state_version;
  return rc ? rc : ok();
}

int sp_step_plain(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames, int learn,
                  int32_t* overlaps_dev, int32_t* winners_dev, void* stream) {
  int rc = check_step_args(h, frames_dev, num_frames, overlaps_dev, winners_dev);
  if (rc) return rc;
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  IdleOnExit idle{h, s};
  const Shape& sh = h->sh;
  note_learned(h, num_frames, learn);
  for (uint32_t t = 0; t < num_frames; ++t) {
    const uint32_t* frame = frames_dev + (size_t)t * sh.W;
    int32_t* ov = overlaps_dev ? overlaps_dev + (size_t)t * sh.C : h->ov_scratch;
    int32_t* win = winners_dev + (size_t)t * sh.k;
    hipError_t e = htmsp::launch_overlap_plain(h->idx, h->perm, frame, ov, sh, s);
    if (e == hipSuccess) e = htmsp::launch_topk_plain(ov, win, sh, s);
    if (e == hipSuccess && learn) e = htmsp::launch_learn_plain(h->idx, h->perm, frame, win, sh, s);
    if (e != hipSuccess) return hip_fail(e, "plain step launch");
  }
  return add_histogram(h, winners_dev, num_frames, s);
}

int sp_step(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames, int learn,
            int32_t* overlaps_dev, int32_t* winners_dev, void* stream) {
  int rc = check_step_args(h, frames_dev, num_frames, overlaps_dev, winners_dev);
  if (rc) return rc;
  if (num_frames == 0) return ok();
  if (!h->persistent)
    return sp_step_plain(h, frames_dev, num_frames, learn, overlaps_dev, winners_dev, stream);
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  IdleOnExit idle{h, s};
  uint32_t chunk = 0;
  rc = pair_stage(h, num_frames, &chunk);
  if (rc) return rc;
  const Shape& sh = h->sh;
  htmsp::PersistArgs a;
  a.idx = h->idx;
  a.perm = h->perm;
  a.fpair = h->fpair;
  a.xchg = h->xchg;
  a.err = h->err;
  a.learn = learn ? 1u : 0u;
  a.replicas = h->replicas;
  a.sh = sh;
  void* args[] = {&a};
  // Launches of at most `chunk` frames, each after pairing its frames; the
  // state goes back to idx/perm between them, so the results are those of
  // one launch.
  for (uint64_t t0 = 0; t0 < num_frames; t0 += chunk) {
    const uint32_t F = (uint32_t)std::min<uint64_t>(chunk, num_frames - t0);
    hipError_t e = htmsp::launch_pair_frames(frames_dev + t0 * sh.W, F, sh.W, h->fpair, s);
    if (e != hipSuccess) {
      note_learned(h, (uint32_t)t0, learn);
      return hip_fail(e, "frame pairing launch");
    }
    a.ov_out = overlaps_dev ? overlaps_dev + t0 * sh.C : nullptr;
    a.win_out = winners_dev + t0 * sh.k;
    a.F = F;
    a.frame_base = (uint32_t)h->xchg_frames;
    a.spin_limit = h->stall_spins ? h->stall_spins : kSpinLimit;
    a.stall = h->stall_spins ? 1u : 0u;
    h->stall_spins = 0;
    e = hipLaunchCooperativeKernel(h->pkernel, dim3(h->grid), dim3(h->block), args, 0, s);
    if (e != hipSuccess) {
      note_learned(h, (uint32_t)t0, learn);
      return hip_fail(e, "persistent step launch");
    }
    h->xchg_frames += F / 2 + (F & 1u);
  }
  note_learned(h, num_frames, learn);
  return add_histogram(h, winners_dev, num_frames, s);
}

}  // extern "C"

namespace {

// The [F][C] overlap buffer sp_infer uses when the caller passes none.
int infer_ov_scratch(sp_handle* h, uint32_t F, int32_t** out) {
  if (h->infer_ov_frames < F) {
    if (h->infer_ov) {
      hipError_t e = hipFree(h->infer_ov);
      h->infer_ov = nullptr;
      h->infer_ov_frames = 0;
      if (e != hipSuccess) return hip_fail(e, "inference scratch free");
    }
    const size_t bytes = sizeof(int32_t) * (size_t)F * h->sh.C;
    hipError_t e = hipMalloc(&h->infer_ov, bytes);
    if (e != hipSuccess) {
      h->infer_ov = nullptr;
      return fail(SP_ENOMEM, "inference scratch hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    h->infer_ov_frames = F;
  }
  *out = h->infer_ov;
  return SP_OK;
}

// Winners of F frames from their gated overlaps, and the histogram.
int infer_topk(sp_handle* h, const int32_t* ov, uint32_t F, int32_t* winners, hipStream_t s) {
  hipError_t e;
  if (h->sh.C <= htmsp::kPersistMaxColumns)
    e = htmsp::launch_topk_batch(ov, F, h->sh, winners, s);
  else
    e = htmsp::launch_topk_plain(ov, winners, h->sh, s, F);
  if (e != hipSuccess) return hip_fail(e, "inference top-k launch");
  return add_histogram(h, winners, F, s);
}

int infer_gather(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames,
                 int32_t* overlaps_dev, int32_t* winners_dev, hipStream_t s) {
  const Shape& sh = h->sh;
  hipError_t e = hipSuccess;
  if (!h->infer_list) {
    const size_t bytes = sizeof(uint32_t) * ((size_t)sh.S * sh.C + sh.C + 64);
    e = hipMalloc(&h->infer_list, bytes);
    if (e != hipSuccess) {
      h->infer_list = nullptr;
      return fail(SP_ENOMEM, "inference lists hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    h->infer_cnt = h->infer_list + (size_t)sh.S * sh.C;
    h->infer_maxcnt = h->infer_cnt + sh.C;
  }
  if (h->infer_version != h->state_version) {
    e = htmsp::launch_infer_prep(h->idx, h->perm, sh, h->infer_list, h->infer_cnt,
                                 h->infer_maxcnt, s);
    uint32_t maxn = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&maxn, h->infer_maxcnt, sizeof(maxn),
                                            hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "inference prep");
    h->infer_maxn = maxn;
    h->infer_version = h->state_version;
  }
  int32_t* ov = overlaps_dev;
  if (!ov) {
    int rc = infer_ov_scratch(h, num_frames, &ov);
    if (rc) return rc;
  }
  e = htmsp::launch_infer_gather(h->infer_maxn, frames_dev, num_frames, h->infer_list,
                                 h->infer_cnt, sh, ov, (uint32_t)h->cus, s);
  if (e != hipSuccess) return hip_fail(e, "inference gather launch");
  return infer_topk(h, ov, num_frames, winners_dev, s);
}

// Largest bit mask the matrix-product inference builds (C * Wm words).
constexpr size_t kMfmaMaskMaxBytes = size_t(1) << 32;

int infer_mfma(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames,
               int32_t* overlaps_dev, int32_t* winners_dev, hipStream_t s) {
  const Shape& sh = h->sh;
  const size_t Wm = htmsp::mfma_mask_words(sh.W);
  const size_t mask_bytes = sizeof(uint32_t) * Wm * sh.C;
  if (mask_bytes > kMfmaMaskMaxBytes)
    return fail(SP_EINVAL,
                "the connected mask of %u columns x %u words exceeds %zu bytes; use the gather mode",
                sh.C, (unsigned)Wm, kMfmaMaskMaxBytes);
  hipError_t e = hipSuccess;
  if (!h->mfma_mask) {
    e = hipMalloc(&h->mfma_mask, mask_bytes + 256);
    if (e != hipSuccess) {
      h->mfma_mask = nullptr;
      return fail(SP_ENOMEM, "connected mask hipMalloc(%zu): %s", mask_bytes + 256,
                  hipGetErrorString(e));
    }
  }
  uint32_t* dup = h->mfma_mask + Wm * sh.C;
  if (h->mfma_version != h->state_version) {
    e = htmsp::launch_mfma_mask(h->idx, h->perm, sh, h->mfma_mask, dup, s);
    uint32_t dups = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&dups, dup, sizeof(dups), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "connected mask");
    h->mfma_dups = dups;
    h->mfma_version = h->state_version;
  }
  if (h->mfma_dups)
    return fail(SP_EINVAL,
                "%u connected synapses repeat a pixel of their column; the 0/1 mask of the "
                "matrix-product mode cannot count them (use the gather mode)",
                h->mfma_dups);
  int32_t* ov = overlaps_dev;
  if (!ov) {
    int rc = infer_ov_scratch(h, num_frames, &ov);
    if (rc) return rc;
  }
  // frame chunks whose word offsets stay below 2^31
  const uint32_t fmax = (uint32_t)std::min<size_t>(num_frames, ((size_t)1 << 31) / sh.W - 1);
  for (uint32_t f0 = 0; f0 < num_frames; f0 += fmax) {
    const uint32_t F = std::min(fmax, num_frames - f0);
    const uint32_t splits = htmsp::mfma_splits(sh, F, (uint32_t)h->cus);
    const size_t need = splits > 1 ? (size_t)splits * F * sh.C : 0;
    if (need > h->mfma_part_elems) {
      if (h->mfma_part) {
        e = hipFree(h->mfma_part);
        h->mfma_part = nullptr;
        h->mfma_part_elems = 0;
        if (e != hipSuccess) return hip_fail(e, "partial sums free");
      }
      e = hipMalloc(&h->mfma_part, sizeof(int32_t) * need);
      if (e != hipSuccess) {
        h->mfma_part = nullptr;
        return fail(SP_ENOMEM, "partial sums hipMalloc(%zu): %s", sizeof(int32_t) * need,
                    hipGetErrorString(e));
      }
      h->mfma_part_elems = need;
    }
    e = htmsp::launch_infer_mfma(frames_dev + (size_t)f0 * sh.W, F, h->mfma_mask, sh, splits,
                                 h->mfma_part, ov + (size_t)f0 * sh.C, s);
    if (e != hipSuccess) return hip_fail(e, "matrix-product inference launch");
  }
  return infer_topk(h, ov, num_frames, winners_dev, s);
}

}  // namespace

extern "C" {

int sp_infer(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames, int mode,
             int32_t* overlaps_dev, int32_t* winners_dev, void* stream) {
  int rc = check_step_args(h, frames_dev, num_frames, overlaps_dev, winners_dev);
  if (rc) return rc;
  if (mode != SP_INFER_GATHER && mode != SP_INFER_MFMA_I8)
    return fail(SP_EINVAL, "unknown inference mode %d", mode);
  if (num_frames == 0) return ok();
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  IdleOnExit idle{h, s};
  rc = mode == SP_INFER_GATHER
           ? infer_gather(h, frames_dev, num_frames, overlaps_dev, winners_dev, s)
           : infer_mfma(h, frames_dev, num_frames, overlaps_dev, winners_dev, s);
  return rc ? rc : ok();
}

}  // extern "C"

namespace {

// Scratch of sp_infer_noalloc: the compacted connected lists (slot-major
// [S][C], then counts [C]) of the handle being served.  Each GPU the library
// runs on holds its own copy for the life of the process; host code uses
// only the address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
__device__ __align__(256) uint32_t scratch[kNoAllocScratchBytes / sizeof(uint32_t)];

std::mutex g_scratch_mu;
uint32_t* g_scratch[16];

// The device address of this device's scratch, looked up once per device.
int noalloc_scratch(int device, uint32_t** out) {
  if (device < 0 || device >= 16) return fail(SP_EDEVICE, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "scratch address");
    if (!ptr) return fail(SP_EDEVICE, "scratch address is NULL");
    g_scratch[device] = static_cast<uint32_t*>(ptr);
  }
  *out = g_scratch[device];
  return SP_OK;
}

}  // namespace

extern "C" {

size_t sp_infer_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int sp_infer_noalloc(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames,
                     int32_t* overlaps_dev, int32_t* winners_dev, void* stream) {
  int rc = check_step_args(h, frames_dev, num_frames, overlaps_dev, winners_dev);
  if (rc) return rc;
  if (num_frames && !overlaps_dev) return fail(SP_EINVAL, "overlaps is NULL");
  const Shape& sh = h->sh;
  if (sh.S > htmsp::infer_max_list())
    return fail(SP_EINVAL, "synapses_per_column=%u > %u: a list could outgrow the gather registers",
                sh.S, htmsp::infer_max_list());
  const size_t need = sizeof(uint32_t) * ((size_t)sh.S * sh.C + sh.C);
  if (need > kNoAllocScratchBytes)
    return fail(SP_EINVAL, "the lists need %zu bytes; the scratch holds %zu", need,
                kNoAllocScratchBytes);
  if (num_frames == 0) return ok();
  DeviceScope ds(h->device);
  uint32_t* list = nullptr;
  rc = noalloc_scratch(h->device, &list);
  if (rc) return rc;
  uint32_t* cnt = list + (size_t)sh.S * sh.C;
  hipStream_t s = static_cast<hipStream_t>(stream);
  IdleOnExit idle{h, s};
  // every slot and count is rewritten, so nothing has to start at zero
  hipError_t e = htmsp::launch_infer_prep(h->idx, h->perm, sh, list, cnt, nullptr, s);
  if (e == hipSuccess)
    e = htmsp::launch_infer_gather(sh.S, frames_dev, num_frames, list, cnt, sh, overlaps_dev,
                                   (uint32_t)h->cus, s);
  if (e != hipSuccess) return hip_fail(e, "inference launch");
  rc = infer_topk(h, overlaps_dev, num_frames, winners_dev, s);
  return rc ? rc : ok();
}

int sp_step_many(sp_handle* const* hs, uint32_t n, const uint32_t* const* frames_dev,
                 const uint32_t* num_frames, int learn, int32_t* const* overlaps_dev,
                 int32_t* const* winners_dev, void* stream) {
  if (n == 0) return ok();
  if (!hs || !frames_dev || !num_frames || !winners_dev)
    return fail(SP_EINVAL, "handles, frames, num_frames and winners arrays are required");
  int dev = -1;
  size_t nact = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const sp_handle* h = hs[i];
    int rc = check_step_args(h, frames_dev[i], num_frames[i],
                             overlaps_dev ? overlaps_dev[i] : nullptr, winners_dev[i]);
    if (rc) return fail(rc, "instance %u: %s", i, g_err.c_str());
    if (dev < 0) dev = h->device;
    if (h->device != dev) return fail(SP_EINVAL, "instance %u is on another device", i);
    if (h->sh.C > 4 * 64 * htmsp::kManyNV)
      return fail(SP_EINVAL, "instance %u has %u columns; stepping many instances holds at most %u",
                  i, h->sh.C, 4 * 64 * htmsp::kManyNV);
    for (uint32_t j = 0; j < i; ++j)
      if (hs[j] == h) return fail(SP_EINVAL, "instance %u repeats instance %u", i, j);
    if (num_frames[i] == 0) continue;
    ++nact;
  }
  if (nact == 0) return ok();
  DeviceScope ds(dev);
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool aligned = true;
  for (uint32_t i = 0; i < n; ++i) aligned = aligned && hs[i]->sh.S % 64 == 0;
  const int maxb = htmsp::many_max_blocks(dev, aligned);
  if (maxb <= 0) return fail(SP_EDEVICE, "cannot size the many-instance launch");
  // Instances are independent, so they may be split over consecutive
  // launches: each launch holds at most kMaxTileSlots tiles per workgroup,
  // next to one top-k workgroup per kMaxTopkSlots instances.
  if (maxb < 2) return fail(SP_EDEVICE, "the many-instance kernel needs two co-resident workgroups");
  const size_t cap = (size_t)htmsp::kMaxTileSlots * (size_t)(maxb - 1);
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t ct = htmsp::many_tile_columns(hs[i]->sh.S);
    const size_t nt = (hs[i]->sh.C + ct - 1) / ct;
    if (num_frames[i] != 0 && nt > cap)
      return fail(SP_EINVAL, "instance %u needs %zu tiles; one launch holds %zu on this device", i,
                  nt, cap);
  }
  std::lock_guard<std::mutex> lock(g_many_mu);
  uint32_t i0 = 0;
  while (i0 < n) {
    uint32_t i1 = i0, nact_c = 0;
    size_t tiles_c = 0;
    uint32_t Fmax_c = 0;
    for (; i1 < n; ++i1) {
      if (num_frames[i1] == 0) continue;
      const uint32_t ct = htmsp::many_tile_columns(hs[i1]->sh.S);
      const size_t nt = (hs[i1]->sh.C + ct - 1) / ct;
      // room for the tiles next to the top-k workgroups the instances need
      const size_t kb = htmsp::many_topk_blocks(nact_c + 1, (size_t)maxb);
      if (nact_c > 0 &&
          (kb >= (size_t)maxb || tiles_c + nt > htmsp::kMaxTileSlots * ((size_t)maxb - kb)))
        break;
      tiles_c += nt;
      ++nact_c;
      Fmax_c = std::max(Fmax_c, num_frames[i1]);
    }
    if (nact_c > 0) {
      int rc = many_launch(hs + i0, i1 - i0, frames_dev + i0, num_frames + i0, learn,
                           overlaps_dev ? overlaps_dev + i0 : nullptr, winners_dev + i0, s, dev,
                           maxb, aligned, tiles_c, nact_c, Fmax_c);
      if (rc) {
        // the instances of this and later launches were not stepped; those of
        // earlier launches were (their counters have moved on)
        for (uint32_t i = i0; i < n; ++i)
          if (num_frames[i]) hs[i]->broken = true;
        return rc;
      }
    }
    i0 = i1;
  }
  return ok();
}

}  // extern "C"

namespace {

int encoder_shape(const sp_encoder_config* c, htmsp::EncShape* e) {
  if (!c) return fail(SP_EINVAL, "encoder config is NULL");
  if (c->factor < 1 || c->factor > 32) return fail(SP_EINVAL, "factor=%u outside 1..32", c->factor);
  if (c->block < 3 || c->block > 11 || c->block % 2 == 0)
    return fail(SP_EINVAL, "block=%u must be odd in 3..11", c->block);
  if (c->offset < -255 || c->offset > 255)
    return fail(SP_EINVAL, "offset=%d outside -255..255", c->offset);
  const uint32_t w = c->width / c->factor, h = c->height / c->factor;
  if (w < 1 || h < 1) return fail(SP_EINVAL, "frame smaller than the reduction factor");
  if (w > 4096) return fail(SP_EINVAL, "encoded width %u > 4096", w);
  if ((uint64_t)w * h > SP_MAX_INPUT_BITS)
    return fail(SP_EINVAL, "encoded frame has %llu bits > %u", (unsigned long long)w * h,
                SP_MAX_INPUT_BITS);
  e->W = c->width;
  e->H = c->height;
  e->factor = c->factor;
  e->block = c->block;
  e->offset = c->offset;
  e->w = w;
  e->h = h;
  e->words = (uint32_t)(((uint64_t)w * h + 31) / 32);
  e->area = c->factor * c->factor;
  e->area_magic = (uint32_t)(((1ull << 32) + e->area - 1) / e->area);
  return SP_OK;
}

}  // namespace

extern "C" {

int sp_inhibit_local(const int32_t* overlaps_dev, uint32_t num_frames, uint32_t num_columns,
                     uint32_t grid_w, uint32_t radius, uint32_t n, uint8_t* active_dev,
                     void* stream) {
  if (num_columns < 1 || num_columns > SP_MAX_COLUMNS)
    return fail(SP_EINVAL, "num_columns=%u outside 1..%u", num_columns, SP_MAX_COLUMNS);
  if (grid_w < 1 || grid_w > num_columns)
    return fail(SP_EINVAL, "grid_w=%u outside 1..num_columns", grid_w);
  if (n < 1) return fail(SP_EINVAL, "n must be >= 1");
  if (num_frames == 0) return ok();
  if (!overlaps_dev || !active_dev || !aligned4(overlaps_dev))
    return fail(SP_EINVAL, "overlaps (4-byte aligned) and active are required");
  hipError_t e = htmsp::launch_inhibit_local(overlaps_dev, num_frames, num_columns, grid_w,
                                             radius, n, active_dev,
                                             static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "local inhibition launch");
  return ok();
}

int sp_step_local(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames, int learn,
                  uint32_t grid_w, uint32_t radius, int32_t* overlaps_dev, uint8_t* active_dev,
                  void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  const Shape& sh = h->sh;
  if (grid_w < 1 || grid_w > sh.C) return fail(SP_EINVAL, "grid_w=%u outside 1..C", grid_w);
  if (num_frames == 0) return ok();
  if (!frames_dev || !active_dev || !aligned4(frames_dev) || (overlaps_dev && !aligned4(overlaps_dev)))
    return fail(SP_EINVAL, "frames (4-byte aligned) and active are required");
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  IdleOnExit idle{h, s};
  note_learned(h, num_frames, learn);
  const bool pair = h->lkernel2 && htmsp::persistent_local2_fits(sh.C, h->lwgc, grid_w, radius);
  if (h->lkernel) {
    // The two-frame kernel reads the frames in pairs, in launches of at
    // most `chunk` frames (the one-frame kernel takes all at once).
    uint32_t chunk = num_frames;
    if (pair) {
      rc = pair_stage(h, num_frames, &chunk);
      if (rc) return rc;
    }
    htmsp::LocalArgs a;
    a.idx = h->idx;
    a.perm = h->perm;
    a.fpair = h->fpair;
    a.xchg = pair ? h->xloc2 : h->xloc;
    a.err = h->err;
    a.learn = learn ? 1u : 0u;
    a.replicas = htmsp::kPersistReplicas;
    a.grid_w = grid_w;
    a.radius = radius;
    a.sh = sh;
    void* args[] = {&a};
    for (uint64_t t0 = 0; t0 < num_frames; t0 += chunk) {
      const uint32_t F = (uint32_t)std::min<uint64_t>(chunk, num_frames - t0);
      hipError_t e = hipSuccess;
      if (pair) e = htmsp::launch_pair_frames(frames_dev + t0 * sh.W, F, sh.W, h->fpair, s);
      if (e != hipSuccess) return hip_fail(e, "frame pairing launch");
      a.frames = frames_dev + t0 * sh.W;
      a.ov_out = overlaps_dev ? overlaps_dev + t0 * sh.C : nullptr;
      a.active_out = active_dev + t0 * sh.C;
      a.F = F;
      a.frame_base = (uint32_t)(pair ? h->xloc2_pairs : h->xloc_frames);
      a.spin_limit = h->stall_spins ? h->stall_spins : kSpinLimit;
      a.stall = h->stall_spins ? 1u : 0u;
      h->stall_spins = 0;
      e = hipLaunchCooperativeKernel(pair ? h->lkernel2 : h->lkernel, dim3(h->lgrid),
                                     dim3(htmsp::kPersistWaves * 64), args, 0, s);
      if (e != hipSuccess) return hip_fail(e, "persistent local step launch");
      if (pair)
        h->xloc2_pairs += F / 2 + (F & 1u);
      else
        h->xloc_frames += F;
    }
    return add_histogram_active(h, active_dev, num_frames, s);
  }
  for (uint32_t t = 0; t < num_frames; ++t) {
    const uint32_t* frame = frames_dev + (size_t)t * sh.W;
    int32_t* ov = overlaps_dev ? overlaps_dev + (size_t)t * sh.C : h->ov_scratch;
    uint8_t* act = active_dev + (size_t)t * sh.C;
    hipError_t e = htmsp::launch_overlap_plain(h->idx, h->perm, frame, ov, sh, s);
    if (e == hipSuccess)
      e = htmsp::launch_inhibit_local(ov, 1, sh.C, grid_w, radius, sh.k, act, s);
    if (e == hipSuccess && learn) e = htmsp::launch_learn_active(h->idx, h->perm, frame, act, sh, s);
    if (e != hipSuccess) return hip_fail(e, "local step launch");
  }
  return add_histogram_active(h, active_dev, num_frames, s);
}

int sp_step_local_adaptive(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames,
                           int learn, uint32_t input_w, uint32_t grid_w, uint32_t* radius_dev,
                           int32_t* overlaps_dev, uint8_t* active_dev, uint32_t* radii_dev,
                           void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  const Shape& sh = h->sh;
  if (grid_w < 1 || grid_w > sh.C) return fail(SP_EINVAL, "grid_w=%u outside 1..C", grid_w);
  if (input_w < 1 || input_w > sh.N)
    return fail(SP_EINVAL, "input_w=%u outside 1..input_bits", input_w);
  if (!radius_dev || !aligned4(radius_dev) || (radii_dev && !aligned4(radii_dev)))
    return fail(SP_EINVAL, "radius (4-byte aligned) is required");
  if (num_frames == 0) return ok();
  if (!frames_dev || !active_dev || !aligned4(frames_dev) || (overlaps_dev && !aligned4(overlaps_dev)))
    return fail(SP_EINVAL, "frames (4-byte aligned) and active are required");
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  IdleOnExit idle{h, s};
  note_learned(h, num_frames, learn);
  hipError_t e = htmsp::launch_radius_adapt(h->idx, h->perm, sh, input_w, grid_w, h->racc,
                                            radius_dev, s, true);
  for (uint32_t t = 0; t < num_frames && e == hipSuccess; ++t) {
    const uint32_t* frame = frames_dev + (size_t)t * sh.W;
    int32_t* ov = overlaps_dev ? overlaps_dev + (size_t)t * sh.C : h->ov_scratch;
    uint8_t* act = active_dev + (size_t)t * sh.C;
    e = htmsp::launch_overlap_plain(h->idx, h->perm, frame, ov, sh, s);
    if (e == hipSuccess)
      e = htmsp::launch_inhibit_local(ov, 1, sh.C, grid_w, 0, sh.k, act, s, radius_dev,
                                      radii_dev ? radii_dev + t : nullptr);
    if (e == hipSuccess && learn) e = htmsp::launch_learn_active(h->idx, h->perm, frame, act, sh, s);
    if (e == hipSuccess && learn)
      e = htmsp::launch_radius_adapt(h->idx, h->perm, sh, input_w, grid_w, h->racc, radius_dev,
                                     s);
  }
  if (e != hipSuccess) return hip_fail(e, "adaptive local step launch");
  return add_histogram_active(h, active_dev, num_frames, s);
}

}  // extern "C"

namespace {

int check_boost(const sp_boost_config* b, uint32_t S) {
  if (!b) return fail(SP_EINVAL, "boost config is NULL");
  if (b->period_log2 > 16) return fail(SP_EINVAL, "period_log2=%u > 16", b->period_log2);
  if (b->min_pct_q16 > 65536) return fail(SP_EINVAL, "min_pct_q16=%u > 65536", b->min_pct_q16);
  if (b->max_boost_q8 < 256 || b->max_boost_q8 > 4096)
    return fail(SP_EINVAL, "max_boost_q8=%u outside 256..4096", b->max_boost_q8);
  if (b->bump_q8 > 256) return fail(SP_EINVAL, "bump_q8=%u > 256", b->bump_q8);
  (void)S;
  return SP_OK;
}

// Boost state on the device, set to duty cycles 0 and boosts 1 on first use.
int ensure_boost(sp_handle* h, hipStream_t s) {
  if (h->boost_mem) return SP_OK;
  const uint32_t C = h->sh.C;
  const size_t bytes = sizeof(uint32_t) * 3 * (size_t)C + align_up(C, 4);
  hipError_t e = hipMalloc(&h->boost_mem, bytes);
  if (e != hipSuccess) {
    h->boost_mem = nullptr;
    return fail(SP_ENOMEM, "boost state hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  h->boost_C = C;
  e = htmsp::launch_boost_init(h->boost_mem, h->boost_mem + C, h->boost_mem + 2 * (size_t)C, C,
                               s);
  if (e != hipSuccess) return hip_fail(e, "boost state init");
  return SP_OK;
}

}  // namespace

extern "C" {

int sp_step_boost(sp_handle* h, const sp_boost_config* bc, const uint32_t* frames_dev,
                  uint32_t num_frames, int learn, int32_t* overlaps_dev, int32_t* winners_dev,
                  void* stream) {
  int rc = check_step_args(h, frames_dev, num_frames, overlaps_dev, winners_dev);
  if (rc) return rc;
  rc = check_boost(bc, h->sh.S);
  if (rc) return rc;
  if (num_frames == 0) return ok();
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  IdleOnExit idle{h, s};
  rc = ensure_boost(h, s);
  if (rc) return rc;
  const Shape& sh = h->sh;
  uint32_t* adc = h->boost_mem;
  uint32_t* odc = adc + sh.C;
  uint32_t* boost = odc + sh.C;
  uint8_t* raise = reinterpret_cast<uint8_t*>(boost + sh.C);
  const htmsp::BoostParams bp = {bc->period_log2, bc->min_pct_q16, bc->max_boost_q8,
                                 bc->bump_q8};
  note_learned(h, num_frames, learn);
  if (h->bkernel) {
    htmsp::BoostArgs a;
    a.idx = h->idx;
    a.perm = h->perm;
    a.frames = frames_dev;
    a.ov_out = overlaps_dev;
    a.win_out = winners_dev;
    a.xchg = h->xloc;
    a.err = h->err;
    a.adc = adc;
    a.odc = odc;
    a.boost = boost;
    a.F = num_frames;
    a.learn = learn ? 1u : 0u;
    a.frame_base = (uint32_t)h->xloc_frames;
    a.replicas = htmsp::kPersistReplicas;
    a.spin_limit = h->stall_spins ? h->stall_spins : kSpinLimit;
    a.stall = h->stall_spins ? 1u : 0u;
    h->stall_spins = 0;
    a.b = bp;
    a.sh = sh;
    void* args[] = {&a};
    hipError_t e = hipLaunchCooperativeKernel(h->bkernel, dim3(h->bgrid),
                                              dim3(htmsp::kPersistWaves * 64), args, 0, s);
    if (e != hipSuccess) return hip_fail(e, "persistent boosted step launch");
    h->xloc_frames += num_frames;
    return add_histogram(h, winners_dev, num_frames, s);
  }
  for (uint32_t t = 0; t < num_frames; ++t) {
    const uint32_t* frame = frames_dev + (size_t)t * sh.W;
    int32_t* ov = overlaps_dev ? overlaps_dev + (size_t)t * sh.C : h->ov_scratch;
    int32_t* win = winners_dev + (size_t)t * sh.k;
    hipError_t e = htmsp::launch_overlap_plain(h->idx, h->perm, frame, ov, sh, s, boost);
    if (e == hipSuccess) e = htmsp::launch_topk_plain(ov, win, sh, s, 1, sh.S * bc->max_boost_q8);
    if (learn) {
      if (e == hipSuccess) e = htmsp::launch_learn_plain(h->idx, h->perm, frame, win, sh, s);
      if (e == hipSuccess)
        e = htmsp::launch_boost_update(ov, win, sh, bp, adc, odc, boost, raise, h->perm, s);
    }
    if (e != hipSuccess) return hip_fail(e, "boosted step launch");
  }
  return add_histogram(h, winners_dev, num_frames, s);
}

int sp_boost_state(sp_handle* h, uint32_t* active_duty_dev, uint32_t* overlap_duty_dev,
                   uint32_t* boost_dev, void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  IdleOnExit idle{h, s};
  rc = ensure_boost(h, s);
  if (rc) return rc;
  const size_t n = sizeof(uint32_t) * h->sh.C;
  hipError_t e = hipSuccess;
  if (active_duty_dev)
    e = hipMemcpyAsync(active_duty_dev, h->boost_mem, n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && overlap_duty_dev)
    e = hipMemcpyAsync(overlap_duty_dev, h->boost_mem + h->sh.C, n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && boost_dev)
    e = hipMemcpyAsync(boost_dev, h->boost_mem + 2 * (size_t)h->sh.C, n,
                       hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "boost state copy");
  return ok();
}

int sp_boost_reset(sp_handle* h, void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!h->boost_mem) return ok();
  DeviceScope ds(h->device);
  IdleOnExit idle{h, static_cast<hipStream_t>(stream)};
  hipError_t e = htmsp::launch_boost_init(h->boost_mem, h->boost_mem + h->sh.C,
                                          h->boost_mem + 2 * (size_t)h->sh.C, h->sh.C,
                                          static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "boost state reset");
  return ok();
}

size_t sp_encoded_bits(const sp_encoder_config* cfg) {
  htmsp::EncShape e;
  if (encoder_shape(cfg, &e)) return 0;
  ok();
  return (size_t)e.w * e.h;
}

int sp_encode(const sp_encoder_config* cfg, const uint8_t* rgb_dev, uint32_t num_frames,
              uint32_t* frames_dev, void* stream) {
  htmsp::EncShape e;
  int rc = encoder_shape(cfg, &e);
  if (rc) return rc;
  if (num_frames == 0) return ok();
  if (!rgb_dev || !frames_dev) return fail(SP_EINVAL, "rgb and frames are required");
  if (!aligned4(frames_dev)) return fail(SP_EINVAL, "frames must be 4-byte aligned");
  hipError_t err = htmsp::launch_encode(rgb_dev, num_frames, e, frames_dev,
                                        static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "encoder launch");
  return ok();
}

int sp_set_histogram(sp_handle* h, uint32_t* hist_dev) {
  if (!h) return fail(SP_EINVAL, "handle is NULL");
  if (hist_dev && ((uintptr_t)hist_dev & 3u))
    return fail(SP_EINVAL, "histogram must be 4-byte aligned");
  h->hist = hist_dev;
  return ok();
}

int sp_step_is_persistent(const sp_handle* h) {
  if (!h) return fail(SP_EINVAL, "handle is NULL");
  return h->persistent ? 1 : 0;
}

int sp_test_stall(sp_handle* h, uint32_t spin_limit) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (spin_limit < 1 || spin_limit > kSpinLimit)
    return fail(SP_EINVAL, "spin_limit=%u outside 1..%u", spin_limit, kSpinLimit);
  h->stall_spins = spin_limit;
  return ok();
}

int sp_step_boost_kernel(const sp_handle* h) {
  if (!h) return fail(SP_EINVAL, "handle is NULL");
  return h->bkernel ? SP_KERNEL_PERSISTENT_WAVE : SP_KERNEL_PLAIN;
}

int sp_step_local_kernel(const sp_handle* h) {
  if (!h) return fail(SP_EINVAL, "handle is NULL");
  return h->lkernel ? SP_KERNEL_PERSISTENT_WAVE : SP_KERNEL_PLAIN;
}

int sp_step_local_kernel_for(const sp_handle* h, uint32_t grid_w, uint32_t radius) {
  if (!h) return fail(SP_EINVAL, "handle is NULL");
  if (grid_w < 1 || grid_w > h->sh.C) return fail(SP_EINVAL, "grid_w=%u outside 1..C", grid_w);
  if (h->lkernel2 && htmsp::persistent_local2_fits(h->sh.C, h->lwgc, grid_w, radius))
    return SP_KERNEL_PERSISTENT_PAIR;
  return h->lkernel ? SP_KERNEL_PERSISTENT_WAVE : SP_KERNEL_PLAIN;
}

int sp_step_kernel(const sp_handle* h) {
  if (!h) return fail(SP_EINVAL, "handle is NULL");
  return h->persistent ? SP_KERNEL_PERSISTENT_WAVE : SP_KERNEL_PLAIN;
}

int sp_sync(sp_handle* h, void* stream) {
  if (!h) return fail(SP_EINVAL, "handle is NULL");
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t err = 0;
  hipError_t e = hipMemcpyAsync(&err, h->err, sizeof(err), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    h->broken = true;
    return hip_fail(e, "sync");
  }
  if (err) {
    h->broken = true;
    return fail(SP_EDEVICE, "a persistent step gave up waiting for the per-frame exchange");
  }
  if (h->broken) return fail(SP_EBROKEN, "handle saw a device failure; destroy it");
  return ok();
}

int sp_destroy(sp_handle* h) {
  if (!h) return ok();
  int rc = SP_OK;
  {
    DeviceScope ds(h->device);
    // the handle's own work, not the whole device
    hipError_t e = h->idle_used ? hipEventSynchronize(h->idle) : hipSuccess;
    if (e == hipSuccess) e = many_wait(h);
    // buffers of batched inference and boosting (hipFree waits for the device)
    if (e == hipSuccess && h->infer_list) e = hipFree(h->infer_list);
    if (e == hipSuccess && h->infer_ov) e = hipFree(h->infer_ov);
    if (e == hipSuccess && h->boost_mem) e = hipFree(h->boost_mem);
    if (e == hipSuccess && h->mfma_mask) e = hipFree(h->mfma_mask);
    if (e == hipSuccess && h->mfma_part) e = hipFree(h->mfma_part);
    if (e == hipSuccess && h->fpair) e = hipFree(h->fpair);
    if (e == hipSuccess && !ws_give(h->device, h->ws, h->ws_bytes)) e = hipFree(h->ws);
    const hipError_t e2 = hipEventDestroy(h->idle);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) rc = hip_fail(e, "destroy");
  }
  delete h;
  return rc ? rc : ok();
}

size_t sp_state_bytes(const sp_config* cfg) {
  if (check_config(cfg)) return 0;
  return (sizeof(uint32_t) + sizeof(float)) * (size_t)cfg->num_columns * cfg->synapses_per_column;
}

int sp_get_state(sp_handle* h, uint32_t* idx_host, float* perm_host, uint64_t* frames_seen,
                 void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t n = (size_t)h->sh.C * h->sh.S;
  hipError_t e = hipSuccess;
  if (idx_host) e = hipMemcpyAsync(idx_host, h->idx, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && perm_host)
    e = hipMemcpyAsync(perm_host, h->perm, sizeof(float) * n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "state copy");
  if (frames_seen) *frames_seen = h->frames_seen;
  return ok();
}

int sp_set_state(sp_handle* h, const uint32_t* idx_host, const float* perm_host,
                 uint64_t frames_seen, void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!perm_host) return fail(SP_EINVAL, "perm is NULL");
  const size_t n = (size_t)h->sh.C * h->sh.S;
  for (size_t i = 0; idx_host && i < n; ++i)
    if (idx_host[i] >= h->sh.N)
      return fail(SP_EINVAL, "idx[%zu]=%u >= input_bits=%u", i, idx_host[i], h->sh.N);
  for (size_t i = 0; i < n; ++i) {
    const float q = perm_host[i] * 256.0f;
    if (!(q >= 0.0f && q <= 256.0f && q == (float)(int)q))
      return fail(SP_EINVAL, "perm[%zu]=%.9g is off the 1/256 grid or outside [0,1]", i,
                  (double)perm_host[i]);
  }
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (idx_host) e = hipMemcpyAsync(h->idx, idx_host, sizeof(uint32_t) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->perm, perm_host, sizeof(float) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    h->broken = true;
    return hip_fail(e, "state copy");
  }
  ++h->state_version;
  h->frames_seen = frames_seen;
  return ok();
}

int sp_get_boost_state(sp_handle* h, uint32_t* active_duty_host, uint32_t* overlap_duty_host,
                       uint32_t* boost_host, void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = ensure_boost(h, s);
  if (rc) return rc;
  const size_t C = h->sh.C, n = sizeof(uint32_t) * C;
  uint32_t* dst[3] = {active_duty_host, overlap_duty_host, boost_host};
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < 3 && e == hipSuccess; ++i)
    if (dst[i]) e = hipMemcpyAsync(dst[i], h->boost_mem + i * C, n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "boost state copy");
  return ok();
}

int sp_set_boost_state(sp_handle* h, const uint32_t* active_duty_host,
                       const uint32_t* overlap_duty_host, const uint32_t* boost_host,
                       void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!active_duty_host || !overlap_duty_host || !boost_host)
    return fail(SP_EINVAL, "active duty, overlap duty and boost are all required");
  const uint32_t C = h->sh.C;
  for (uint32_t c = 0; c < C; ++c) {
    if (active_duty_host[c] > 65536 || overlap_duty_host[c] > 65536)
      return fail(SP_EINVAL, "duty cycle of column %u above 65536", c);
    if (boost_host[c] < 256 || boost_host[c] > 4096)
      return fail(SP_EINVAL, "boost[%u]=%u outside 256..4096", c, boost_host[c]);
  }
  DeviceScope ds(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = ensure_boost(h, s);
  if (rc) return rc;
  const uint32_t* src[3] = {active_duty_host, overlap_duty_host, boost_host};
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < 3 && e == hipSuccess; ++i)
    e = hipMemcpyAsync(h->boost_mem + i * (size_t)C, src[i], sizeof(uint32_t) * C,
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    h->broken = true;
    return hip_fail(e, "boost state copy");
  }
  return ok();
}

const char* sp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
