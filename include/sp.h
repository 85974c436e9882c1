/*
 * htmsp -- HTM spatial pooler step on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library libhtmsp.so.  One spatial pooler instance maps a
 * binary input frame to a sparse set of winning columns and, when learning,
 * updates its synapse permanences (Wielgosz & Pietron, arXiv 1608.01966,
 * Section 1.1):
 *
 *   overlap     Algorithm 1: per column, the number of connected synapses
 *               (permanence >= connected threshold) whose input bit is on;
 *               a count below min_overlap becomes 0; boost is 1.
 *   inhibition  Algorithm 2, global form: the winners_set_size columns of
 *               highest positive overlap, ties to the lower column index;
 *               a column with overlap 0 never wins, so fewer than
 *               winners_set_size columns win when fewer have overlap > 0.
 *   learning    the learning stage the paper takes from the Numenta CLA
 *               whitepaper: for every winner, each potential synapse gains
 *               inc if its input bit is on and loses dec otherwise, clipped
 *               to [0, 1].
 *
 * Data layout (all device memory, row-major, no padding):
 *   idx     uint32 [C][S]  input pixel of each potential synapse, < N
 *   perm    float  [C][S]  permanence, a multiple of 1/256 in [0, 1]
 *   frames  uint32 [F][W]  W = ceil(N / 32); pixel p is bit (p & 31) of word
 *                          (p >> 5), least significant bit first; bits at or
 *                          past N are ignored
 *   overlaps int32 [F][C]  gated overlap per frame and column
 *   winners  int32 [F][k]  winners of each frame in ascending column order,
 *                          padded with -1
 *
 * Permanences are restricted to the 1/256 grid (and inc, dec and the
 * threshold are given in 1/256 units) so that every update is exact in FP32
 * and results are reproducible bit for bit.
 *
 * Ownership: idx and perm are caller-owned device buffers that the handle
 * borrows for its lifetime; the library reads idx and reads/writes perm in
 * place.  frames, overlaps and winners are caller-owned per call.  The
 * library allocates a small per-handle workspace (sp_workspace_bytes) in
 * sp_create (or reuses one a destroyed handle left in the library's pool)
 * and, on the first sp_infer, the compacted connected lists
 * (4 * (S * C + C) bytes) plus, when sp_infer gets no overlap buffer, an
 * [F][C] scratch, on the first sp_step_boost the boost state
 * (13 C bytes, rounded up), and on the first sp_step that runs the
 * persistent kernel a copy of the step's frames in pairs (8 bytes per
 * input word per pair of frames, at most 64 MiB: longer steps run as
 * several launches); sp_destroy frees or pools all of it.
 * sp_step_many keeps two staging buffers per device for the library's
 * lifetime (descriptors, and a packed copy of the launch's synapses, 4 bytes
 * each, rebuilt by every launch), grown when a launch needs more.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  Steps are
 * enqueued and return at once; results are valid once the stream has
 * synchronised.  A handle must not be used by two calls at the same time,
 * and its calls must be ordered on the device (one stream, or streams the
 * caller synchronises between calls): each call reuses the handle's state,
 * workspace and buffers.
 *
 * Errors: every call returns SP_OK (0) or a negative sp_status; argument and
 * configuration checks happen on the host before anything is enqueued, and
 * out-parameters are written only on SP_OK.  sp_last_error() describes the
 * last failure of the calling thread.  Nothing is thrown across the ABI.
 */
#ifndef HTMSP_SP_H
#define HTMSP_SP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sp_status {
  SP_OK = 0,
  SP_EINVAL = -1,  /* bad argument, configuration or state contents        */
  SP_ENOMEM = -2,  /* workspace allocation failed                          */
  SP_EDEVICE = -3, /* HIP error, no usable device, or a failed device step */
  SP_EBROKEN = -4  /* the handle saw a device failure and must be destroyed */
} sp_status;

/* Limits checked by sp_config_check. */
#define SP_MAX_INPUT_BITS (1u << 23)
#define SP_MAX_COLUMNS 65536u
#define SP_MAX_SYNAPSES 4096u

typedef struct sp_config {
  uint32_t input_bits;          /* N, 1..SP_MAX_INPUT_BITS                   */
  uint32_t num_columns;         /* C, 1..SP_MAX_COLUMNS                      */
  uint32_t synapses_per_column; /* S, 1..SP_MAX_SYNAPSES                     */
  uint32_t min_overlap;         /* m (any value; m > S means no winners)     */
  uint32_t winners;             /* k = winners_set_size, 1..C                */
  uint32_t connected_q8;        /* connected threshold x 256, 0..256         */
  uint32_t inc_q8;              /* permanence increment x 256, 0..256        */
  uint32_t dec_q8;              /* permanence decrement x 256, 0..256        */
} sp_config;

typedef struct sp_handle sp_handle;

/* Host-only check of a configuration against the limits above. */
int sp_config_check(const sp_config* cfg);

/* Words per packed frame, ceil(N / 32); 0 for an invalid configuration. */
size_t sp_frame_words(const sp_config* cfg);

/* Bytes of device workspace sp_create allocates for this configuration; 0
 * for an invalid configuration. */
size_t sp_workspace_bytes(const sp_config* cfg);

/* Host-only check of state held in host memory: every idx < N and every
 * permanence a multiple of 1/256 in [0, 1].  SP_EINVAL names the first bad
 * entry. */
int sp_check_state_host(const sp_config* cfg, const uint32_t* idx, const float* perm);

/* Creates a handle over the caller's device state (borrowed, see above) on
 * the current HIP device.  Validates the configuration on the host and the
 * state contents on the device (synchronising `stream`): SP_EINVAL if an
 * index is >= N or a permanence is off the 1/256 grid. */
int sp_create(const sp_config* cfg, uint32_t* idx_dev, float* perm_dev, void* stream,
              sp_handle** out);

/* Re-validates the borrowed state on the device after the caller changed it
 * (synchronises `stream`). */
int sp_check_state(sp_handle* h, void* stream);

/* One spatial pooler step for each of F frames, in order (Section 1.1:
 * overlap, inhibition, then learning when learn != 0, the permanences left
 * by frame t feeding frame t + 1).  learn == 0 leaves the state untouched.
 * overlaps may be NULL; winners must not be.  F == 0 is a no-op.
 *
 * The frames run in one persistent launch that keeps the handle's synapse
 * state in registers (a group of columns per wave, one workgroup per CU, the
 * per-frame overlaps exchanged through device memory, two frames per
 * exchange), after a short pass that copies the frames side by side in
 * pairs; a step whose pairs exceed 64 MiB runs as several such launches.
 * Shapes the kernel cannot hold (see sp_step_kernel) run as sp_step_plain,
 * with the same results.  A device-side failure of the
 * persistent launch is reported by the next sp_sync. */
int sp_step(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames, int learn,
            int32_t* overlaps_dev, int32_t* winners_dev, void* stream);

/* Same contract as sp_step, executed one frame per launch sequence
 * (overlap, inhibition, learning kernels per frame): the plain baseline. */
int sp_step_plain(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames, int learn,
                  int32_t* overlaps_dev, int32_t* winners_dev, void* stream);

/* Batched inference (Section 4.1's testing mode, learning off): overlap
 * and global inhibition of F independent frames against the handle's
 * current state, which is left unchanged.  Results equal sp_step with
 * learn = 0 frame by frame, in either mode.
 *
 * mode SP_INFER_GATHER compacts every column's connected synapses once per
 * state change (a step that learned, or sp_check_state), then counts active
 * inputs by gathering bits of each frame staged in LDS, each column's list
 * held in registers.  The first call after a state change synchronises
 * `stream` (it reads back the longest connected list); when that list is
 * longer than 256 synapses the lists are read from device memory for every
 * frame instead (same results, slower).
 *
 * mode SP_INFER_MFMA_I8 computes the overlaps as one dense matrix product,
 * frames (0/1 per pixel) times the connected mask (1 where a connected
 * synapse of the column sits on the pixel), both widened from bits to int8
 * in registers and accumulated in int32 by the matrix cores, then gates and
 * selects as the gather mode does.  The mask, C x ceil(N / 512) x 64 bytes,
 * is built once per state change (that first call synchronises `stream`);
 * SP_EINVAL if it would exceed 4 GiB or if two connected synapses of one
 * column share a pixel (a 0/1 mask cannot count them).  Frames and mask
 * stay bit-packed; there is no limit on connected synapses per column.
 *
 * overlaps may be NULL (the library then keeps an internal [F][C] buffer,
 * grown on demand); winners must not be.  Library-owned buffers, freed by
 * sp_destroy: gather lists 4 (S C + C + 64) bytes; the mask plus 256 bytes;
 * for the matrix product on few frames (F x C below about 2^24), partial
 * sums of up to 8 pixel ranges, 4 x ranges x F x C bytes. */
#define SP_INFER_GATHER 0
#define SP_INFER_MFMA_I8 1
int sp_infer(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames, int mode,
             int32_t* overlaps_dev, int32_t* winners_dev, void* stream);

/* Batched inference that allocates nothing, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the gather mode of sp_infer with the
 * same results, its working lists held in a fixed device scratch array of
 * sp_infer_noalloc_max_bytes() (16 MiB) per GPU that the library keeps for
 * the life of the process, instead of lists the handle allocates.  The
 * caller passes every input and output: overlaps_dev [F][C] is required.
 * The lists are rebuilt by every call (no state version is kept, and the
 * stream is never synchronised).  SP_EINVAL if S > 256 or if the lists,
 * 4 (S C + C) bytes, exceed the scratch.  All calls on one GPU share its
 * scratch: calls that overlap in time on one GPU (on different streams, or
 * from different threads) race and give wrong results. */
size_t sp_infer_noalloc_max_bytes(void);
int sp_infer_noalloc(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames,
                     int32_t* overlaps_dev, int32_t* winners_dev, void* stream);

/* Steps n independent handles together (each handle as by sp_step: its
 * frames in order, overlap, inhibition and, when learn != 0, learning) in one
 * persistent launch whose workgroups serve tiles of every instance and one
 * top-k task per instance, synapse state streamed from device memory every
 * step.  Arrays have n entries: frames_dev[i] holds num_frames[i] frames of
 * handle i (0 = skip it), winners_dev[i] is [num_frames[i]][k_i],
 * overlaps_dev may be NULL or hold NULL entries.  Handles must be distinct,
 * on one device, with at most 4096 columns each.  Results equal stepping each
 * handle alone.  Instances beyond what one launch holds go into further
 * launches on the same stream.  A device-side failure (a wait that gives up)
 * is reported by sp_sync on every handle whose steps it may have cut short;
 * a handle of the failing launch whose steps all completed reports nothing
 * and holds the results of stepping it alone.  If a
 * launch cannot be enqueued, the call returns SP_EDEVICE: the handles of
 * earlier launches of the call were stepped, those of the failed launch and
 * later ones are broken (SP_EBROKEN).  Calls are serialised by the library;
 * one call's launch must not overlap another call's on a different stream. */
int sp_step_many(sp_handle* const* hs, uint32_t n, const uint32_t* const* frames_dev,
                 const uint32_t* num_frames, int learn, int32_t* const* overlaps_dev,
                 int32_t* const* winners_dev, void* stream);

/* Boosting and duty cycles: Algorithm 1 multiplies each column's gated
 * overlap by its boost (Section 3.2.2 computes it in the kernel); after each
 * learning frame the duty cycles, the boosts and the permanence raise follow
 * the whitepaper's spatial pooler phase 3, in exact fixed point:
 *   boosts in 1/256 (>= 1), duty cycles in 1/65536, each updated as
 *   d <- floor((d (P - 1) + 65536 e) / P), P = 2^period_log2, e = 1 when
 *   the column won (active duty cycle) / had a positive gated overlap
 *   (overlap duty cycle);
 *   min duty = floor(max active duty * min_pct_q16 / 65536);
 *   boost = 1 when min == 0 or active duty >= min, else
 *   1 + floor((max_boost_q8 - 256) (min - duty) / min) / 256;
 *   a column whose overlap duty cycle is below min has every permanence
 *   raised by bump_q8 / 256, clipped at 1. */
typedef struct sp_boost_config {
  uint32_t period_log2;  /* 0..16                                         */
  uint32_t min_pct_q16;  /* 0..65536 (655 ~ 0.01)                         */
  uint32_t max_boost_q8; /* 256..4096                                     */
  uint32_t bump_q8;      /* 0..256                                        */
} sp_boost_config;

/* Frames in order with boosting: boosted overlap, global top-k of the
 * boosted overlaps (ties to the lower index), and with learn != 0 the
 * winners' learning and the duty-cycle/boost/raise update; one persistent
 * launch for all frames where the shape allows it (C <= 1024, S <= 1024,
 * see sp_step_boost_kernel), else one launch sequence per frame, with the
 * same results.  The boost state lives in the handle (allocated on
 * first use, duty cycles 0 and boosts 1) and carries over between calls;
 * learn = 0 leaves it and the permanences unchanged.  overlaps_dev, if not
 * NULL, receives the boosted overlaps in 1/256 units. */
int sp_step_boost(sp_handle* h, const sp_boost_config* cfg, const uint32_t* frames_dev,
                  uint32_t num_frames, int learn, int32_t* overlaps_dev, int32_t* winners_dev,
                  void* stream);

/* Copies the boost state (uint32 [C] each; NULL skips one) on `stream`. */
int sp_boost_state(sp_handle* h, uint32_t* active_duty_dev, uint32_t* overlap_duty_dev,
                   uint32_t* boost_dev, void* stream);

/* Duty cycles back to 0 and boosts to 1. */
int sp_boost_reset(sp_handle* h, void* stream);

/* Checkpoint and resume (the pooler as a unit that keeps learning across
 * sessions, Section 3.2.1, and switches between learning and testing,
 * Section 4.1).  The state of a handle is its borrowed idx and perm, the
 * count of learning frames it has applied (every step with learn != 0 adds
 * its frame count), and the boost state of sp_step_boost.  Stepping a
 * handle restored from a checkpoint gives the same results as stepping the
 * handle the checkpoint was taken from.
 *
 * sp_state_bytes: bytes of idx plus perm, 8 C S (0 on a bad configuration).
 * sp_get_state: copies idx [C][S] and perm [C][S] into host memory (either
 *   may be NULL) and the frame count into *frames_seen (may be NULL), then
 *   synchronises `stream`.
 * sp_set_state: checks the host arrays (idx < N, permanences on the 1/256
 *   grid in [0, 1]; SP_EINVAL names the first bad entry, nothing changes),
 *   copies them into the handle's borrowed device buffers (idx NULL keeps
 *   the pools), sets the frame count and synchronises `stream`.  A failed
 *   copy breaks the handle.
 * sp_get_boost_state / sp_set_boost_state: the boost state, uint32 [C]
 *   each, in host memory (duty cycles 0..65536, boosts 256..4096; the setter
 *   checks these ranges and needs all three arrays); both synchronise
 *   `stream`.  A handle that never boosted reports duty cycles 0 and boosts
 *   1 (256). */
size_t sp_state_bytes(const sp_config* cfg);
int sp_get_state(sp_handle* h, uint32_t* idx_host, float* perm_host, uint64_t* frames_seen,
                 void* stream);
int sp_set_state(sp_handle* h, const uint32_t* idx_host, const float* perm_host,
                 uint64_t frames_seen, void* stream);
int sp_get_boost_state(sp_handle* h, uint32_t* active_duty_host, uint32_t* overlap_duty_host,
                       uint32_t* boost_host, void* stream);
int sp_set_boost_state(sp_handle* h, const uint32_t* active_duty_host,
                       const uint32_t* overlap_duty_host, const uint32_t* boost_host,
                       void* stream);

/* Local inhibition, Algorithm 2 as printed: every column competes within
 * the neighbourhood an inhibition radius gives it (Section 3.2.2), instead
 * of the global top-k of sp_step.  Columns sit on a row-major grid of grid_w
 * columns per row; the neighbourhood of c is every other column whose row
 * and column coordinates differ from c's by at most `radius` (no wrap); with
 * v the n-th largest neighbour overlap (0 if there are fewer than n
 * neighbours), c is active iff overlap[c] > max(v, 1).  Ties at v lose, so
 * the number of active columns is not fixed.
 * overlaps_dev: int32 [num_frames][num_columns] gated overlaps (as sp_step or
 * sp_infer write them); active_dev: uint8 [num_frames][num_columns], 0 or 1.
 * 1 <= grid_w <= num_columns, n >= 1.  Asynchronous; allocates nothing. */
int sp_inhibit_local(const int32_t* overlaps_dev, uint32_t num_frames, uint32_t num_columns,
                     uint32_t grid_w, uint32_t radius, uint32_t n, uint8_t* active_dev,
                     void* stream);

/* Frames in order through overlap (Algorithm 1), local inhibition (as
 * sp_inhibit_local, n = the handle's `winners`) and, when learn != 0,
 * learning on the active columns.  One persistent launch for all frames
 * where the shape allows it (C <= 4096, S <= 1024, see
 * sp_step_local_kernel), else one launch sequence per frame; the results
 * are the same.  overlaps_dev [F][C] may be NULL; active_dev is [F][C]
 * uint8.  The handle's histogram, if set, gains 1 per frame for each
 * active column.  A device-side failure of the persistent launch is
 * reported by sp_sync. */
int sp_step_local(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames, int learn,
                  uint32_t grid_w, uint32_t radius, int32_t* overlaps_dev, uint8_t* active_dev,
                  void* stream);

/* sp_step_local with the inhibition radius adapted after every learning
 * frame (Section 4.4: a change of winners_set_size is compensated by
 * adapting the inhibition radius, which the paper takes from the
 * whitepaper, where it becomes the average connected receptive field size
 * of the columns).  The input is an image of input_w pixels per row (pixel
 * p at x = p mod input_w, y = p div input_w; in_h = ceil(N / input_w)
 * rows) and the columns a grid of grid_w per row (grid_h = ceil(C /
 * grid_w) rows).  After a learning frame, over the n columns with at least
 * one connected synapse, A = the sum of span_x + span_y, span = max - min
 * + 1 of the connected inputs' coordinates, and
 *   radius = max(1, floor(A (grid_w in_h + grid_h in_w) / (8 n in_w in_h))),
 * i.e. the mean extent A / 2n times the mean grid-per-input ratio is the
 * diameter d and the radius is (d - 1) / 2 rounded half up; with n = 0 the
 * radius stays.  radius_dev: a device uint32 holding the radius of the
 * first frame, updated on the stream after each learning frame (learn = 0
 * leaves it); radii_dev [F] (may be NULL) receives the radius each frame
 * used.  Runs one launch sequence per frame (no persistent execution).
 * SP_EINVAL on a bad grid_w, input_w or pointer. */
int sp_step_local_adaptive(sp_handle* h, const uint32_t* frames_dev, uint32_t num_frames,
                           int learn, uint32_t input_w, uint32_t grid_w, uint32_t* radius_dev,
                           int32_t* overlaps_dev, uint8_t* active_dev, uint32_t* radii_dev,
                           void* stream);

/* Adaptive video encoder (Section 3.1.2): colour frames to the pooler's
 * packed binary input.  Each frame may be reduced by an integer factor
 * (block means, rounded half up), is converted to grayscale (BT.601 luma in
 * 14-bit fixed point) and binarised against its neighbourhood: a pixel is
 * on iff its gray value exceeds the Gaussian-weighted mean of the block x
 * block window around it minus `offset`, with the binomial weights
 * C(block - 1, i) as the Gaussian window, edge pixels repeated outside the
 * image, and the mean rounded half up. */
typedef struct sp_encoder_config {
  uint32_t width, height; /* input frame size in pixels                        */
  uint32_t factor;        /* reduction factor 1..32 (1 = none); output is       */
                          /* (width / factor) x (height / factor), at most 4096 */
                          /* pixels wide                                        */
  uint32_t block;         /* odd window size, 3..11                             */
  int32_t offset;         /* subtracted from the weighted mean, -255..255       */
} sp_encoder_config;

/* Input bits of one encoded frame: (width / factor) * (height / factor); 0
 * on a bad configuration. */
size_t sp_encoded_bits(const sp_encoder_config* cfg);

/* Encodes num_frames frames.  rgb_dev: device bytes [num_frames][height]
 * [width][3] (R, G, B).  frames_dev: device words [num_frames][ceil(bits /
 * 32)] in the layout sp_step reads (pixel p = y w + x at bit p & 31 of word
 * p >> 5, trailing bits zero); the call clears it first.  Asynchronous on
 * `stream`; allocates nothing.
 * SP_EINVAL on a bad configuration or pointer. */
int sp_encode(const sp_encoder_config* cfg, const uint8_t* rgb_dev, uint32_t num_frames,
              uint32_t* frames_dev, void* stream);

/* Per-stream SDR histogram (Section 2: the pooler output of every frame of a
 * video is accumulated into a histogram, the video's feature vector).
 * hist_dev: caller-owned uint32 [num_columns] device buffer, or NULL to stop.
 * From then on every sp_step, sp_step_plain, sp_infer, sp_infer_noalloc,
 * sp_step_many, sp_step_boost and sp_step_local of this handle adds, for
 * each frame, 1 to hist_dev[c] for each winner (for sp_step_local: each
 * active column) c, on the call's stream after its outputs are written.  The library never clears
 * it; the buffer must outlive its use.  SP_EINVAL on a bad handle or a
 * misaligned pointer. */
int sp_set_histogram(sp_handle* h, uint32_t* hist_dev);

/* 1 if sp_step runs this handle's shape as one persistent launch, 0 if it
 * runs the plain path, negative on a bad handle. */
int sp_step_is_persistent(const sp_handle* h);

/* Which execution sp_step uses for this handle's shape on its device:
 * SP_KERNEL_PLAIN (three launches a frame) or SP_KERNEL_PERSISTENT_WAVE (one
 * persistent launch, a column group per wave, one workgroup per CU);
 * negative on a bad handle.  Informational: every execution gives the same
 * results. */
#define SP_KERNEL_PLAIN 0
#define SP_KERNEL_PERSISTENT_WAVE 2
int sp_step_kernel(const sp_handle* h);

/* Which execution sp_step_local uses for this handle's shape on its device:
 * SP_KERNEL_PLAIN (three launches a frame) or SP_KERNEL_PERSISTENT_WAVE (one
 * persistent launch, a column group per wave); negative on a bad handle.
 * The persistent launch exchanges one frame at a time, or two frames at a
 * time where the neighbourhood allows it (sp_step_local_kernel_for). */
int sp_step_local_kernel(const sp_handle* h);

/* Which execution sp_step_local uses for this handle with this grid width
 * and radius: SP_KERNEL_PERSISTENT_PAIR (one persistent launch, two frames
 * per exchange: every workgroup also decides the columns of its
 * neighbourhoods' bounding box, at most 1024 of them, each over a window of
 * at most 2048 columns), else as sp_step_local_kernel.  SP_EINVAL for
 * grid_w outside 1..C, negative on a bad handle.  Informational: every
 * execution gives the same results. */
#define SP_KERNEL_PERSISTENT_PAIR 3
int sp_step_local_kernel_for(const sp_handle* h, uint32_t grid_w, uint32_t radius);

/* Which execution sp_step_boost uses for this handle's shape on its device:
 * SP_KERNEL_PLAIN (five launches a frame) or SP_KERNEL_PERSISTENT_WAVE (one
 * persistent launch, a column group per wave, C <= 1024); negative on a bad
 * handle. */
int sp_step_boost_kernel(const sp_handle* h);

/* For tests of the failure path (callers: test suites, not applications):
 * the next persistent launch of sp_step, sp_step_local, sp_step_boost or
 * sp_step_many that holds this handle waits for exchange entries that are
 * never written, giving up after `spin_limit` polls (1..2^21) as a stalled
 * exchange would, so that every wave leaves its loop and the launch drains;
 * sp_sync then reports SP_EDEVICE (for sp_step_many: on this handle and on
 * every other handle whose steps the launch cut short) and the handle is
 * broken.  Applies to one launch; a plain
 * (non-persistent) step ignores it.  SP_EINVAL on a bad handle or limit. */
int sp_test_stall(sp_handle* h, uint32_t spin_limit);

/* Synchronises `stream` and reports a device-side failure of an earlier
 * step on this handle (SP_EDEVICE, after which the handle is SP_EBROKEN). */
int sp_sync(sp_handle* h, void* stream);

/* Waits for the work enqueued on this handle (its own calls, not the rest
 * of the device), returns its workspace to a per-device pool that later
 * sp_create calls reuse (at most 256 MiB per device, held until the process
 * ends, so that retiring a handle never waits for other streams), and frees
 * the buffers of batched inference and boosting if it has any (that free
 * waits for the device).  NULL is accepted.  The borrowed state is left as
 * it is; the caller may free it once this returns. */
int sp_destroy(sp_handle* h);

/* Message for the calling thread's last failure ("" if none).  Valid until
 * the thread's next call into the library. */
const char* sp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
