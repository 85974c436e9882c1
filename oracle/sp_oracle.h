/*
 * Oracle for the HTM spatial pooler step -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what one spatial
 * pooler step computes for a binary input frame, written from the paper
 * (Wielgosz & Pietron, "OpenCL-accelerated object classification in video
 * streams using Spatial Pooler of HTM", arXiv 1608.01966):
 *   - overlap, Section 1.1 Algorithm 1,
 *   - inhibition, Section 1.1 Algorithm 2, in its global form,
 *   - learning, which Section 1.1 defers to the Numenta CLA whitepaper
 *     (the paper's reference [Numenta]), spatial pooler phase 3.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this code.  It shares nothing with the GPU library: no header, no
 * helper, no table.  Permanences are held in double precision; every
 * permanence the method produces lies on the 1/256 grid, so double holds
 * each value and each update exactly.
 *
 * Readings taken where the paper is silent or ambiguous (each one is also
 * listed in the design notes):
 *   R1  a synapse is connected iff permanence >= connected threshold;
 *   R2  an overlap below min_overlap is zeroed, so overlap == min_overlap
 *       passes (Algorithm 1's comparison, not the prose's "larger than");
 *   R3  boost is identically 1;
 *   R4  inhibition is global: the winners are the min(k, |E|) columns of
 *       E = {overlap > 0} with the highest overlap, ties going to the lower
 *       column index; a column with zero overlap never wins;
 *   R5  learning visits every potential synapse of every winner: an active
 *       input raises the permanence by inc, an inactive one lowers it by
 *       dec, and the result is clipped to [0, 1];
 *   R6  input pixel p is bit (p & 31) of 32-bit word (p >> 5), LSB first;
 *       bits at or past input_bits are ignored.
 */
#ifndef SP_ORACLE_H
#define SP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spo_config {
  uint32_t input_bits;          /* N: input pixels per frame                */
  uint32_t num_columns;         /* C                                        */
  uint32_t synapses_per_column; /* S: potential synapses per column         */
  uint32_t min_overlap;         /* m                                        */
  uint32_t winners;             /* k: winners_set_size                      */
  double connected_perm;        /* connected threshold, e.g. 0.5            */
  double perm_inc;              /* learning increment, e.g. 8/256           */
  double perm_dec;              /* learning decrement, e.g. 4/256           */
} spo_config;

/* Algorithm 1.  idx and perm are [C][S] row-major; frame is ceil(N/32)
 * words.  Writes overlap[C]. */
void spo_overlap(const spo_config* cfg, const uint32_t* idx, const double* perm,
                 const uint32_t* frame, int32_t* overlap);

/* Algorithm 2, global form (R4).  Writes active[C] (0/1) and
 * winners[k] in ascending column order padded with -1; returns the number
 * of winners. */
int spo_inhibit(const spo_config* cfg, const int32_t* overlap, uint8_t* active,
                int32_t* winners);

/* Learning (R5) on the columns flagged in active[C]; updates perm in place. */
void spo_learn(const spo_config* cfg, const uint32_t* idx, double* perm,
               const uint32_t* frame, const uint8_t* active);

/* F frames in order (frames is [F][ceil(N/32)]): overlap, inhibition and,
 * when learn != 0, learning, the state after frame t feeding frame t + 1.
 * overlaps is [F][C] (may be NULL), winners is [F][k].  Returns 0, or -1 on
 * a bad argument. */
int spo_run(const spo_config* cfg, const uint32_t* idx, double* perm,
            const uint32_t* frames, uint32_t num_frames, int learn,
            int32_t* overlaps, int32_t* winners);

/* Local inhibition, Algorithm 2 as printed (the radius form Section 3.2.2
 * describes), on one frame's gated overlaps.  Columns sit on a grid of
 * grid_w columns per row (row-major; C need not fill the last row).  The
 * neighbourhood of c is every other column d whose row and column
 * coordinates differ from c's by at most `radius` (no wrap-around); the
 * n-th largest overlap among the neighbours (0 when there are fewer than n)
 * gives max_column = max(that, 1), and c is active iff its overlap >
 * max_column.  Readings L1-L4 (grid, neighbourhood without c, strict
 * comparison, the 1 floor) are listed in the design notes.  Writes
 * active[C]; returns the number of active columns, -1 on a bad argument. */
int spo_inhibit_local(const int32_t* overlap, uint32_t C, uint32_t grid_w, uint32_t radius,
                      uint32_t n, uint8_t* active);

/* F frames in order with local inhibition: overlap (Algorithm 1), local
 * inhibition, and, when learn != 0, learning (R5) on the active columns.
 * overlaps [F][C] may be NULL; active is [F][C].  Returns 0, -1 on a bad
 * argument. */
int spo_run_local(const spo_config* cfg, const uint32_t* idx, double* perm,
                  const uint32_t* frames, uint32_t num_frames, int learn, uint32_t grid_w,
                  uint32_t radius, uint32_t n, int32_t* overlaps, uint8_t* active);

/* Inhibition radius adaptation (Section 4.4: a change of winners_set_size
 * is compensated by adapting the inhibition radius, which the paper takes
 * from the whitepaper; its rule sets the radius, after each learning frame,
 * to the average connected receptive field size of the columns).  Reading
 * L5: the input is an image of in_w pixels per row (pixel p at x = p mod
 * in_w, y = p div in_w, in_h = ceil(N / in_w) rows) and the columns a grid
 * of grid_w per row (grid_h = ceil(C / grid_w) rows).  A column with at
 * least one connected synapse has the extent span_x = max x - min x + 1 and
 * span_y = max y - min y + 1 of its connected inputs; over the n such
 * columns the mean extent is A / (2 n), A = sum of span_x + span_y; it is
 * carried to the column grid by the mean of the two grid-per-input ratios,
 * (grid_w / in_w + grid_h / in_h) / 2, giving a diameter d, and the radius
 * is (d - 1) / 2 rounded half up, at least 1:
 *   radius = max(1, floor(A (grid_w in_h + grid_h in_w) / (8 n in_w in_h))).
 * With no connected synapse anywhere (n = 0) the radius stays as it was.
 * Returns the new radius. */
uint32_t spo_adapt_radius(const spo_config* cfg, const uint32_t* idx, const double* perm,
                          uint32_t in_w, uint32_t grid_w, uint32_t radius);

/* spo_run_local with the radius adapted after every learning frame: frame t
 * uses the radius left by frame t - 1 (the first frame uses `radius`);
 * radii [F] (may be NULL) receives the radius each frame used.  Returns the
 * radius after the last frame, or 0 on a bad argument. */
uint32_t spo_run_local_adaptive(const spo_config* cfg, const uint32_t* idx, double* perm,
                                const uint32_t* frames, uint32_t num_frames, int learn,
                                uint32_t in_w, uint32_t grid_w, uint32_t radius, uint32_t n,
                                int32_t* overlaps, uint8_t* active, uint32_t* radii);

/* Boosting and duty cycles (Algorithm 1 multiplies each gated overlap by the
 * column's boost, which Section 3.2.2 computes in the kernel; the update
 * rules are the whitepaper's, spatial pooler phase 3), in exact fixed
 * point (readings B1-B7 of the design notes):
 *   B1 boost b[c] in 1/256 units (>= 256); the inhibition ranks the boosted
 *      overlaps ov[c] * b[c] (R4: global top-k, ties to the lower index);
 *   B2 duty cycles in 1/65536 units, after each learning frame
 *      d <- floor((d (P - 1) + 65536 e) / P), P = 2^period_log2, with e = 1
 *      iff the column won (active duty cycle) or iff its gated overlap is
 *      positive (overlap duty cycle);
 *   B3 min duty cycle = floor(max over all columns of the active duty cycle
 *      * min_pct_q16 / 65536) (global inhibition: every column is a
 *      neighbour);
 *   B4 b[c] = 256 if min == 0 or active duty >= min, else
 *      256 + floor((max_boost_q8 - 256) (min - duty) / min);
 *   B5 a column whose overlap duty cycle is below the min has every
 *      permanence raised by bump_q8 / 256, clipped at 1;
 *   B6 per frame: boosted overlap with the boosts of the previous frame,
 *      inhibition, learning of the winners, duty cycles, min, boosts, bumps;
 *   B7 learn = 0 changes nothing (permanences, duty cycles, boosts). */
typedef struct spo_boost {
  uint32_t period_log2;  /* P = 2^period_log2, 0..16                       */
  uint32_t min_pct_q16;  /* min duty cycle as a fraction of the max, /65536 */
  uint32_t max_boost_q8; /* boost at duty cycle 0, 256..4096                */
  uint32_t bump_q8;      /* permanence raise on a low overlap duty cycle    */
} spo_boost;

/* F frames in order with boosting.  adc, odc (duty cycles) and boost
 * ([C] each) hold the state and are updated in place; overlaps [F][C] (the
 * boosted overlaps, may be NULL) and winners [F][k] are written.  Returns 0,
 * -1 on a bad argument. */
int spo_run_boost(const spo_config* cfg, const spo_boost* bc, const uint32_t* idx, double* perm,
                  const uint32_t* frames, uint32_t num_frames, int learn, uint32_t* adc,
                  uint32_t* odc, uint32_t* boost, int32_t* overlaps, int32_t* winners);

/* Per-stream SDR histogram (Section 2: the pooler's output of every frame of
 * a video is accumulated into a histogram that serves as the video's
 * feature vector).  For every frame t < num_frames and every entry
 * c = winners[t][j] >= 0, adds 1 to hist[c]; hist[C] is not cleared first.
 * Returns 0, or -1 on an entry >= C. */
/* spo_run on `threads` host threads (1..1024), with the same results: the
 * overlap and the learning of each frame split by contiguous column ranges,
 * the inhibition on one thread (sp_oracle_mt.c). */
int spo_run_threads(const spo_config* cfg, const uint32_t* idx, double* perm,
                    const uint32_t* frames, uint32_t num_frames, int learn, int32_t* overlaps,
                    int32_t* winners, uint32_t threads);

int spo_histogram(const int32_t* winners, uint32_t num_frames, uint32_t k, uint32_t C,
                  uint32_t* hist);

#ifdef __cplusplus
}
#endif

#endif
