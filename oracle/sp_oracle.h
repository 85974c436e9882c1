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

/* Per-stream SDR histogram (Section 2: the pooler's output of every frame of
 * a video is accumulated into a histogram that serves as the video's
 * feature vector).  For every frame t < num_frames and every entry
 * c = winners[t][j] >= 0, adds 1 to hist[c]; hist[C] is not cleared first.
 * Returns 0, or -1 on an entry >= C. */
int spo_histogram(const int32_t* winners, uint32_t num_frames, uint32_t k, uint32_t C,
                  uint32_t* hist);

#ifdef __cplusplus
}
#endif

#endif
