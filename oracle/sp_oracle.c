/*
 * Oracle for the HTM spatial pooler step -- TEST INFRASTRUCTURE ONLY.
 * See sp_oracle.h for the paper passages followed and the readings R1-R6.
 * Each function below is the definition written out, with no blocking,
 * fusion or reordering beyond the paper's own order of steps.
 */
#include "sp_oracle.h"

#include <stdlib.h>
#include <string.h>

/* R6: input pixel p of a frame is bit (p & 31) of word (p >> 5). */
static int input_active(const uint32_t* frame, uint32_t p) {
  return (int)((frame[p >> 5] >> (p & 31u)) & 1u);
}

/* R1: the synapse is connected when its permanence reaches the threshold. */
static int synapse_connected(const spo_config* cfg, double perm) {
  return perm >= cfg->connected_perm;
}

/* Section 1.1, Algorithm 1: for every column, count its connected synapses
 * whose input is active; a count below min_overlap becomes 0 (R2), any other
 * count is multiplied by the column's boost, which is 1 here (R3). */
void spo_overlap(const spo_config* cfg, const uint32_t* idx, const double* perm,
                 const uint32_t* frame, int32_t* overlap) {
  const uint32_t C = cfg->num_columns, S = cfg->synapses_per_column;
  for (uint32_t c = 0; c < C; ++c) {
    int32_t ov = 0;
    for (uint32_t s = 0; s < S; ++s) {
      const size_t syn = (size_t)c * S + s;
      if (synapse_connected(cfg, perm[syn])) ov += input_active(frame, idx[syn]);
    }
    if (ov < (int32_t)cfg->min_overlap) {
      ov = 0;
    } else {
      const int32_t boost = 1;
      ov = ov * boost;
    }
    overlap[c] = ov;
  }
}

/* Section 1.1, Algorithm 2, global form (R4): winners_set_size rounds, each
 * taking the not-yet-active column of highest overlap; scanning columns in
 * index order with a strict comparison gives ties to the lower index.  A
 * round that finds no column with positive overlap ends the selection. */
int spo_inhibit(const spo_config* cfg, const int32_t* overlap, uint8_t* active,
                int32_t* winners) {
  const uint32_t C = cfg->num_columns, k = cfg->winners;
  memset(active, 0, C);
  int count = 0;
  for (uint32_t round = 0; round < k; ++round) {
    int32_t best = -1;
    int32_t best_ov = 0;
    for (uint32_t c = 0; c < C; ++c) {
      if (!active[c] && overlap[c] > best_ov) {
        best = (int32_t)c;
        best_ov = overlap[c];
      }
    }
    if (best < 0) break;
    active[best] = 1;
    ++count;
  }
  uint32_t w = 0;
  for (uint32_t c = 0; c < C; ++c)
    if (active[c]) winners[w++] = (int32_t)c;
  for (; w < k; ++w) winners[w] = -1;
  return count;
}

/* Learning (R5), the whitepaper's spatial pooler phase 3: for each active
 * column, each potential synapse is strengthened if its input bit is on and
 * weakened otherwise, the permanence staying within [0, 1]. */
void spo_learn(const spo_config* cfg, const uint32_t* idx, double* perm,
               const uint32_t* frame, const uint8_t* active) {
  const uint32_t C = cfg->num_columns, S = cfg->synapses_per_column;
  for (uint32_t c = 0; c < C; ++c) {
    if (!active[c]) continue;
    for (uint32_t s = 0; s < S; ++s) {
      const size_t syn = (size_t)c * S + s;
      double p = perm[syn];
      if (input_active(frame, idx[syn])) {
        p = p + cfg->perm_inc;
        if (p > 1.0) p = 1.0;
      } else {
        p = p - cfg->perm_dec;
        if (p < 0.0) p = 0.0;
      }
      perm[syn] = p;
    }
  }
}

int spo_run(const spo_config* cfg, const uint32_t* idx, double* perm,
            const uint32_t* frames, uint32_t num_frames, int learn,
            int32_t* overlaps, int32_t* winners) {
  if (!cfg || !idx || !perm || (!frames && num_frames) || (!winners && num_frames)) return -1;
  const uint32_t C = cfg->num_columns, k = cfg->winners;
  if (C == 0 || cfg->synapses_per_column == 0 || k == 0 || k > C || cfg->input_bits == 0)
    return -1;
  const size_t W = ((size_t)cfg->input_bits + 31) / 32;
  for (size_t i = 0; i < (size_t)C * cfg->synapses_per_column; ++i)
    if (idx[i] >= cfg->input_bits) return -1;
  int32_t* ov = (int32_t*)malloc(sizeof(int32_t) * C);
  uint8_t* active = (uint8_t*)malloc(C);
  if (!ov || !active) {
    free(ov);
    free(active);
    return -1;
  }
  for (uint32_t t = 0; t < num_frames; ++t) {
    const uint32_t* frame = frames + (size_t)t * W;
    spo_overlap(cfg, idx, perm, frame, ov);
    spo_inhibit(cfg, ov, active, winners + (size_t)t * k);
    if (learn) spo_learn(cfg, idx, perm, frame, active);
    if (overlaps) memcpy(overlaps + (size_t)t * C, ov, sizeof(int32_t) * C);
  }
  free(ov);
  free(active);
  return 0;
}

int spo_histogram(const int32_t* winners, uint32_t num_frames, uint32_t k, uint32_t C,
                  uint32_t* hist) {
  for (uint32_t t = 0; t < num_frames; ++t) {
    for (uint32_t j = 0; j < k; ++j) {
      const int32_t c = winners[(size_t)t * k + j];
      if (c < 0) continue; /* padding after the last winner */
      if ((uint32_t)c >= C) return -1;
      hist[c] += 1;
    }
  }
  return 0;
}

static int cmp_desc(const void* a, const void* b) {
  const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x < y) - (x > y);
}

int spo_inhibit_local(const int32_t* overlap, uint32_t C, uint32_t grid_w, uint32_t radius,
                      uint32_t n, uint8_t* active) {
  if (C == 0 || grid_w == 0 || n == 0) return -1;
  int32_t* nb = (int32_t*)malloc(sizeof(int32_t) * C);
  if (!nb) return -1;
  int count = 0;
  for (uint32_t c = 0; c < C; ++c) {
    const int64_t cx = c % grid_w, cy = c / grid_w;
    uint32_t m = 0;
    for (uint32_t d = 0; d < C; ++d) {
      if (d == c) continue;
      const int64_t dx = (int64_t)(d % grid_w) - cx, dy = (int64_t)(d / grid_w) - cy;
      if (dx <= (int64_t)radius && -dx <= (int64_t)radius && dy <= (int64_t)radius &&
          -dy <= (int64_t)radius)
        nb[m++] = overlap[d];
    }
    /* n_max_overlap: the n-th largest neighbour overlap */
    qsort(nb, m, sizeof(int32_t), cmp_desc);
    const int32_t nth = m >= n ? nb[n - 1] : 0;
    const int32_t max_column = nth > 1 ? nth : 1;
    active[c] = overlap[c] > max_column ? 1 : 0;
    count += active[c];
  }
  free(nb);
  return count;
}

int spo_run_local(const spo_config* cfg, const uint32_t* idx, double* perm,
                  const uint32_t* frames, uint32_t num_frames, int learn, uint32_t grid_w,
                  uint32_t radius, uint32_t n, int32_t* overlaps, uint8_t* active) {
  if (!cfg || !idx || !perm || (!frames && num_frames) || (!active && num_frames)) return -1;
  const uint32_t C = cfg->num_columns;
  if (C == 0 || cfg->synapses_per_column == 0 || cfg->input_bits == 0 || grid_w == 0 || n == 0)
    return -1;
  const size_t W = ((size_t)cfg->input_bits + 31) / 32;
  for (size_t i = 0; i < (size_t)C * cfg->synapses_per_column; ++i)
    if (idx[i] >= cfg->input_bits) return -1;
  int32_t* ov = (int32_t*)malloc(sizeof(int32_t) * C);
  if (!ov) return -1;
  for (uint32_t t = 0; t < num_frames; ++t) {
    const uint32_t* frame = frames + (size_t)t * W;
    uint8_t* act = active + (size_t)t * C;
    spo_overlap(cfg, idx, perm, frame, ov);
    spo_inhibit_local(ov, C, grid_w, radius, n, act);
    if (learn) spo_learn(cfg, idx, perm, frame, act);
    if (overlaps) memcpy(overlaps + (size_t)t * C, ov, sizeof(int32_t) * C);
  }
  free(ov);
  return 0;
}

uint32_t spo_adapt_radius(const spo_config* cfg, const uint32_t* idx, const double* perm,
                          uint32_t in_w, uint32_t grid_w, uint32_t radius) {
  const uint32_t C = cfg->num_columns, S = cfg->synapses_per_column, N = cfg->input_bits;
  const uint64_t in_h = ((uint64_t)N + in_w - 1) / in_w;
  const uint64_t grid_h = ((uint64_t)C + grid_w - 1) / grid_w;
  uint64_t A = 0, n = 0;
  for (uint32_t c = 0; c < C; ++c) {
    uint32_t x0 = 0, x1 = 0, y0 = 0, y1 = 0;
    int any = 0;
    for (uint32_t s = 0; s < S; ++s) {
      const size_t syn = (size_t)c * S + s;
      if (!synapse_connected(cfg, perm[syn])) continue;
      const uint32_t x = idx[syn] % in_w, y = idx[syn] / in_w;
      if (!any || x < x0) x0 = x;
      if (!any || x > x1) x1 = x;
      if (!any || y < y0) y0 = y;
      if (!any || y > y1) y1 = y;
      any = 1;
    }
    if (!any) continue;
    A += (uint64_t)(x1 - x0 + 1) + (uint64_t)(y1 - y0 + 1);
    n += 1;
  }
  if (n == 0) return radius;
  const unsigned __int128 num =
      (unsigned __int128)A * ((uint64_t)grid_w * in_h + grid_h * (uint64_t)in_w);
  const unsigned __int128 den = (unsigned __int128)8 * n * in_w * in_h;
  const uint64_t r = (uint64_t)(num / den);
  return r < 1 ? 1u : (r > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)r);
}

uint32_t spo_run_local_adaptive(const spo_config* cfg, const uint32_t* idx, double* perm,
                                const uint32_t* frames, uint32_t num_frames, int learn,
                                uint32_t in_w, uint32_t grid_w, uint32_t radius, uint32_t n,
                                int32_t* overlaps, uint8_t* active, uint32_t* radii) {
  if (!cfg || !idx || !perm || (!frames && num_frames) || (!active && num_frames)) return 0;
  const uint32_t C = cfg->num_columns;
  if (C == 0 || cfg->synapses_per_column == 0 || cfg->input_bits == 0 || grid_w == 0 ||
      grid_w > C || in_w == 0 || in_w > cfg->input_bits || n == 0 || radius == 0)
    return 0;
  const size_t W = ((size_t)cfg->input_bits + 31) / 32;
  for (size_t i = 0; i < (size_t)C * cfg->synapses_per_column; ++i)
    if (idx[i] >= cfg->input_bits) return 0;
  int32_t* ov = (int32_t*)malloc(sizeof(int32_t) * C);
  if (!ov) return 0;
  for (uint32_t t = 0; t < num_frames; ++t) {
    const uint32_t* frame = frames + (size_t)t * W;
    uint8_t* act = active + (size_t)t * C;
    if (radii) radii[t] = radius;
    spo_overlap(cfg, idx, perm, frame, ov);
    spo_inhibit_local(ov, C, grid_w, radius, n, act);
    if (learn) {
      spo_learn(cfg, idx, perm, frame, act);
      radius = spo_adapt_radius(cfg, idx, perm, in_w, grid_w, radius);
    }
    if (overlaps) memcpy(overlaps + (size_t)t * C, ov, sizeof(int32_t) * C);
  }
  free(ov);
  return radius;
}

int spo_run_boost(const spo_config* cfg, const spo_boost* bc, const uint32_t* idx, double* perm,
                  const uint32_t* frames, uint32_t num_frames, int learn, uint32_t* adc,
                  uint32_t* odc, uint32_t* boost, int32_t* overlaps, int32_t* winners) {
  if (!cfg || !bc || !idx || !perm || !adc || !odc || !boost) return -1;
  if ((!frames || !winners) && num_frames) return -1;
  const uint32_t C = cfg->num_columns, S = cfg->synapses_per_column, k = cfg->winners;
  if (C == 0 || S == 0 || k == 0 || k > C || cfg->input_bits == 0) return -1;
  if (bc->period_log2 > 16 || bc->max_boost_q8 < 256 || bc->max_boost_q8 > 4096 ||
      bc->min_pct_q16 > 65536 || bc->bump_q8 > 256)
    return -1;
  const size_t W = ((size_t)cfg->input_bits + 31) / 32;
  for (size_t i = 0; i < (size_t)C * S; ++i)
    if (idx[i] >= cfg->input_bits) return -1;
  const uint64_t P = 1ull << bc->period_log2;
  int32_t* ov = (int32_t*)malloc(sizeof(int32_t) * C);
  int32_t* bov = (int32_t*)malloc(sizeof(int32_t) * C);
  uint8_t* active = (uint8_t*)malloc(C);
  if (!ov || !bov || !active) {
    free(ov);
    free(bov);
    free(active);
    return -1;
  }
  for (uint32_t t = 0; t < num_frames; ++t) {
    const uint32_t* frame = frames + (size_t)t * W;
    /* B1: boosted overlaps, then the global inhibition on them */
    spo_overlap(cfg, idx, perm, frame, ov);
    for (uint32_t c = 0; c < C; ++c) bov[c] = ov[c] * (int32_t)boost[c];
    spo_inhibit(cfg, bov, active, winners + (size_t)t * k);
    if (overlaps) memcpy(overlaps + (size_t)t * C, bov, sizeof(int32_t) * C);
    if (!learn) continue; /* B7 */
    spo_learn(cfg, idx, perm, frame, active);
    /* B2: duty cycles */
    uint32_t max_adc = 0;
    for (uint32_t c = 0; c < C; ++c) {
      adc[c] = (uint32_t)(((uint64_t)adc[c] * (P - 1) + (active[c] ? 65536u : 0u)) / P);
      odc[c] = (uint32_t)(((uint64_t)odc[c] * (P - 1) + (ov[c] > 0 ? 65536u : 0u)) / P);
      if (adc[c] > max_adc) max_adc = adc[c];
    }
    /* B3: the minimum duty cycle */
    const uint32_t min_dc = (uint32_t)(((uint64_t)max_adc * bc->min_pct_q16) >> 16);
    for (uint32_t c = 0; c < C; ++c) {
      /* B4: boost, linear below the minimum */
      if (min_dc == 0 || adc[c] >= min_dc)
        boost[c] = 256;
      else
        boost[c] = 256 + (uint32_t)(((uint64_t)(bc->max_boost_q8 - 256) * (min_dc - adc[c])) /
                                    min_dc);
      /* B5: a column that rarely overlaps gets all its permanences raised */
      if (odc[c] < min_dc)
        for (uint32_t s2 = 0; s2 < S; ++s2) {
          double* p = &perm[(size_t)c * S + s2];
          *p += bc->bump_q8 / 256.0;
          if (*p > 1.0) *p = 1.0;
        }
    }
  }
  free(ov);
  free(bov);
  free(active);
  return 0;
}
