/*
 * The oracle on several host threads -- TEST INFRASTRUCTURE ONLY (the CPU
 * baseline of the benchmark at all host cores).  It adds no arithmetic of
 * its own: per frame, each thread runs spo_overlap on a contiguous range of
 * columns (a column's overlap depends only on that column, Algorithm 1),
 * one thread runs spo_inhibit over every column (Algorithm 2 needs all
 * overlaps), then each thread runs spo_learn on its range (learning changes
 * only the winners' own synapses).  The results equal spo_run's exactly; the
 * tests check that for several thread counts.
 */
#define _POSIX_C_SOURCE 200809L
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#include "sp_oracle.h"

typedef struct {
  const spo_config* cfg;
  const uint32_t* idx;
  double* perm;
  const uint32_t* frames;
  uint32_t num_frames;
  int learn;
  int32_t* overlaps;
  int32_t* winners;
  int32_t* ov;
  uint8_t* active;
  size_t W;
  uint32_t threads;
  pthread_barrier_t bar;
} mt_job;

typedef struct {
  mt_job* job;
  uint32_t id;
} mt_arg;

/* The columns [c0, c1) of a configuration as a configuration of their own,
 * with idx, perm, overlap and active shifted to the range's first column. */
static spo_config column_range(const spo_config* cfg, uint32_t c0, uint32_t c1) {
  spo_config r = *cfg;
  r.num_columns = c1 - c0;
  return r;
}

static void* mt_worker(void* p) {
  mt_arg* a = (mt_arg*)p;
  mt_job* j = a->job;
  const uint32_t C = j->cfg->num_columns, S = j->cfg->synapses_per_column, k = j->cfg->winners;
  const uint32_t c0 = (uint32_t)((uint64_t)C * a->id / j->threads);
  const uint32_t c1 = (uint32_t)((uint64_t)C * (a->id + 1) / j->threads);
  const spo_config part = column_range(j->cfg, c0, c1);
  const size_t base = (size_t)c0 * S;
  for (uint32_t t = 0; t < j->num_frames; ++t) {
    const uint32_t* frame = j->frames + (size_t)t * j->W;
    if (c1 > c0) spo_overlap(&part, j->idx + base, j->perm + base, frame, j->ov + c0);
    pthread_barrier_wait(&j->bar);
    if (a->id == 0) {
      spo_inhibit(j->cfg, j->ov, j->active, j->winners + (size_t)t * k);
      if (j->overlaps) memcpy(j->overlaps + (size_t)t * C, j->ov, sizeof(int32_t) * C);
    }
    pthread_barrier_wait(&j->bar);
    if (j->learn && c1 > c0) spo_learn(&part, j->idx + base, j->perm + base, frame, j->active + c0);
    pthread_barrier_wait(&j->bar);
  }
  return NULL;
}

int spo_run_threads(const spo_config* cfg, const uint32_t* idx, double* perm,
                    const uint32_t* frames, uint32_t num_frames, int learn, int32_t* overlaps,
                    int32_t* winners, uint32_t threads) {
  if (!cfg || !idx || !perm || (!frames && num_frames) || (!winners && num_frames)) return -1;
  const uint32_t C = cfg->num_columns, k = cfg->winners;
  if (C == 0 || cfg->synapses_per_column == 0 || k == 0 || k > C || cfg->input_bits == 0 ||
      threads == 0 || threads > 1024)
    return -1;
  for (size_t i = 0; i < (size_t)C * cfg->synapses_per_column; ++i)
    if (idx[i] >= cfg->input_bits) return -1;
  mt_job job;
  job.cfg = cfg;
  job.idx = idx;
  job.perm = perm;
  job.frames = frames;
  job.num_frames = num_frames;
  job.learn = learn;
  job.overlaps = overlaps;
  job.winners = winners;
  job.W = ((size_t)cfg->input_bits + 31) / 32;
  job.threads = threads;
  job.ov = (int32_t*)malloc(sizeof(int32_t) * C);
  job.active = (uint8_t*)malloc(C);
  pthread_t* tid = (pthread_t*)malloc(sizeof(pthread_t) * threads);
  mt_arg* args = (mt_arg*)malloc(sizeof(mt_arg) * threads);
  int rc = -1;
  if (job.ov && job.active && tid && args && pthread_barrier_init(&job.bar, NULL, threads) == 0) {
    uint32_t started = 0;
    for (; started < threads; ++started) {
      args[started].job = &job;
      args[started].id = started;
      if (started > 0 && pthread_create(&tid[started], NULL, mt_worker, &args[started]) != 0) break;
    }
    if (started == threads) {
      mt_worker(&args[0]);
      rc = 0;
    } else {
      abort(); /* a partial team would wait at the first barrier for ever */
    }
    for (uint32_t i = 1; i < started; ++i) pthread_join(tid[i], NULL);
    pthread_barrier_destroy(&job.bar);
  }
  free(job.ov);
  free(job.active);
  free(tid);
  free(args);
  return rc;
}
