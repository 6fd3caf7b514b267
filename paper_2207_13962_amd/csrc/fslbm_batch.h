// Batched launches for serving: one launch of each step kernel covers every
// resident run of a batch. Run r owns the blocks [blk0, blk0 + nblk) of the
// launch (blk0 a multiple of the XCD count), and its own device arena, Dev
// record and counters; a block finds its run in a table sorted by blk0. A
// run admitted at tick tick0 is at its own step tick - tick0: the parity of
// that step picks which of its two population grids and fill-level buffers
// is read, exactly as the host-side pointer swap does for a single run, so a
// run's arithmetic does not depend on what else shares the launch. Runs past
// their last step return at once (the host retires them between ticks).
#pragma once

#include "fslbm_kernels.h"

namespace fslbm {

struct BatchEntry {
  int32_t slot;    // index of the run's Dev record
  int32_t blk0;    // first block of the run in this launch
  int32_t nblk;    // blocks of the run in this launch
  int32_t a, b;    // per kernel: stream (gen, bord); compact (per, workers)
  int32_t pad;
  int64_t tick0;   // tick of the run's step 0
  int64_t nsteps;  // steps the run takes
};

// The table entry of this block (binary search over blk0).
__device__ __forceinline__ BatchEntry batch_entry(const BatchEntry* tab, int n) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].blk0 <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return tab[lo];
}

// The run's Dev at this tick (grids and fill levels swapped on odd steps; the
// two grid pointers of an in-place run are the same);
// false when the block lies past the run's range or the run is done.
__device__ __forceinline__ bool batch_dev(const Dev* devs, const BatchEntry& e, int64_t tick, Dev& d) {
  const int b = (int)blockIdx.x - e.blk0;
  if (b < 0 || b >= e.nblk) return false;
  const int64_t step = tick - e.tick0;
  if (step < 0 || step >= e.nsteps) return false;
  d = devs[e.slot];
  if (step & 1) {
    void* t = d.fA;
    d.fA = d.fB;
    d.fB = t;
    double* p = d.phiA;
    d.phiA = d.phiB;
    d.phiB = p;
  }
  d.step = step;
  return true;
}

template <int S, int Q, bool TRT, bool BUF, bool AA>
__global__ __launch_bounds__(kBlock) void kb_stream(const Dev* devs, const BatchEntry* tab, int n,
                                                    int64_t tick) {
  const BatchEntry e = batch_entry(tab, n);
  Dev d;
  if (!batch_dev(devs, e, tick, d)) return;
  stream_body<S, Q, TRT, BUF, AA>(d, (int)blockIdx.x - e.blk0, e.nblk, e.a, e.b);
}


template <int Q>
__global__ __launch_bounds__(kBlock) void kb_retype(const Dev* devs, const BatchEntry* tab, int n,
                                                    int64_t tick) {
  const BatchEntry e = batch_entry(tab, n);
  Dev d;
  if (!batch_dev(devs, e, tick, d)) return;
  retype_body<Q>(d, (int)blockIdx.x - e.blk0, e.nblk, 0);
}

template <int S, int Q, bool TRT, bool AA>
__global__ __launch_bounds__(kCompBlock) void kb_compact(const Dev* devs, const BatchEntry* tab, int n,
                                                         int64_t tick) {
  const BatchEntry e = batch_entry(tab, n);
  Dev d;
  if (!batch_dev(devs, e, tick, d)) return;
  compact_body<S, Q, TRT, AA>(d, (int)blockIdx.x - e.blk0, e.nblk, 0, e.a, e.b);
}

#ifdef FSLBM_HOST_KERNELS
// The launches of surface tension (before the streaming launch) and of the
// single-bubble volume pressure (after the compaction) for the runs of a
// batch that have them; their tables list only those runs. Each run's blocks
// do what a single context's launch does with the same block index.
__global__ __launch_bounds__(kBlock) void kb_smooth(const Dev* devs, const BatchEntry* tab, int n, int64_t tick) {
  const BatchEntry e = batch_entry(tab, n);
  Dev d;
  if (!batch_dev(devs, e, tick, d)) return;
  smooth_body(d, (int)blockIdx.x - e.blk0, true);
}

__global__ __launch_bounds__(kBlock) void kb_curvature(const Dev* devs, const BatchEntry* tab, int n,
                                                       int64_t tick) {
  const BatchEntry e = batch_entry(tab, n);
  Dev d;
  if (!batch_dev(devs, e, tick, d)) return;
  curvature_body(d, (int)blockIdx.x - e.blk0, e.nblk);
}

__global__ __launch_bounds__(kBlock) void kb_volume(const Dev* devs, const BatchEntry* tab, int n, int64_t tick) {
  const BatchEntry e = batch_entry(tab, n);
  Dev d;
  if (!batch_dev(devs, e, tick, d)) return;
  reduce_volume_body(d, (int)blockIdx.x - e.blk0, kVolCells);
}

// one block per run
__global__ __launch_bounds__(kBlock) void kb_sum_volume(const Dev* devs, const BatchEntry* tab, int n,
                                                        int64_t tick) {
  const BatchEntry e = batch_entry(tab, n);
  Dev d;
  if (!batch_dev(devs, e, tick, d)) return;
  sum_volume_body(d.partial, (int)vol_blocks_of(d.g.N), d.partial + kRedN * red_blocks_of(d.g.N), d.pV, 0);
}

// The seven passes of tracked bubbles (after the compaction) for the runs of
// a batch that track them; each run has the blocks of its single-context
// launch (one thread per cell, or bub_walk_blocks for the volume and amount
// passes), so its per-wave partial sums are the same.
#define FSLBM_KB_BUB(name, body)                                                                       \
  __global__ __launch_bounds__(kBlock) void name(const Dev* devs, const BatchEntry* tab, int n, int64_t tick) { \
    const BatchEntry e = batch_entry(tab, n);                                                          \
    Dev d;                                                                                             \
    if (!batch_dev(devs, e, tick, d)) return;                                                          \
    body;                                                                                              \
  }
FSLBM_KB_BUB(kb_bub_init, bub_init_body(d, (int)blockIdx.x - e.blk0, 0))
FSLBM_KB_BUB(kb_bub_volume, bub_volume_body(d, (int)blockIdx.x - e.blk0))
FSLBM_KB_BUB(kb_bub_amount, bub_amount_body(d, (int)blockIdx.x - e.blk0))
FSLBM_KB_BUB(kb_bub_target, bub_target_body(d, (int)blockIdx.x - e.blk0))
FSLBM_KB_BUB(kb_bub_pressure, bub_pressure_body(d, (int)blockIdx.x - e.blk0))
FSLBM_KB_BUB(kb_bub_cells, bub_cells_body(d, (int)blockIdx.x - e.blk0))
#undef FSLBM_KB_BUB

template <int Q>
__global__ __launch_bounds__(kBlock) void kb_bub_union(const Dev* devs, const BatchEntry* tab, int n, int64_t tick) {
  const BatchEntry e = batch_entry(tab, n);
  Dev d;
  if (!batch_dev(devs, e, tick, d)) return;
  bub_union_body<Q>(d, (int)blockIdx.x - e.blk0, 0);
}
#endif  // FSLBM_HOST_KERNELS

}  // namespace fslbm
