// Device-resident tables of the batched solver pool.
//
// The pool keeps many solves resident at once.  Each solve owns a slot in a
// device table (geometry, state buffers, iteration counter, gap
// accumulators, decision) and its tiles are items of a per-class device work
// list.  An advance runs `steps` steps; at step h every class launch walks
// its work list and takes each solve's iterate iter + h (iter: the iterate at
// the start of the advance), reading the buffer parity from the slot; with
// depth 2 the two-label 2-D classes run the two-iteration kernel at even
// steps only.  The first step carries the gaps and is followed by one
// bookkeeping launch that takes every checking solve's decision; the last
// step is followed by one that moves every running solve on by `steps`.
// Because all of this state lives in device memory, one hipGraph of the
// advance serves any mix; admission and retirement only edit the tables
// between replays.
#pragma once
#include "mf_kernels.h"

namespace mf {

enum { SLOT_FREE = 0, SLOT_RUNNING = 1, SLOT_DONE = 2, SLOT_PROMOTE = 3 };

// Classes: two-label 2-D, Potts n = 2, 3, 4, 8 (2-D), two-label 3-D; x2 storage.
constexpr int kPoolModels = 6;
// Iterations per advance (the only supported value).
constexpr int kPoolSteps = 10;
constexpr int kPoolClasses = 2 * kPoolModels;

struct PoolSlot {
  int state;          // SLOT_*
  int cls;
  int W, H, D, ndim;
  int nl, two, bf16, iso;
  int pitch;          // row stride (W rounded up to a multiple of 4)
  long long P;        // plane stride (elements)
  int tiles_x, tiles_y, tz, check_every;
  int bufdiv;         // iterate k lives in state buffer (k / bufdiv) & 1 (2: two-iteration passes)
  const void* cap;
  StateView st[2];
  Coef k;
  double alpha, tol;
  long long iter, max_iter, nres;
  int check_now, status;
  double promote_gap;       // BF16 -> FP32 promotion triggers (0: off)
  long long promote_iter;
  double acc[kAccSlots][8];
};

// Compact per-slot status the host polls.
struct PoolStat {
  int state, status;
  long long iter;
  double last[6];     // primal, dual, rel_gap, resid_rms, flow, iter
};

struct WorkItem {
  int slot, x0, y0, z0;
};

struct PoolDev {
  PoolSlot* slots;
  PoolStat* stats;
  WorkItem* items[kPoolClasses];
  int* counts;        // kPoolClasses entries
};

const void* pool_kernel(int cls, bool check, bool vec);
const void* pool_kernel_d2(int cls, bool check);   // two-label 2-D classes
const void* pool_book_kernel();

// Tile height of a 2-D pool class (model index as in the class table; the
// same defaults as single solves: 16 rows, 8 for BF16 Potts with n = 8).
constexpr int pool_tile_rows(int model, bool bf16) { return (model == 4 && bf16) ? 8 : 16; }

}  // namespace mf
