// Pool kernels: one launch per class walks that class's work list of
// (solve, tile) items drawn from many grids of different sizes, one item per
// workgroup, and advances every running solve by one iteration; two
// bookkeeping launches per advance take the solves' gap decisions (after the
// first step, whose sweeps carry the gaps) and move their counters on (after
// the last).  The tile bodies
// are the same device functions as the single-solve kernels, so a solve
// produces the same bits in the pool, alone or in any mix, and through the
// single-solve API with the same tile shape.
#include <type_traits>

#include "mf_pool.h"
#include "tile2d.h"
#include "tile2d_d2.h"
#include "tile3d.h"

namespace mf {

// Work item of this workgroup, or -1.  The list is cut into 8 contiguous
// chunks and the workgroups dispatched to one XCD (block b runs on XCD b & 7)
// take the items of one chunk, so neighbouring tiles of a grid share that
// XCD's L2.  The launch's grid is a capacity of at least 8 * ceil(n / 8)
// workgroups that only grows (the pool's graphs are cached per class set);
// workgroups past the items return at once.  One item per workgroup: a loop
// over several items per workgroup doubles the register footprint of the
// tile bodies (the compiler keeps the next item's state live) and costs
// occupancy.
__device__ __forceinline__ int xcd_item(int n) {
  const int b = blockIdx.x, x = b & 7;
  const int it = (int)((long long)n * x / 8) + (b >> 3);
  return it < (int)((long long)n * (x + 1) / 8) ? it : -1;
}

// A launch at step `step` of an advance takes the slot's iterate
// sl.iter + step (sl.iter: the iterate at the start of the advance); its
// state buffer:
__device__ __forceinline__ int slot_buf(const PoolSlot& sl, int step) {
  return (int)(((sl.iter + step) / sl.bufdiv) & 1);
}

template <typename TS>
__device__ __forceinline__ K2<TS> slot_k2(const PoolSlot& sl, int step) {
  K2<TS> a;
  const int src = slot_buf(sl, step), dst = src ^ 1;
  a.W = sl.W;
  a.H = sl.H;
  a.pitch = sl.pitch;
  a.P = sl.P;
  a.tiles_x = sl.tiles_x;
  a.cap = (const TS*)sl.cap;
  a.u_in = sl.st[src].u;
  a.u_out = sl.st[dst].u;
  a.q_in = (const TS*)sl.st[src].q;
  a.q_out = (TS*)sl.st[dst].q;
  a.ps_in = (const TS*)sl.st[src].ps;
  a.ps_out = (TS*)sl.st[dst].ps;
  a.p_in = (const TS*)sl.st[src].p;
  a.p_out = (TS*)sl.st[dst].p;
  a.wbuf = nullptr;
  a.k = sl.k;
  a.acc = nullptr;
  a.done = nullptr;
  a.write = sl.iter + step < sl.max_iter ? 1 : 0;
  a.iso = sl.iso;
  a.strip = 1 << 30;
  a.nt = 0;
  return a;
}

// CHECK selects the items this launch processes: the sweeps that also
// accumulate the gap of their input iterate (solves at a check), or all the
// others.  Two specialised launches keep the common no-gap body lean.
template <int NL, bool TWO, typename TS, int TY, bool CHECK, bool VEC>
__global__ __launch_bounds__(256) void k_pool2d(PoolDev d, int cls, int step) {
  __shared__ Smem2<TY, CHECK, CHECK && !TWO> S;
  const int it = xcd_item(d.counts[cls]);
  if (it < 0) return;
  const WorkItem w = d.items[cls][it];
  PoolSlot* sl = d.slots + w.slot;
  if (sl->state != SLOT_RUNNING) return;
  // the gap of a checking solve's input iterate is fused into its sweep
  const bool check = sl->check_now != 0;
  if (check != CHECK) return;
  const K2<TS> A = slot_k2<TS>(*sl, step);
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (d1_interior<TY>(w.x0, w.y0, A.W, A.H)) tile2d<NL, TWO, TS, CHECK, TY, VEC, CHECK, false, false>(A, w.x0, w.y0, S, g);
  else tile2d<NL, TWO, TS, CHECK, TY, VEC, CHECK, false, true>(A, w.x0, w.y0, S, g);
  if (CHECK) block_accumulate<5, 4>(g, &sl->acc[0][0], S.sred);
}

// Two iterations (k -> k+2) of a two-label 2-D solve per launch, iterate
// k+1 kept in LDS (the depth-2 tile body); iterate k is in buffer
// (k / 2) & 1 and k+2 goes to the other one.
template <typename TS, int TY, bool CHECK>
__global__ __launch_bounds__(256) void k_pool2d_d2(PoolDev d, int cls, int step) {
  __shared__ Smem2d2<TY> S;
  const int it = xcd_item(d.counts[cls]);
  if (it < 0) return;
  const WorkItem w = d.items[cls][it];
  PoolSlot* sl = d.slots + w.slot;
  if (sl->state != SLOT_RUNNING) return;
  if ((sl->check_now != 0) != CHECK) return;
  const K2<TS> A = slot_k2<TS>(*sl, step);
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (d2_interior<TY>(w.x0, w.y0, A.W, A.H)) tile2d_d2<TS, CHECK, TY, false, false>(A, w.x0, w.y0, S, g);
  else tile2d_d2<TS, CHECK, TY, false, true>(A, w.x0, w.y0, S, g);
  if (CHECK) block_accumulate<5, 4>(g, &sl->acc[0][0], S.sred);
}

template <typename TS, bool CHECK, bool VEC>
__global__ __launch_bounds__(256) void k_pool3d(PoolDev d, int cls, int step) {
  __shared__ Smem3<CHECK> S;
  const int it = xcd_item(d.counts[cls]);
  if (it < 0) return;
  const WorkItem w = d.items[cls][it];
  PoolSlot* sl = d.slots + w.slot;
  if (sl->state != SLOT_RUNNING) return;
  if ((sl->check_now != 0) != CHECK) return;
  {
    K3<TS> A;
    const int src = slot_buf(*sl, step), dst = src ^ 1;
    A.W = sl->W;
    A.H = sl->H;
    A.D = sl->D;
    A.pitch = sl->pitch;
    A.P = sl->P;
    A.SZ = (long long)sl->pitch * sl->H;
    A.tiles_x = sl->tiles_x;
    A.tiles_y = sl->tiles_y;
    A.tz = sl->tz;
    A.cap = (const TS*)sl->cap;
    A.u_in = sl->st[src].u;
    A.u_out = sl->st[dst].u;
    A.q_in = (const TS*)sl->st[src].q;
    A.q_out = (TS*)sl->st[dst].q;
    A.ps_in = (const TS*)sl->st[src].ps;
    A.ps_out = (TS*)sl->st[dst].ps;
    A.p_in = (const TS*)sl->st[src].p;
    A.p_out = (TS*)sl->st[dst].p;
    A.k = sl->k;
    A.acc = nullptr;
    A.done = nullptr;
    A.write = sl->iter + step < sl->max_iter ? 1 : 0;
    A.iso = sl->iso;
    A.strip = 1 << 30;
    A.nt = 0;
    const int z1 = min(w.z0 + A.tz, A.D);
    double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    tile3d<TS, CHECK, VEC, CHECK>(A, w.x0, w.y0, w.z0, z1, S, g);
    if (CHECK) block_accumulate<5, 4>(g, &sl->acc[0][0], S.sred);
  }
}

// One workgroup (64 threads) per slot.  Two launches per advance:
//   decide (after the first step, whose launches carried the gaps): sum the
//     64 accumulator rows of every checking slot, clear them, decide
//     (converged / cap reached / diverged / promote) and publish the gap;
//     a slot that keeps running stops checking for the rest of the advance;
//   advance_by > 0 (after the last step): every running slot's iterate
//     moves on by the advance's iterations, its next check is set up and
//     its status published.
// A stopped or frozen slot keeps the iterate its check accepted: the first
// step wrote only the other buffer, and later launches skip it.  Status
// codes follow mf_status: 0 converged, 1 cap reached, -4 diverged.
__global__ __launch_bounds__(64) void k_pool_book(PoolDev d, int decide, int advance_by) {
  PoolSlot* sl = d.slots + blockIdx.x;
  const int t = threadIdx.x;
  if (sl->state != SLOT_RUNNING) return;
  if (decide) {
    if (!sl->check_now) return;
    double v[5];
#pragma unroll
    for (int j = 0; j < 5; j++) v[j] = wave_total(sl->acc[t][j]);
#pragma unroll
    for (int j = 0; j < 8; j++) sl->acc[t][j] = 0.0;
    if (t != 0) return;
    const long long k = sl->iter;
    int state = SLOT_RUNNING;
    const double P = v[0] + sl->alpha * v[1];
    const double D = v[2];
    const double m = fmax(fmax(fabs(P), fabs(D)), 1e-300);
    const double rel = (P - D) / m;
    PoolStat& ps = d.stats[blockIdx.x];
    ps.last[0] = P;
    ps.last[1] = D;
    ps.last[2] = rel;
    ps.last[3] = sqrt(v[3] / (double)sl->nres);
    ps.last[4] = v[4];
    ps.last[5] = (double)k;
    const bool bad = !isfinite(P) || !isfinite(D) || !isfinite(v[3]) || rel < -neg_gap_tol(sl->bf16 != 0);
    if (bad) {
      state = SLOT_DONE;
      sl->status = -4;
    } else if (rel <= sl->tol) {
      state = SLOT_DONE;
      sl->status = 0;
    } else if (k >= sl->max_iter) {
      state = SLOT_DONE;
      sl->status = 1;
    } else if (sl->bf16 && ((sl->promote_gap > 0.0 && rel <= sl->promote_gap) ||
                            (sl->promote_iter > 0 && k >= sl->promote_iter))) {
      state = SLOT_PROMOTE;   // frozen at k until the host moves it to FP32 storage
    }
    sl->check_now = 0;
    sl->state = state;
    ps.state = state;
    ps.status = sl->status;
    ps.iter = k;
    return;
  }
  if (t != 0) return;
  const long long kn = sl->iter + advance_by;
  sl->iter = kn;
  sl->check_now = (kn % sl->check_every == 0 || kn >= sl->max_iter) ? 1 : 0;
  d.stats[blockIdx.x].state = sl->state;
  d.stats[blockIdx.x].status = sl->status;
  d.stats[blockIdx.x].iter = kn;
}

// Kernel of one (class, gap-carrying, vector-aligned) launch.
template <typename TS, bool CHECK, bool VEC>
static const void* pool_kernel_ts(int model) {
  constexpr bool BF = std::is_same<TS, bf16_t>::value;
  if (CHECK) {
    switch (model) {
      case 0: return (const void*)k_pool2d<1, true, TS, pool_tile_rows(0, BF), true, VEC>;
      case 1: return (const void*)k_pool2d<2, false, TS, pool_tile_rows(1, BF), true, VEC>;
      case 2: return (const void*)k_pool2d<3, false, TS, pool_tile_rows(2, BF), true, VEC>;
      case 3: return (const void*)k_pool2d<4, false, TS, pool_tile_rows(3, BF), true, VEC>;
      case 4: return (const void*)k_pool2d<8, false, TS, pool_tile_rows(4, BF), true, VEC>;
      default: return (const void*)k_pool3d<TS, true, VEC>;
    }
  }
  switch (model) {
    case 0: return (const void*)k_pool2d<1, true, TS, pool_tile_rows(0, BF), false, VEC>;
    case 1: return (const void*)k_pool2d<2, false, TS, pool_tile_rows(1, BF), false, VEC>;
    case 2: return (const void*)k_pool2d<3, false, TS, pool_tile_rows(2, BF), false, VEC>;
    case 3: return (const void*)k_pool2d<4, false, TS, pool_tile_rows(3, BF), false, VEC>;
    case 4: return (const void*)k_pool2d<8, false, TS, pool_tile_rows(4, BF), false, VEC>;
    default: return (const void*)k_pool3d<TS, false, VEC>;
  }
}

const void* pool_kernel(int cls, bool check, bool vec) {
  const int model = cls % kPoolModels;
  const bool bf16 = cls >= kPoolModels;
  if (bf16) {
    if (check) return vec ? pool_kernel_ts<bf16_t, true, true>(model) : pool_kernel_ts<bf16_t, true, false>(model);
    return vec ? pool_kernel_ts<bf16_t, false, true>(model) : pool_kernel_ts<bf16_t, false, false>(model);
  }
  if (check) return vec ? pool_kernel_ts<float, true, true>(model) : pool_kernel_ts<float, true, false>(model);
  return vec ? pool_kernel_ts<float, false, true>(model) : pool_kernel_ts<float, false, false>(model);
}

const void* pool_kernel_d2(int cls, bool check) {
  const int model = cls % kPoolModels;
  if (model != 0) return nullptr;
  constexpr int TY = pool_tile_rows(0, false);
  static_assert(pool_tile_rows(0, false) == pool_tile_rows(0, true), "one tile height for both storages");
  if (cls >= kPoolModels)
    return check ? (const void*)k_pool2d_d2<bf16_t, TY, true> : (const void*)k_pool2d_d2<bf16_t, TY, false>;
  return check ? (const void*)k_pool2d_d2<float, TY, true> : (const void*)k_pool2d_d2<float, TY, false>;
}

const void* pool_book_kernel() { return (const void*)k_pool_book; }

}  // namespace mf
