// Batched solver pool behind the mf_pool_* part of include/maxflow.h.
//
// The caller hands the pool one device arena.  Its head holds the device
// tables (slot table, per-slot status, per-class work lists and counts); the
// rest is carved first-fit into one block per admitted solve (capacities and
// two state buffers), so admission is decided exactly by footprint.  A step
// launches, for every class as a parallel graph branch, the sweep over the
// class work list (at the first step the variant that also accumulates the
// gap of every checking solve).  With depth 2 the two-label 2-D classes run a two-iteration pass
// at even steps and sit out the odd ones.  Bookkeeping runs twice per
// advance: after the first step (decisions) and after the last (counters).
// The steps of one advance (steps_per_advance iterations) form one hipGraph
// per set of classes, replayed by every mf_pool_advance while that set is
// running.  A class node's grid is a per-class capacity that only grows
// (doubling when the class's item count passes it); workgroups past the
// count return at once.  Admission and retirement therefore change only the
// device work lists: a graph is never edited, and graphs are destroyed only
// with the pool.  A set whose graph was built with a smaller capacity than
// a class now needs gets a new graph; the old one is kept until the pool is
// destroyed.  Each graph is instantiated twice and the two are launched in
// turn, each only after the status snapshot of its previous launch's advance
// has arrived.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/maxflow.h"
#include "mf_pool.h"

using namespace mf;

namespace mf {
// from capi.cpp
std::string resolve_params(const mf_params* in, mf_params& out, Geom& g, int& nl, int& ncap);
void set_error(const std::string& m);
}  // namespace mf

namespace {

mf_status pfail(mf_status s, const std::string& m) {
  set_error(m);
  return s;
}

#define PHIP(expr)                                                                            \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess) return pfail(MF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

size_t al(size_t v) { return (v + 255) / 256 * 256; }

struct Footprint {
  mf_params p;
  Geom g;          // g.plane: plane stride of the padded layout
  int pitch;       // row stride: W rounded up to a multiple of 4
  int nl, ncap, cls, model;
  size_t esz, cap_bytes, state_bytes, total;
};

std::string plan_solve(const mf_params* in, Footprint& f) {
  std::string e = resolve_params(in, f.p, f.g, f.nl, f.ncap);
  if (!e.empty()) return e;
  if (f.p.method != MF_RPADMM_FG && f.p.method != MF_RPADMM_EB) return "the pool runs the rpADMM methods (fg, eb)";
  if (f.p.relax0 != 0.0) return "the pool runs a constant relaxation (relax0 = 0)";
  if (f.p.cap_source != MF_CAPS_PLANES) return "the pool takes capacity planes (cap_source MF_CAPS_PLANES)";
  if (f.g.ndim == 3 && f.p.model != MF_TWO_LABEL) return "the pool runs 3-D solves of the two-label model only";
  if (f.g.ndim == 3) {
    f.model = 5;
  } else if (f.p.model == MF_TWO_LABEL) {
    f.model = 0;
  } else {
    f.model = f.p.nlabels == 2 ? 1 : f.p.nlabels == 3 ? 2 : f.p.nlabels == 4 ? 3 : 4;
  }
  f.cls = f.model + (f.p.storage == MF_BF16 ? kPoolModels : 0);
  f.esz = f.p.storage == MF_BF16 ? 2 : 4;
  // rows padded to a multiple of 4 elements: every tile group is one vector access
  f.pitch = (f.g.W + 3) / 4 * 4;
  f.g.pitch = f.pitch;
  f.g.plane = plane_stride((long long)f.pitch * f.g.H * f.g.D, f.g.ndim);
  const size_t P = (size_t)f.g.plane;
  f.cap_bytes = al((size_t)f.ncap * P * f.esz);
  f.state_bytes = al((size_t)f.nl * P * 4) + al((size_t)f.nl * f.g.ndim * P * f.esz) + al(P * f.esz) +
                  al((size_t)f.nl * P * f.esz);
  f.total = f.cap_bytes + 2 * f.state_bytes;
  return "";
}

StateView carve(char* b, const Footprint& f) {
  const size_t P = (size_t)f.g.plane;
  StateView v;
  v.u = (float*)b;
  b += al((size_t)f.nl * P * 4);
  v.q = b;
  b += al((size_t)f.nl * f.g.ndim * P * f.esz);
  v.ps = b;
  b += al(P * f.esz);
  v.p = b;
  return v;
}

Coef coef_for(const mf_params& p) {
  Coef k;
  k.alpha = (float)p.alpha;
  k.inv_c = (float)(1.0 / p.c);
  k.c = (float)p.c;
  const bool eb = p.method == MF_RPADMM_EB;
  k.rho = eb ? (float)p.relax : 1.f;
  k.omr = eb ? (float)(1.0 - p.relax) : 0.f;
  k.ku = eb ? (float)p.c : (float)(p.relax * p.c);
  k.inv_a = (float)(1.0 / p.a);
  if (p.model == MF_TWO_LABEL) {
    k.inv_a1 = k.inv_a2 = (float)(1.0 / p.a_tilde);
  } else {
    k.inv_a1 = (float)(1.0 / p.a1);
    k.inv_a2 = (float)(1.0 / p.a2);
  }
  return k;
}

struct HostSlot {
  bool used = false;
  bool reported = false;
  int64_t id = -1;
  long long adv0 = 0;   // first advance whose status snapshot reflects this solve's last host update
  Footprint f;
  size_t off = 0;
  StateView st[2];
};

}  // namespace

struct mf_pool {
  char* arena = nullptr;
  size_t arena_bytes = 0;
  hipStream_t stream = nullptr;
  int max_slots = 0, max_tiles = 0, steps = 0;   // steps: iterations per advance
  int depth = 1;                                  // iterations per pass of the two-label 2-D classes
  PoolDev dev;
  size_t data_off = 0;
  std::vector<std::pair<size_t, size_t>> free_list;   // (offset, size), sorted
  std::vector<HostSlot> slots;
  std::vector<PoolSlot> slot_img;                       // host images for uploads
  std::vector<std::vector<WorkItem>> lists;
  std::vector<int> counts;
  // Status snapshots: every advance ends with a copy of the status array
  // into snap[a & 1] (pinned) and an event.  A poll after an advance reads
  // the snapshot of the advance before it, so the device keeps the queued
  // advance while the host reads; a poll with no advance since the last
  // one reads the newest.  stats_h: the snapshot the last poll read.
  PoolStat* snap[2] = {nullptr, nullptr};
  hipEvent_t snap_ev[2] = {nullptr, nullptr};
  long long nadv = 0;           // advances issued
  long long last_read = -1;     // advance whose snapshot the last poll read
  int adv_since_poll = 0;
  PoolStat* stats_h = nullptr;
  PoolStat* one_stat = nullptr;                         // pinned: a single slot's status
  struct Graph {
    int mask = 0;                  // classes the graph launches
    std::vector<unsigned> grid;    // per class: workgroups of its nodes
    hipGraph_t graph = nullptr;
    // two instantiations used in turn, each relaunched only after the
    // snapshot event of the advance that last launched it (recorded after
    // that launch) has completed: no executable graph is launched while an
    // earlier launch of it may still run
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    long long adv[2] = {-1, -1};   // advance that last launched exec[e]
    int next = 0;
  };
  std::vector<Graph> graphs;       // one per class set in use (cached)
  std::vector<Graph> retired;      // superseded graphs, destroyed with the pool
  std::vector<unsigned> cap;       // per class: grid capacity (grow-only)
  long long promotions = 0;
  int64_t next_id = 1;
  size_t in_use = 0;
};

namespace {

bool alloc_block(mf_pool* P, size_t bytes, size_t& off) {
  for (size_t i = 0; i < P->free_list.size(); i++) {
    auto& fb = P->free_list[i];
    if (fb.second >= bytes) {
      off = fb.first;
      fb.first += bytes;
      fb.second -= bytes;
      if (fb.second == 0) P->free_list.erase(P->free_list.begin() + i);
      return true;
    }
  }
  return false;
}

void free_block(mf_pool* P, size_t off, size_t bytes) {
  auto& fl = P->free_list;
  auto it = std::lower_bound(fl.begin(), fl.end(), std::make_pair(off, (size_t)0));
  it = fl.insert(it, {off, bytes});
  size_t i = it - fl.begin();
  if (i + 1 < fl.size() && fl[i].first + fl[i].second == fl[i + 1].first) {
    fl[i].second += fl[i + 1].second;
    fl.erase(fl.begin() + i + 1);
  }
  if (i > 0 && fl[i - 1].first + fl[i - 1].second == fl[i].first) {
    fl[i - 1].second += fl[i].second;
    fl.erase(fl.begin() + i);
  }
}

mf_status upload_list(mf_pool* P, int cls) {
  const auto& L = P->lists[cls];
  if (!L.empty())
    PHIP(hipMemcpyAsync(P->dev.items[cls], L.data(), L.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                        P->stream));
  P->counts[cls] = (int)L.size();
  PHIP(hipMemcpyAsync(P->dev.counts + cls, &P->counts[cls], sizeof(int), hipMemcpyHostToDevice, P->stream));
  return MF_OK;
}

int class_mask(const mf_pool* P) {
  int m = 0;
  for (int c = 0; c < kPoolClasses; c++)
    if (!P->lists[c].empty()) m |= 1 << c;
  return m;
}

// Workgroups of a class launch: one per work item (a multiple of 8 for the
// XCD partition of the item list), at least 8.
unsigned grid_for(int items) {
  const int g = (items + 7) / 8 * 8;
  return (unsigned)(g < 8 ? 8 : g);
}

hipKernelNodeParams node_params(const void* func, unsigned grid, unsigned block, void** args) {
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.func = const_cast<void*>(func);
  kp.gridDim = dim3(grid);
  kp.blockDim = dim3(block);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  return kp;
}

// Build the steps of one advance for the classes in `mask` as an explicit
// graph.  Step h launches, per class and in parallel, the sweep of each
// solve's iterate iter + h (the gap-carrying variant at step 0).  Depth 2: the
// two-label 2-D classes launch their two-iteration pass at even steps only.
// Every pool solve checks at multiples of check_every == steps_per_advance,
// starting at a replay boundary, so step 0 is the check step of every
// solve; the deciding bookkeeping follows it, so a solve that stops or is
// frozen there keeps its iterate (step 0 wrote only its other buffer and
// later launches skip it).  Class nodes take the capacities in P->cap.
mf_status build_graph(mf_pool* P, int mask, mf_pool::Graph& G) {
  G.mask = mask;
  G.grid.assign(kPoolClasses, 0);
  PHIP(hipGraphCreate(&G.graph, 0));
  PoolDev dev = P->dev;
  // Steps h = 0 .. steps-1 of one advance: every class launch of step h
  // depends on all launches of step h-1.  The first step carries the gaps
  // and is followed by the deciding bookkeeping; the last is followed by the
  // bookkeeping that moves every running solve on by `steps` iterations.
  // With depth 2 the two-label 2-D classes launch the two-iteration pass at
  // even steps only.
  std::vector<hipGraphNode_t> prev;   // the nodes the next step depends on
  auto add = [&](const void* f, unsigned grid, unsigned block, void** args, hipGraphNode_t& n) -> mf_status {
    hipKernelNodeParams kp = node_params(f, grid, block, args);
    PHIP(hipGraphAddKernelNode(&n, G.graph, prev.empty() ? nullptr : prev.data(), prev.size(), &kp));
    return MF_OK;
  };
  for (int c = 0; c < kPoolClasses; c++)
    if (mask & (1 << c)) G.grid[c] = P->cap[c];
  const void* book = pool_book_kernel();
  for (int h = 0; h < P->steps; h++) {
    const bool cstep = h == 0;
    const bool odd = P->depth == 2 && (h & 1);   // the one-iteration classes only
    std::vector<hipGraphNode_t> step_nodes;
    for (int c = 0; c < kPoolClasses; c++) {
      if (!(mask & (1 << c))) continue;
      const int model = c % kPoolModels;
      const bool d2 = P->depth == 2 && model == 0;
      if (odd && d2) continue;
      // every class's sweep carries the gap of its checking solves
      const void* f = d2 ? pool_kernel_d2(c, cstep) : pool_kernel(c, cstep, true);
      if (!f) continue;
      int cls = c, step = h;
      void* args[] = {&dev, &cls, &step};
      hipGraphNode_t n;
      const mf_status ms = add(f, G.grid[c], 256, args, n);
      if (ms != MF_OK) return ms;
      step_nodes.push_back(n);
    }
    if (!step_nodes.empty()) prev = step_nodes;
    if (cstep) {
      int decide = 1, by = 0;
      void* bargs[] = {&dev, &decide, &by};
      hipGraphNode_t b;
      const mf_status ms = add(book, (unsigned)P->max_slots, 64, bargs, b);
      if (ms != MF_OK) return ms;
      prev.assign(1, b);
    }
  }
  {
    int decide = 0, by = P->steps;
    void* bargs[] = {&dev, &decide, &by};
    hipGraphNode_t b;
    const mf_status ms = add(book, (unsigned)P->max_slots, 64, bargs, b);
    if (ms != MF_OK) return ms;
  }
  for (int e = 0; e < 2; e++) PHIP(hipGraphInstantiate(&G.exec[e], G.graph, nullptr, nullptr, 0));
  return MF_OK;
}

void destroy_graph(mf_pool::Graph& G) {
  for (int e = 0; e < 2; e++) {
    if (G.exec[e]) hipGraphExecDestroy(G.exec[e]);
    G.exec[e] = nullptr;
  }
  if (G.graph) hipGraphDestroy(G.graph);
  G.graph = nullptr;
}

// The graph for the running class set (its index in P->graphs), with node
// grids at least the current item counts: the cached one, else a new one
// (capacities grown first).
mf_status graph_for(mf_pool* P, int mask, int& index) {
  for (int c = 0; c < kPoolClasses; c++) {
    if (!(mask & (1 << c))) continue;
    const unsigned need = grid_for(P->counts[c]);
    if (P->cap[c] < need) P->cap[c] = std::max(need, 2 * P->cap[c]);
  }
  auto fits = [&](const mf_pool::Graph& G) {
    for (int c = 0; c < kPoolClasses; c++)
      if ((mask & (1 << c)) && G.grid[c] < grid_for(P->counts[c])) return false;
    return true;
  };
  int found = -1;
  for (size_t i = 0; i < P->graphs.size(); i++)
    if (P->graphs[i].mask == mask) found = (int)i;
  if (found >= 0 && fits(P->graphs[found])) {
    index = found;
    return MF_OK;
  }
  mf_pool::Graph G;
  const mf_status ms = build_graph(P, mask, G);
  if (ms != MF_OK) {
    destroy_graph(G);
    return ms;
  }
  if (found >= 0) {
    P->retired.push_back(P->graphs[found]);
    P->graphs[found] = G;
    index = found;
  } else {
    P->graphs.push_back(G);
    index = (int)P->graphs.size() - 1;
  }
  return MF_OK;
}

// Device image of a slot from its host record, at iterate `iter`.
void fill_image(mf_pool* P, int slot, long long iter) {
  HostSlot& H = P->slots[slot];
  const Footprint& f = H.f;
  PoolSlot& S = P->slot_img[slot];
  std::memset(&S, 0, sizeof(S));
  S.state = SLOT_RUNNING;
  S.cls = f.cls;
  S.W = f.g.W;
  S.H = f.g.H;
  S.D = f.g.D;
  S.ndim = f.g.ndim;
  S.nl = f.nl;
  S.two = f.p.model == MF_TWO_LABEL;
  S.bf16 = f.p.storage == MF_BF16;
  S.iso = f.p.tv == MF_TV_ISO;
  S.pitch = f.pitch;
  S.P = f.g.plane;
  S.tiles_x = (f.g.W + 63) / 64;
  const int TY = pool_tile_rows(f.model, f.p.storage == MF_BF16);
  S.tiles_y = f.g.ndim == 2 ? (f.g.H + TY - 1) / TY : (f.g.H + 7) / 8;
  S.tz = f.g.ndim == 3 ? std::min(f.g.D, 16) : 1;
  S.check_every = f.p.check_every;
  S.bufdiv = (P->depth == 2 && f.model == 0) ? 2 : 1;
  S.cap = P->arena + H.off;
  S.st[0] = H.st[0];
  S.st[1] = H.st[1];
  S.k = coef_for(f.p);
  S.alpha = f.p.alpha;
  S.tol = f.p.tol;
  S.iter = iter;
  S.max_iter = f.p.max_iter;
  S.nres = f.g.npix() * f.nl;
  S.check_now = (iter % f.p.check_every == 0 || iter >= f.p.max_iter) ? 1 : 0;
  S.status = 0;
  S.promote_gap = f.p.promote_gap;
  S.promote_iter = f.p.promote_iter;
}

// Move a solve frozen at iterate k from BF16 to FP32 storage: widen its
// capacities and iterate k into a new arena block (exact), point its slot at
// it, move its tiles to the FP32 class and release the BF16 block.  The
// solve resumes at k with the gap re-evaluated there, so the trajectory does
// not depend on when the host gets to it.
// Work items (tile origins) of a solve in `slot`: 64 x TY tiles of the
// class's tile height (2-D), 64 x 8 x 16 bricks (3-D).
std::vector<WorkItem> make_items(int slot, const Footprint& f) {
  std::vector<WorkItem> items;
  const int tx = (f.g.W + 63) / 64;
  if (f.g.ndim == 2) {
    const int TY = pool_tile_rows(f.model, f.p.storage == MF_BF16);
    const int ty = (f.g.H + TY - 1) / TY;
    for (int y = 0; y < ty; y++)
      for (int x = 0; x < tx; x++) items.push_back({slot, x * 64, y * TY, 0});
  } else {
    const int ty = (f.g.H + 7) / 8;
    const int tz = std::min(f.g.D, 16);
    const int nz = (f.g.D + tz - 1) / tz;
    for (int z = 0; z < nz; z++)
      for (int y = 0; y < ty; y++)
        for (int x = 0; x < tx; x++) items.push_back({slot, x * 64, y * 8, z * tz});
  }
  return items;
}

mf_status promote(mf_pool* P, int slot, long long k, bool& moved) {
  moved = false;
  HostSlot& H = P->slots[slot];
  mf_params p32 = H.f.p;
  p32.storage = MF_F32;
  Footprint f2;
  const std::string e = plan_solve(&p32, f2);
  if (!e.empty()) return pfail(MF_EINVAL, e);
  const std::vector<WorkItem> items = make_items(slot, f2);
  if ((long long)P->lists[f2.cls].size() + (long long)items.size() > P->max_tiles) return MF_OK;   // stays frozen
  size_t off;
  if (!alloc_block(P, f2.total, off)) return MF_OK;   // no room yet: stays frozen
  char* base = P->arena + off;
  StateView n0 = carve(base + f2.cap_bytes, f2), n1 = carve(base + f2.cap_bytes + f2.state_bytes, f2);
  const int b = (int)((k / P->slot_img[slot].bufdiv) & 1);   // the buffer of iterate k (same in both classes)
  const StateView src = H.st[b];
  const StateView& dst = b ? n1 : n0;
  const long long n = H.f.g.plane, pl = H.f.g.plane;   // whole planes, pads included
  PHIP(launch_convert_planes(P->arena + H.off, true, base, false, n, H.f.ncap, pl, pl, P->stream));
  PHIP(launch_convert_planes(src.u, false, dst.u, false, n, H.f.nl, pl, pl, P->stream));
  PHIP(launch_convert_planes(src.q, true, dst.q, false, n, H.f.nl * H.f.g.ndim, pl, pl, P->stream));
  PHIP(launch_convert_planes(src.ps, true, dst.ps, false, n, 1, pl, pl, P->stream));
  PHIP(launch_convert_planes(src.p, true, dst.p, false, n, H.f.nl, pl, pl, P->stream));
  const int old_cls = H.f.cls;
  const size_t old_off = H.off, old_total = H.f.total;
  H.f = f2;
  H.off = off;
  H.st[0] = n0;
  H.st[1] = n1;
  H.adv0 = P->nadv;   // earlier snapshots still show it frozen for promotion
  fill_image(P, slot, k);
  PHIP(hipMemcpyAsync(P->dev.slots + slot, &P->slot_img[slot], sizeof(PoolSlot), hipMemcpyHostToDevice,
                      P->stream));
  PoolStat st;
  std::memset(&st, 0, sizeof(st));
  st.state = SLOT_RUNNING;
  st.iter = k;
  PHIP(hipMemcpyAsync(P->dev.stats + slot, &st, sizeof(st), hipMemcpyHostToDevice, P->stream));
  // the FP32 class may tile differently: rebuild this solve's items there
  auto& Lo = P->lists[old_cls];
  auto& Ln = P->lists[f2.cls];
  Lo.erase(std::remove_if(Lo.begin(), Lo.end(), [&](const WorkItem& w) { return w.slot == slot; }), Lo.end());
  Ln.insert(Ln.end(), items.begin(), items.end());
  mf_status ms = upload_list(P, old_cls);
  if (ms == MF_OK) ms = upload_list(P, f2.cls);
  if (ms != MF_OK) return ms;
  PHIP(hipStreamSynchronize(P->stream));
  free_block(P, old_off, old_total);
  P->in_use += f2.total;
  P->in_use -= old_total;
  P->promotions++;
  moved = true;
  return MF_OK;
}

}  // namespace

extern "C" {

size_t mf_pool_footprint(const mf_params* p) {
  Footprint f;
  const std::string e = plan_solve(p, f);
  if (!e.empty()) {
    set_error(e);
    return 0;
  }
  return f.total;
}

size_t mf_pool_table_bytes(int32_t max_slots, int32_t max_tiles) {
  return al(sizeof(PoolSlot) * (size_t)max_slots) + al(sizeof(PoolStat) * (size_t)max_slots) +
         (size_t)kPoolClasses * al(sizeof(WorkItem) * (size_t)max_tiles) + al(sizeof(int) * kPoolClasses);
}

mf_status mf_pool_create(void* arena, size_t arena_bytes, int32_t max_slots, int32_t max_tiles,
                         int32_t steps_per_advance, int32_t depth, void* hip_stream, mf_pool** out) {
  if (!out) return pfail(MF_EINVAL, "out is null");
  *out = nullptr;
  if (!arena || ((uintptr_t)arena & 255)) return pfail(MF_EINVAL, "arena must be a 256-byte aligned device pointer");
  if (!hip_stream) return pfail(MF_EINVAL, "the pool needs a created (non-default) stream for graph capture");
  if (max_slots < 1 || max_slots > 65536 || max_tiles < 1 || steps_per_advance < 1)
    return pfail(MF_EINVAL, "max_slots in [1, 65536], max_tiles >= 1, steps_per_advance >= 1");
  // Only 10-step advances are supported: a process that ran a 20-step pool
  // after a 10-step one ended in a host segmentation fault whose cause has
  // not been found, and no other step count has been run.
  if (steps_per_advance != kPoolSteps)
    return pfail(MF_EINVAL, "steps_per_advance must be 10 (other step counts are not supported)");
  if (depth == 0) depth = steps_per_advance % 2 == 0 ? 2 : 1;
  if (depth != 1 && depth != 2) return pfail(MF_EINVAL, "depth must be 0, 1 or 2");
  if (steps_per_advance % depth != 0) return pfail(MF_EINVAL, "steps_per_advance must be a multiple of depth");
  const size_t tb = mf_pool_table_bytes(max_slots, max_tiles);
  if (arena_bytes <= tb) return pfail(MF_ENOMEM, "arena smaller than the pool tables");
  mf_pool* P = new (std::nothrow) mf_pool();
  if (!P) return pfail(MF_ENOMEM, "host allocation failed");
  P->arena = (char*)arena;
  P->arena_bytes = arena_bytes;
  P->stream = (hipStream_t)hip_stream;
  P->max_slots = max_slots;
  P->max_tiles = max_tiles;
  P->steps = steps_per_advance;
  P->depth = depth;
  size_t off = 0;
  P->dev.slots = (PoolSlot*)(P->arena + off);
  off += al(sizeof(PoolSlot) * (size_t)max_slots);
  P->dev.stats = (PoolStat*)(P->arena + off);
  off += al(sizeof(PoolStat) * (size_t)max_slots);
  for (int c = 0; c < kPoolClasses; c++) {
    P->dev.items[c] = (WorkItem*)(P->arena + off);
    off += al(sizeof(WorkItem) * (size_t)max_tiles);
  }
  P->dev.counts = (int*)(P->arena + off);
  off += al(sizeof(int) * kPoolClasses);
  P->data_off = off;
  P->free_list.push_back({off, arena_bytes - off});
  P->slots.resize(max_slots);
  P->slot_img.resize(max_slots);
  P->lists.resize(kPoolClasses);
  for (auto& l : P->lists) l.reserve(1024);
  P->counts.assign(kPoolClasses, 0);
  P->cap.assign(kPoolClasses, 8);
  std::vector<PoolSlot> zero(max_slots);
  std::memset(zero.data(), 0, zero.size() * sizeof(PoolSlot));
  std::vector<PoolStat> zs(max_slots);
  std::memset(zs.data(), 0, zs.size() * sizeof(PoolStat));
  hipError_t e = hipMemcpyAsync(P->dev.slots, zero.data(), zero.size() * sizeof(PoolSlot), hipMemcpyHostToDevice,
                                P->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(P->dev.stats, zs.data(), zs.size() * sizeof(PoolStat), hipMemcpyHostToDevice, P->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(P->dev.counts, P->counts.data(), sizeof(int) * kPoolClasses, hipMemcpyHostToDevice,
                       P->stream);

  for (int i = 0; i < 2 && e == hipSuccess; i++) {
    e = hipHostMalloc((void**)&P->snap[i], sizeof(PoolStat) * (size_t)max_slots, hipHostMallocDefault);
    if (e == hipSuccess) std::memset(P->snap[i], 0, sizeof(PoolStat) * (size_t)max_slots);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->snap_ev[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&P->one_stat, sizeof(PoolStat), hipHostMallocDefault);
  P->stats_h = P->snap[0];
  if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
  if (e != hipSuccess) {
    mf_pool_destroy(P);
    return pfail(MF_EDEVICE, std::string("pool create: ") + hipGetErrorString(e));
  }
  *out = P;
  return MF_OK;
}

mf_status mf_pool_admit(mf_pool* P, const mf_params* p, const float* cap, int64_t* solve_id) {
  if (!P || !cap || !solve_id) return pfail(MF_EINVAL, "null argument");
  Footprint f;
  const std::string e = plan_solve(p, f);
  if (!e.empty()) return pfail(MF_EINVAL, e);
  if (f.p.check_every != P->steps || f.p.max_iter % f.p.check_every != 0)
    return pfail(MF_EINVAL, "pool solves need check_every == steps_per_advance and max_iter a multiple of it");
  int slot = -1;
  for (int i = 0; i < P->max_slots; i++)
    if (!P->slots[i].used) {
      slot = i;
      break;
    }
  if (slot < 0) return pfail(MF_ENOMEM, "no free slot");
  const std::vector<WorkItem> items = make_items(slot, f);
  auto& L = P->lists[f.cls];
  if ((long long)L.size() + (long long)items.size() > P->max_tiles) return pfail(MF_ENOMEM, "work list full");
  size_t off;
  if (!alloc_block(P, f.total, off)) return pfail(MF_ENOMEM, "arena full");
  HostSlot& H = P->slots[slot];
  H.used = true;
  H.reported = false;
  H.id = P->next_id++;
  H.adv0 = P->nadv;   // earlier snapshots show the slot's previous occupant
  H.f = f;
  H.off = off;
  char* base = P->arena + off;
  H.st[0] = carve(base + f.cap_bytes, f);
  H.st[1] = carve(base + f.cap_bytes + f.state_bytes, f);
  P->in_use += f.total;
  const bool bf16 = f.p.storage == MF_BF16;
  const long long rows = (long long)f.g.H * f.g.D;
  PHIP(launch_pitch_copy(cap, false, f.g.npix(), f.g.W, base, bf16, f.g.plane, f.pitch, f.g.W, rows, f.ncap,
                         P->stream));
  // initialise the padded planes whole (pads hold zero capacities)
  PHIP(launch_init(f.g, f.nl, f.p.model == MF_TWO_LABEL, bf16, base, CapGen{}, H.st[0], P->stream));
  fill_image(P, slot, 0);
  PoolSlot& S = P->slot_img[slot];
  PHIP(hipMemcpyAsync(P->dev.slots + slot, &S, sizeof(S), hipMemcpyHostToDevice, P->stream));
  PoolStat st;
  std::memset(&st, 0, sizeof(st));
  st.state = SLOT_RUNNING;
  PHIP(hipMemcpyAsync(P->dev.stats + slot, &st, sizeof(st), hipMemcpyHostToDevice, P->stream));
  L.insert(L.end(), items.begin(), items.end());
  mf_status ms = upload_list(P, f.cls);
  if (ms != MF_OK) return ms;
  // the host images above are the sources of the copies: let them complete
  PHIP(hipStreamSynchronize(P->stream));
  *solve_id = H.id;
  return MF_OK;
}

mf_status mf_pool_advance(mf_pool* P) {
  if (!P) return pfail(MF_EINVAL, "null pool");
  int gi = -1;
  const mf_status ms = graph_for(P, class_mask(P), gi);
  if (ms != MF_OK) return ms;
  mf_pool::Graph& G = P->graphs[gi];
  const int e = G.next;
  // the snapshot event of that parity was last recorded at or after the
  // advance that launched exec[e], and behind it on the stream
  if (G.adv[e] >= 0) PHIP(hipEventSynchronize(P->snap_ev[G.adv[e] & 1]));
  PHIP(hipGraphLaunch(G.exec[e], P->stream));
  G.adv[e] = P->nadv;
  G.next = e ^ 1;
  const int b = (int)(P->nadv & 1);
  PHIP(hipMemcpyAsync(P->snap[b], P->dev.stats, sizeof(PoolStat) * (size_t)P->max_slots, hipMemcpyDeviceToHost,
                      P->stream));
  PHIP(hipEventRecord(P->snap_ev[b], P->stream));
  P->nadv++;
  P->adv_since_poll++;
  return MF_OK;
}

mf_status mf_pool_poll(mf_pool* P, int64_t* done_ids, mf_gap* gaps, int32_t cap, int32_t* ndone) {
  if (!P || !ndone) return pfail(MF_EINVAL, "null argument");
  *ndone = 0;
  const long long j = P->adv_since_poll > 0 ? P->nadv - 2 : P->nadv - 1;
  P->adv_since_poll = 0;
  if (j < 0 || j <= P->last_read) return MF_OK;   // nothing newer to read yet
  PHIP(hipEventSynchronize(P->snap_ev[j & 1]));
  P->stats_h = P->snap[j & 1];
  P->last_read = j;
  for (int i = 0; i < P->max_slots; i++) {
    if (P->slots[i].used && j >= P->slots[i].adv0 && P->stats_h[i].state == SLOT_PROMOTE) {
      bool moved;
      mf_status ms = promote(P, i, P->stats_h[i].iter, moved);
      if (ms != MF_OK) return ms;
    }
  }
  for (int i = 0; i < P->max_slots && *ndone < cap; i++) {
    HostSlot& H = P->slots[i];
    if (!H.used || H.reported || j < H.adv0) continue;
    const PoolStat& s = P->stats_h[i];
    if (s.state != SLOT_DONE) continue;
    H.reported = true;
    if (done_ids) done_ids[*ndone] = H.id;
    if (gaps) {
      mf_gap& g = gaps[*ndone];
      g.iter = s.iter;
      g.primal = s.last[0];
      g.dual = s.last[1];
      g.rel_gap = s.last[2];
      g.resid_rms = s.last[3];
      g.flow = s.last[4];
      g.status = s.status;
    }
    (*ndone)++;
  }
  return MF_OK;
}

mf_status mf_pool_retire(mf_pool* P, int64_t solve_id, float* u_dst, int32_t* labels_dst) {
  if (!P) return pfail(MF_EINVAL, "null pool");
  int slot = -1;
  for (int i = 0; i < P->max_slots; i++)
    if (P->slots[i].used && P->slots[i].id == solve_id) {
      slot = i;
      break;
    }
  if (slot < 0) return pfail(MF_EINVAL, "unknown solve id");
  HostSlot& H = P->slots[slot];
  // a reported solve is stopped: its snapshot holds the final iterate; one
  // retired before a poll reported it is read now, after the queued work
  long long it;
  if (H.reported) {
    it = P->stats_h[slot].iter;
  } else {
    PHIP(hipMemcpyAsync(P->one_stat, P->dev.stats + slot, sizeof(PoolStat), hipMemcpyDeviceToHost, P->stream));
    PHIP(hipStreamSynchronize(P->stream));
    it = P->one_stat->iter;
  }
  const StateView& v = H.st[(it / P->slot_img[slot].bufdiv) & 1];
  const long long rows = (long long)H.f.g.H * H.f.g.D;
  if (u_dst)
    PHIP(launch_pitch_copy(v.u, false, H.f.g.plane, H.f.pitch, u_dst, false, H.f.g.npix(), H.f.g.W, H.f.g.W, rows,
                           H.f.nl, P->stream));
  if (labels_dst)
    PHIP(launch_labels(H.f.g, H.f.nl, H.f.p.model == MF_TWO_LABEL, v.u, labels_dst, P->stream, H.f.pitch));
  // free the slot on the device and drop its tiles
  int zero = SLOT_FREE;
  PHIP(hipMemcpyAsync(&P->dev.slots[slot].state, &zero, sizeof(int), hipMemcpyHostToDevice, P->stream));
  PHIP(hipMemcpyAsync(&P->dev.stats[slot].state, &zero, sizeof(int), hipMemcpyHostToDevice, P->stream));
  auto& L = P->lists[H.f.cls];
  L.erase(std::remove_if(L.begin(), L.end(), [&](const WorkItem& w) { return w.slot == slot; }), L.end());
  mf_status ms = upload_list(P, H.f.cls);
  if (ms != MF_OK) return ms;
  PHIP(hipStreamSynchronize(P->stream));
  free_block(P, H.off, H.f.total);
  P->in_use -= H.f.total;
  H.used = false;
  H.id = -1;
  return MF_OK;
}

int64_t mf_pool_promotions(const mf_pool* P) { return P ? P->promotions : -1; }

mf_status mf_pool_stats(mf_pool* P, int32_t* active, size_t* bytes_in_use, size_t* bytes_free) {
  if (!P) return pfail(MF_EINVAL, "null pool");
  int n = 0;
  for (auto& h : P->slots) n += h.used ? 1 : 0;
  if (active) *active = n;
  if (bytes_in_use) *bytes_in_use = P->in_use;
  if (bytes_free) {
    size_t m = 0;
    for (auto& fb : P->free_list) m = std::max(m, fb.second);
    *bytes_free = m;
  }
  return MF_OK;
}

mf_status mf_pool_destroy(mf_pool* P) {
  if (!P) return MF_OK;
  if (P->stream) hipStreamSynchronize(P->stream);
  for (auto* gs : {&P->graphs, &P->retired})
    for (auto& G : *gs) destroy_graph(G);
  for (int i = 0; i < 2; i++) {
    if (P->snap[i]) hipHostFree(P->snap[i]);
    if (P->snap_ev[i]) hipEventDestroy(P->snap_ev[i]);
  }
  if (P->one_stat) hipHostFree(P->one_stat);
  delete P;
  return MF_OK;
}

}  // extern "C"
