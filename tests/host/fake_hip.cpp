// Host emulation of the HIP runtime for the address-sanitised check of the
// library's host code (the pool's tables, free list, work lists, snapshots
// and graph bookkeeping; the solver's polling loop and workspace layout).
//
// "Device" memory is host memory: copies are memcpy, streams and events
// complete at once, and a graph launch runs its kernel nodes in order through
// host emulations keyed by the kernel address.  The kernels' arithmetic is
// not emulated: sweep launches touch the first and last byte of every plane
// they would read or write (so a pointer outside its buffer is reported),
// and the bookkeeping launches take scripted convergence decisions with the
// same state transitions as the device code.  Test infrastructure only.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/maxflow.h"
#include "../../paper_2004_11227_amd/csrc/mf_pool.h"

using namespace mf;

namespace {

volatile unsigned char g_sink;

// Reads the first and last byte of [p, p + n): ASan reports a range that
// leaves its allocation.
void touch(const void* p, size_t n) {
  if (!p || !n) return;
  const unsigned char* b = (const unsigned char*)p;
  g_sink = b[0];
  g_sink = b[n - 1];
}
void touch_w(void* p, size_t n) {
  if (!p || !n) return;
  unsigned char* b = (unsigned char*)p;
  b[0] = b[0];
  b[n - 1] = b[n - 1];
}

uint64_t mix(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

struct FakeNode {
  const void* func;
  unsigned grid, block;
  PoolDev dev;
  int a1, a2;
};
struct FakeGraph {
  std::vector<FakeNode*> nodes;
};
struct FakeExec {
  std::vector<FakeNode*> src;     // nodes of the graph, in insertion order
  std::vector<FakeNode> nodes;    // this exec's copies
};

FakeNode read_params(const hipKernelNodeParams* kp) {
  FakeNode n;
  n.func = kp->func;
  n.grid = kp->gridDim.x;
  n.block = kp->blockDim.x;
  // every pool kernel takes (PoolDev, int, int)
  std::memcpy(&n.dev, kp->kernelParams[0], sizeof(PoolDev));
  std::memcpy(&n.a1, kp->kernelParams[1], sizeof(int));
  std::memcpy(&n.a2, kp->kernelParams[2], sizeof(int));
  return n;
}

long long g_launches = 0;

// The bookkeeping kernel's transitions (decide after the first step; move
// every running slot on by the advance's iterations after the last), with a
// scripted decision in place of the gap.
void book(const FakeNode& n, unsigned slots) {
  for (unsigned b = 0; b < slots && b < n.grid; b++) {
    PoolSlot* sl = n.dev.slots + b;
    touch(sl, sizeof(*sl));
    if (sl->state != SLOT_RUNNING) continue;
    if (n.a1) {
      if (!sl->check_now) continue;
      const long long k = sl->iter;
      int state = SLOT_RUNNING;
      const uint64_t h = mix((uint64_t)(uintptr_t)sl->st[0].u ^ (uint64_t)k * 1315423911ull);
      PoolStat& ps = n.dev.stats[b];
      touch_w(&ps, sizeof(ps));
      for (int j = 0; j < 6; j++) ps.last[j] = (double)(h % 1000) * 1e-6;
      if (h % 97 == 0) {
        state = SLOT_DONE;
        sl->status = -4;
      } else if (h % 5 == 0) {
        state = SLOT_DONE;
        sl->status = 0;
      } else if (k >= sl->max_iter) {
        state = SLOT_DONE;
        sl->status = 1;
      } else if (sl->bf16 && sl->promote_iter > 0 && k >= sl->promote_iter) {
        state = SLOT_PROMOTE;
      }
      sl->check_now = 0;
      sl->state = state;
      ps.state = state;
      ps.status = sl->status;
      ps.iter = k;
    } else {
      const long long kn = sl->iter + n.a2;
      sl->iter = kn;
      sl->check_now = (kn % sl->check_every == 0 || kn >= sl->max_iter) ? 1 : 0;
      n.dev.stats[b].state = sl->state;
      n.dev.stats[b].status = sl->status;
      n.dev.stats[b].iter = kn;
    }
  }
}

// A class sweep: every listed item of a running slot, its tile origin inside
// the grid and the planes of both state buffers inside the arena.
void sweep(const FakeNode& n) {
  const int cls = n.a1;
  touch(n.dev.counts + cls, sizeof(int));
  const int cnt = n.dev.counts[cls];
  if (cnt > 0) touch(n.dev.items[cls], sizeof(WorkItem) * (size_t)cnt);
  for (int i = 0; i < cnt; i++) {
    const WorkItem w = n.dev.items[cls][i];
    PoolSlot* sl = n.dev.slots + w.slot;
    touch(sl, sizeof(*sl));
    if (sl->state != SLOT_RUNNING) continue;
    if (sl->cls != cls || w.x0 < 0 || w.x0 >= sl->W || w.y0 < 0 || w.y0 >= sl->H || w.z0 < 0 || w.z0 >= sl->D) {
      std::fprintf(stderr, "fake_hip: work item (%d, %d, %d) of slot %d outside its grid or class\n", w.x0, w.y0,
                   w.z0, w.slot);
      std::abort();
    }
    const size_t e = sl->bf16 ? 2 : 4;
    const size_t P = (size_t)sl->P;
    const int nl = sl->nl, nq = sl->nl * sl->ndim;
    touch(sl->cap, (size_t)(sl->two ? 2 : nl) * P * e);
    for (int b = 0; b < 2; b++) {
      touch_w(sl->st[b].u, (size_t)nl * P * 4);
      touch_w(sl->st[b].q, (size_t)nq * P * e);
      touch_w(sl->st[b].ps, P * e);
      touch_w(sl->st[b].p, (size_t)nl * P * e);
    }
  }
}

}  // namespace

// ------------------------------------------------------------- kernels used by pool.cpp
namespace mf {
static char k_sweep_tag[kPoolClasses * 2 + 2], k_d2_tag[kPoolClasses * 2], k_book_tag;
const void* pool_kernel(int cls, bool check, bool) { return &k_sweep_tag[cls * 2 + (check ? 1 : 0)]; }
const void* pool_kernel_d2(int cls, bool check) {
  return (cls % kPoolModels) == 0 ? &k_d2_tag[cls * 2 + (check ? 1 : 0)] : nullptr;
}
const void* pool_book_kernel() { return &k_book_tag; }

// Element-wise launches: touch the ranges they cover.
hipError_t launch_pitch_copy(const void* src, bool sb, long long sp, int spitch, void* dst, bool db, long long dp,
                             int dpitch, int W, long long rows, int np, hipStream_t) {
  if (np < 1 || W > spitch || W > dpitch) return hipErrorInvalidValue;
  touch(src, ((size_t)(np - 1) * sp + (size_t)(rows - 1) * spitch + W) * (sb ? 2 : 4));
  touch_w(dst, ((size_t)(np - 1) * dp + (size_t)rows * dpitch) * (db ? 2 : 4));
  return hipSuccess;
}
hipError_t launch_init(const Geom& g, int nl, bool two, bool bf16, const void* cap, const CapGen& cg, StateView st,
                       hipStream_t) {
  const size_t e = bf16 ? 2 : 4, n = (size_t)g.nstore(), P = (size_t)g.plane;
  touch(cap, ((size_t)((cg.img ? 1 : (two ? 2 : nl)) - 1) * P + n) * e);
  touch_w(st.u, ((size_t)(nl - 1) * P + n) * 4);
  touch_w(st.q, ((size_t)(nl * g.ndim - 1) * P + n) * e);
  touch_w(st.ps, n * e);
  touch_w(st.p, ((size_t)(nl - 1) * P + n) * e);
  return hipSuccess;
}
hipError_t launch_labels(const Geom& g, int nl, bool, const float* u, int32_t* lab, hipStream_t, int pitch) {
  touch(u, ((size_t)(nl - 1) * g.plane + (size_t)(g.H * g.D - 1) * (pitch > 0 ? pitch : g.W) + g.W) * 4);
  touch_w(lab, (size_t)g.npix() * 4);
  return hipSuccess;
}
hipError_t launch_convert_planes(const void* src, bool sb, void* dst, bool db, long long n, int np, long long ss,
                                 long long ds, hipStream_t) {
  touch(src, ((size_t)(np - 1) * ss + n) * (sb ? 2 : 4));
  touch_w(dst, ((size_t)(np - 1) * ds + n) * (db ? 2 : 4));
  return hipSuccess;
}

// Solver launches (capi.cpp): the scripted decisions of the bookkeeping
// kernel and range checks of the state the sweeps read and write.
long long g_stop_every = 7;
hipError_t launch_ctrl_reset(Ctrl* c, hipStream_t) {
  touch_w(c, sizeof(Ctrl));
  std::memset(c, 0, sizeof(Ctrl));
  return hipSuccess;
}
hipError_t launch_bookkeep(Ctrl* c, long long k, double, double tol, double, long long, int final_check, int decide,
                           hipStream_t) {
  touch_w(c, sizeof(Ctrl));
  if (c->done) return hipSuccess;
  c->last[5] = (double)k;
  c->checks += 1;
  if (decide) {
    const bool stop = tol > 0.0 && (mix((uint64_t)k * 7919u + (uint64_t)c->checks) % g_stop_every) == 0;
    if (stop || final_check) {
      c->done = 1;
      c->status = stop ? 0 : 1;
      c->iter = k;
    }
  }
  return hipSuccess;
}
static void touch_state(const SweepDesc& d, const StateView& v, bool w) {
  const size_t e = d.bf16 ? 2 : 4, n = (size_t)d.g.nstore(), P = (size_t)d.g.plane;
  auto t = [&](void* p, size_t b) { w ? touch_w(p, b) : touch(p, b); };
  t(v.u, ((size_t)(d.nl - 1) * P + n) * 4);
  t(v.q, ((size_t)(d.nl * d.g.ndim - 1) * P + n) * e);
  t(v.ps, n * e);
  t(v.p, ((size_t)(d.nl - 1) * P + n) * e);
}
size_t n_cap_bytes(const SweepDesc& d);
static hipError_t sweep_desc(const SweepDesc& d) {
  if (d.done && *d.done) return hipSuccess;
  touch(d.cap, n_cap_bytes(d));
  touch_state(d, d.in, false);
  if (d.write) touch_state(d, d.out, true);
  if (d.acc) touch_w(d.acc, sizeof(double) * kAccSlots * 8);
  return hipSuccess;
}
size_t n_cap_bytes(const SweepDesc& d) {
  const size_t e = d.bf16 ? 2 : 4;
  const int ncap = d.cg.img ? 1 : (d.two ? 2 : d.nl);
  return ((size_t)(ncap - 1) * d.g.plane + (size_t)d.g.nstore()) * e;
}
hipError_t launch_fused(const SweepDesc& d, hipStream_t) { return sweep_desc(d); }
hipError_t launch_fused2d_d2(const SweepDesc& d, hipStream_t) { return sweep_desc(d); }
hipError_t launch_unfused(const SweepDesc& d, hipStream_t) {
  if (d.wbuf) touch_w(d.wbuf, ((size_t)(d.nl - 1) * d.g.plane + (size_t)d.g.nstore()) * 4);
  return sweep_desc(d);
}
hipError_t launch_first_two(const Geom& g, bool bf16, const void* cap, const StateView& out, const Coef&,
                            double* acc, hipStream_t) {
  const size_t e = bf16 ? 2 : 4, n = (size_t)g.nstore(), P = (size_t)g.plane;
  touch(cap, (P + n) * e);
  touch_w(out.u, n * 4);
  touch_w(out.q, ((size_t)(g.ndim - 1) * P + n) * e);
  touch_w(out.ps, n * e);
  touch_w(out.p, n * e);
  touch_w(acc, sizeof(double) * kAccSlots * 8);
  return hipSuccess;
}
hipError_t launch_gap(const GapDesc& d, hipStream_t) {
  if (d.done && *d.done) return hipSuccess;
  touch_w(d.acc, sizeof(double) * kAccSlots * 8);
  touch(d.st.u, ((size_t)(d.nl - 1) * d.g.plane + (size_t)d.g.nstore()) * 4);
  return hipSuccess;
}
hipError_t launch_pdrq_iter(const PdrqDesc& d, hipStream_t) {
  if (d.done && *d.done) return hipSuccess;
  const size_t e = d.bf16 ? 2 : 4, n = (size_t)d.g.nstore(), P = (size_t)d.g.plane;
  touch_w(d.st.u, ((size_t)(d.nl - 1) * P + n) * 4);
  touch_w(d.out.u, ((size_t)(d.nl - 1) * P + n) * 4);
  touch_w(d.z.q, ((size_t)(d.nl * d.g.ndim - 1) * P + n) * e);
  touch_w(d.b, ((size_t)(d.nl - 1) * P + n) * 4);
  return hipSuccess;
}
}  // namespace mf

// ------------------------------------------------------------- runtime entry points
extern "C" {

const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake error"; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  touch(src, n);
  touch_w(dst, n);
  std::memmove(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t) {
  touch_w(dst, n);
  std::memset(dst, v, n);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
  *p = std::malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
struct FakeEvent {
  int recorded;
};
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = reinterpret_cast<hipEvent_t>(new FakeEvent{0});
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete reinterpret_cast<FakeEvent*>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  reinterpret_cast<FakeEvent*>(e)->recorded = 1;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  touch(e, sizeof(FakeEvent));
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  touch(e, sizeof(FakeEvent));
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  touch(a, sizeof(FakeEvent));
  touch(b, sizeof(FakeEvent));
  *ms = 1.f;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
hipError_t hipGraphCreate(hipGraph_t* g, unsigned int) {
  *g = reinterpret_cast<hipGraph_t>(new FakeGraph);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  FakeGraph* fg = reinterpret_cast<FakeGraph*>(g);
  for (FakeNode* n : fg->nodes) delete n;
  delete fg;
  return hipSuccess;
}
hipError_t hipGraphAddKernelNode(hipGraphNode_t* out, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                                 const hipKernelNodeParams* kp) {
  FakeGraph* fg = reinterpret_cast<FakeGraph*>(g);
  for (size_t i = 0; i < ndeps; i++) touch(deps[i], sizeof(FakeNode));
  FakeNode* n = new FakeNode(read_params(kp));
  fg->nodes.push_back(n);
  *out = reinterpret_cast<hipGraphNode_t>(n);
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  FakeGraph* fg = reinterpret_cast<FakeGraph*>(g);
  FakeExec* fe = new FakeExec;
  fe->src = fg->nodes;
  for (FakeNode* n : fg->nodes) fe->nodes.push_back(*n);
  *e = reinterpret_cast<hipGraphExec_t>(fe);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete reinterpret_cast<FakeExec*>(e);
  return hipSuccess;
}
hipError_t hipGraphExecKernelNodeSetParams(hipGraphExec_t e, hipGraphNode_t node, const hipKernelNodeParams* kp) {
  FakeExec* fe = reinterpret_cast<FakeExec*>(e);
  for (size_t i = 0; i < fe->src.size(); i++)
    if (fe->src[i] == reinterpret_cast<FakeNode*>(node)) {
      fe->nodes[i] = read_params(kp);
      return hipSuccess;
    }
  std::fprintf(stderr, "fake_hip: SetParams on a node that is not in the graph\n");
  std::abort();
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  FakeExec* fe = reinterpret_cast<FakeExec*>(e);
  g_launches++;
  for (const FakeNode& n : fe->nodes) {
    if (n.func == &mf::k_book_tag) book(n, n.grid);
    else sweep(n);
  }
  return hipSuccess;
}

// Registration of the library's static device array (host-side stand-in).
void** __hipRegisterFatBinary(const void*) {
  static void* h = nullptr;
  return &h;
}
void __hipRegisterVar(void**, void*, char*, char*, int, size_t, int, int) {}
void __hipUnregisterFatBinary(void**) {}

long long fake_hip_graph_launches() { return g_launches; }
void fake_hip_stop_every(long long n) { mf::g_stop_every = n; }

}  // extern "C"
