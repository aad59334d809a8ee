// Host runtime behind include/maxflow.h: parameter validation, workspace
// layout, launch schedules and the device-side convergence protocol.
//
// Ping-pong state: iterate k of an rpADMM solve lives in state buffer k % 2.
// A "check" evaluates the gap of iterate k (fused into the sweep k -> k+1 for
// the two-label fused pass, otherwise a standalone reduction before it) and a
// one-thread bookkeeping kernel decides on the GPU whether the solve stops at
// k; every later sweep of the same solve reads that decision and exits at
// once, so buffer k % 2 keeps iterate k.  The host only polls the decision to
// stop enqueueing work; it never has to wait for a gap before continuing.
// rPDRQ updates its state in place and evaluates the gap on the output of
// the check iteration, so it needs no rollback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/maxflow.h"
#include "mf_kernels.h"

using namespace mf;

namespace {

// Last error message of this thread, in a fixed buffer: recording an error
// never allocates (the allocation-free entry point relies on it).
thread_local char g_err[512];

void set_err(const char* a, const char* b = nullptr) {
  if (b) snprintf(g_err, sizeof(g_err), "%s: %s", a, b);
  else snprintf(g_err, sizeof(g_err), "%s", a);
}

mf_status fail(mf_status s, const char* msg, const char* detail = nullptr) {
  set_err(msg, detail);
  return s;
}
mf_status fail(mf_status s, const std::string& msg) { return fail(s, msg.c_str()); }

}  // namespace

namespace mf {
void set_error(const std::string& m) { set_err(m.c_str()); }
}  // namespace mf

namespace {

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess) return fail(MF_EDEVICE, #expr, hipGetErrorString(_e));           \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Resolved {
  mf_params p;
  int nl;         // labels carried (1 two-label, n Potts)
  int ncap;       // capacities per pixel (2 two-label, n Potts)
  int ncp;        // capacity planes stored: ncap, or 1 (the image)
  CapGen cg;      // image-generated capacities
  Geom g;
  size_t esz;     // bytes per flow / capacity element
  int nq;         // q planes per state
};

// Largest sweep count of the fused 2-D rPDRQ pass: its staged rectangle
// grows by 2 cells per side and sweep; beyond these the LDS per workgroup
// (and for Potts the registers) leave one wave per SIMD and the in-place
// launches are faster (measured at 2048^2 two-label, 1024^2 n = 4).
inline int fused_dr_sweeps(int model) { return model == MF_TWO_LABEL ? 4 : 3; }

// Fill defaults and validate; returns an error message or "" (string
// literals only: validation never allocates).
const char* resolve(const mf_params* in, Resolved& r) {
  if (!in) return "null params";
  r.p = *in;
  mf_params& p = r.p;
  if (p.ndim != 2 && p.ndim != 3) return "ndim must be 2 or 3";
  for (int i = 0; i < p.ndim; i++)
    if (p.shape[i] < 1 || p.shape[i] > (1LL << 30)) return "shape entries must be >= 1";
  if (p.model != MF_TWO_LABEL && p.model != MF_POTTS) return "unknown model";
  if (p.method < MF_RPADMM_FG || p.method > MF_CP_ALG1) return "unknown method";
  const bool cmp = p.method == MF_PADMM_TY || p.method == MF_CP_ALG1;
  if (cmp) p.variant = MF_UNFUSED;   // the comparison methods run element-wise kernels
  if (p.tv != MF_TV_ISO && p.tv != MF_TV_ANISO) return "unknown tv";
  if (p.storage != MF_F32 && p.storage != MF_BF16) return "unknown storage";
  if (p.variant != MF_FUSED && p.variant != MF_UNFUSED) return "unknown variant";
  if (p.model == MF_TWO_LABEL) {
    if (p.nlabels != 0 && p.nlabels != 2) return "two-label model needs nlabels = 2";
    p.nlabels = 2;
  } else if (!(p.nlabels == 2 || p.nlabels == 3 || p.nlabels == 4 || p.nlabels == 8)) {
    return "Potts nlabels must be 2, 3, 4 or 8";
  }
  if (!(p.alpha >= 0.0) || !std::isfinite(p.alpha)) return "alpha must be finite and >= 0";
  if (p.c == 0.0) p.c = 0.3;
  if (!(p.c > 0.0) || !std::isfinite(p.c)) return "c must be > 0";
  if (p.relax == 0.0) p.relax = p.method == MF_RPADMM_FG ? 1.618 : (cmp ? 1.0 : 1.9);
  if (cmp) {
    if (p.relax != 1.0) return "pADMM-TY and ALG1 take no relaxation (relax 0 or 1)";
  } else if (p.method == MF_RPADMM_FG) {
    if (!(p.relax > 0.0 && p.relax < 0.5 * (1.0 + std::sqrt(5.0)))) return "FG relaxation r must be in (0, 1.618..)";
  } else if (!(p.relax > 0.0 && p.relax < 2.0)) {
    return "relaxation rho must be in (0, 2)";
  }
  const bool two = p.model == MF_TWO_LABEL;
  if (p.method == MF_CP_ALG1) {
    // |K^* K| <= |div^* div| + 2 (two labels) or + n + 1 (n labels)
    const double l2 = 4.0 * p.ndim + (two ? 2.0 : p.nlabels + 1.0);
    if (p.sigma == 0.0) p.sigma = 0.4;
    if (p.tau == 0.0) p.tau = 1.0 / (l2 * p.sigma);
    if (!(p.sigma > 0.0) || !(p.tau > 0.0)) return "sigma and tau must be > 0";
    if (p.sigma * p.tau * l2 > 1.0 + 1e-12) return "ALG1 needs sigma tau |K^*K| <= 1";
  }
  if (p.sigma == 0.0) p.sigma = two ? 0.2 : 5.0;
  if (p.tau == 0.0) p.tau = two ? 1.0 : 0.4;
  if (!(p.sigma > 0.0) || !(p.tau > 0.0)) return "sigma and tau must be > 0";
  const double amin = 4.0 * p.ndim;
  if (p.a == 0.0) p.a = amin;
  if (p.a < amin) return "a must be >= 4*ndim (||div^* div|| bound)";
  if (p.a_tilde == 0.0) p.a_tilde = 2.0;
  if (p.a_tilde < 2.0) return "a_tilde must be >= 2";
  if (p.a1 == 0.0) p.a1 = 2.0;
  if (p.a2 == 0.0) p.a2 = 2.0 * p.nlabels;
  if (p.a1 < 2.0) return "a1 must be >= 2";
  if (p.a2 < 2.0 * p.nlabels) return "a2 must be >= 2 n";
  if (p.max_iter < 0) return "max_iter must be >= 0";
  if (!(p.tol >= 0.0)) return "tol must be >= 0";
  if (p.check_every == 0) p.check_every = 10;
  if (p.check_every < 1) return "check_every must be >= 1";
  // default tile height: 16 rows, except 8 for BF16 Potts with n >= 8 and
  // for the BF16 3-D sweep, and 32 for the fused Potts rPDRQ pass with one
  // sweep (the measured fastest on gfx950 at 1024^2 and 256^3;
  // maxflow_tune picks per problem)
  if (p.tile_rows == 0) {
    if (p.method == MF_RPDRQ)
      p.tile_rows = (!two && p.ndim == 2 && p.gs_sweeps <= 1) ? 32 : 16;
    else
      p.tile_rows = (p.storage == MF_BF16 && ((!two && p.nlabels >= 8) || (two && p.ndim == 3))) ? 8 : 16;
  }
  if (p.tile_rows != 8 && p.tile_rows != 16 && p.tile_rows != 32) return "tile_rows must be 8, 16 or 32";
  if (!(p.promote_gap >= 0.0) || p.promote_iter < 0) return "promote_gap and promote_iter must be >= 0";
  if (p.slab_depth != 0 && p.slab_depth < 4) return "slab_depth must be 0 or >= 4";
  if (p.gs_sweeps == 0) p.gs_sweeps = 1;
  if (p.gs_sweeps < 1 || p.gs_sweeps > 64) return "gs_sweeps must be in 1..64";
  if (p.gs_sweeps > 1 && p.method != MF_RPDRQ) return "gs_sweeps applies to rPDRQ";
  if (p.relax0 != 0.0) {
    if (p.method != MF_RPADMM_EB) return "a relaxation schedule applies to rpADMMII (eb)";
    if (!(p.relax0 > 0.0) || !(p.relax0 <= p.relax)) return "relax0 must be in (0, relax]";
    if (p.relax_ramp < 1) return "relax_ramp must be >= 1";
  } else if (p.relax_ramp < 0) {
    return "relax_ramp must be >= 0";
  }
  {
    const bool d2ok = two && p.ndim == 2 && p.method != MF_RPDRQ && p.variant == MF_FUSED;
    if (p.depth == 0) p.depth = d2ok ? 2 : 1;
    if (p.depth != 1 && p.depth != 2) return "depth must be 1 or 2";
    if (p.depth == 2 && !d2ok) return "depth 2 applies to the fused two-label 2-D rpADMM sweep";
  }
  r.nl = two ? 1 : p.nlabels;
  r.ncap = two ? 2 : p.nlabels;
  if (p.cap_source != MF_CAPS_PLANES && p.cap_source != MF_CAPS_IMAGE) return "unknown cap_source";
  if (p.cap_power == 0) p.cap_power = 2;
  if (p.cap_power != 1 && p.cap_power != 2) return "cap_power must be 1 or 2";
  r.cg = CapGen{};
  if (p.cap_source == MF_CAPS_IMAGE) {
    for (int i = 0; i < r.ncap; i++)
      if (!std::isfinite(p.levels[i])) return "levels must be finite";
    r.cg.img = 1;
    r.cg.pw = p.cap_power;
    for (int i = 0; i < 8; i++) r.cg.lv[i] = i < r.ncap ? (float)p.levels[i] : 0.f;
  }
  r.ncp = r.cg.img ? 1 : r.ncap;
  r.g.ndim = p.ndim;
  if (p.ndim == 2) {
    r.g.H = (int)p.shape[0];
    r.g.W = (int)p.shape[1];
    r.g.D = 1;
  } else {
    r.g.D = (int)p.shape[0];
    r.g.H = (int)p.shape[1];
    r.g.W = (int)p.shape[2];
  }
  const long long n = r.g.npix();
  if (n > (1LL << 34)) return "grid too large";
  // Fused rpADMM sweeps use rows padded to a multiple of 4 elements, so every
  // owned group of a tile is one vector access whatever the width; the
  // element-wise kernels (unfused passes, in-place rPDRQ) use the dense layout.
  const bool padded = p.variant == MF_FUSED && !(p.ndim == 3 && p.model == MF_POTTS) &&
                      (p.method != MF_RPDRQ || (p.ndim == 2 && p.gs_sweeps <= fused_dr_sweeps(p.model)));
  r.g.pitch = padded ? (r.g.W + 3) / 4 * 4 : r.g.W;
  r.g.plane = plane_stride(r.g.nstore(), r.g.ndim);
  r.esz = p.storage == MF_BF16 ? 2 : 4;
  r.nq = r.nl * p.ndim;
  return "";
}

struct Layout {
  size_t ctrl, cap, state[2], stz, wbuf, wbuf_bytes, total;
  size_t state_bytes;
};

// rPDRQ as one tiled pass per iteration (2-D, fused variant, up to
// fused_dr_sweeps sweeps);
// otherwise three in-place element-wise launches.
bool dr_fused(const Resolved& r) {
  return r.p.method == MF_RPDRQ && r.p.variant == MF_FUSED && r.p.ndim == 2 &&
         r.p.gs_sweeps <= fused_dr_sweeps(r.p.model);
}

Layout plan(const Resolved& r) {
  Layout L{};
  const size_t P = (size_t)r.g.plane;
  size_t off = 0;
  L.ctrl = off;
  off = align_up(off + sizeof(Ctrl), 256);
  L.cap = off;
  off = align_up(off + (size_t)r.ncp * P * r.esz, 256);
  // state: u (nl f32) + q (nq) + ps (1) + p (nl) in storage type
  L.state_bytes = align_up((size_t)r.nl * P * 4, 256) + align_up((size_t)r.nq * P * r.esz, 256) +
                  align_up(P * r.esz, 256) + align_up((size_t)r.nl * P * r.esz, 256);
  if (r.p.method == MF_CP_ALG1) L.state_bytes += align_up((size_t)r.nl * P * 4, 256);   // u-bar
  L.state[0] = off;
  off += L.state_bytes;
  const bool dr = r.p.method == MF_RPDRQ;
  if (!dr || dr_fused(r)) {   // ping-pong buffers
    L.state[1] = off;
    off += L.state_bytes;
  } else {                    // the in-place rPDRQ launches
    L.state[1] = L.state[0];
  }
  // rPDRQ resolvent outputs (same shape as q, ps, p)
  L.stz = off;
  if (dr) off += L.state_bytes;
  // scratch planes: unfused w, or rPDRQ b (the fused rPDRQ pass keeps b in
  // LDS, but initialisation writes the resolvent outputs' u slot here)
  L.wbuf = off;
  const bool unfused = r.p.variant == MF_UNFUSED || (r.p.ndim == 3 && r.p.model == MF_POTTS);
  if (dr || unfused) off = align_up(off + (size_t)r.nl * P * 4, 256);
  L.wbuf_bytes = off - L.wbuf;
  L.total = off;
  return L;
}

StateView view(char* base, size_t off, const Resolved& r) {
  const size_t P = (size_t)r.g.plane;
  StateView v;
  char* b = base + off;
  v.u = (float*)b;
  b += align_up((size_t)r.nl * P * 4, 256);
  v.q = b;
  b += align_up((size_t)r.nq * P * r.esz, 256);
  v.ps = b;
  b += align_up(P * r.esz, 256);
  v.p = b;
  if (r.p.method == MF_CP_ALG1) {
    b += align_up((size_t)r.nl * P * r.esz, 256);
    v.ub = (float*)b;
  }
  return v;
}

}  // namespace

namespace mf {
// Parameter resolution shared with the pool.
std::string resolve_params(const mf_params* in, mf_params& out, Geom& g, int& nl, int& ncap) {
  Resolved r;
  const char* e = resolve(in, r);
  if (*e) return e;
  out = r.p;
  g = r.g;
  nl = r.nl;
  ncap = r.ncap;
  return "";
}
}  // namespace mf

struct mf_solver {
  Resolved r;
  Layout L;
  char* ws;
  hipStream_t stream;
  Ctrl* ctrl;
  void* cap;
  StateView st[2];
  StateView z;
  float* wbuf;
  int64_t iter;
  int off;          // iterate k lives in state buffer (k + off) & 1
  int* host_done;   // pinned polling slots
  hipEvent_t ev[8];
  int dev;
  bool fresh;       // the state is the initial point init_state set up
  bool pending;     // ... and iterate 0 is not in memory yet (see materialize)
};

namespace {

// rpADMMII relaxation of the step from iterate k: the constant relax, or
// the linear rise from relax0 (k = 0) to relax (k >= relax_ramp).
double rho_at(const mf_params& p, int64_t k) {
  if (p.relax0 == 0.0 || k >= p.relax_ramp) return p.relax;
  return p.relax0 + (p.relax - p.relax0) * ((double)k / (double)p.relax_ramp);
}

// Iterations k and k+1 share their coefficients (a depth-2 pass applies).
bool same_coef(const mf_params& p, int64_t k) { return p.relax0 == 0.0 || k >= p.relax_ramp; }

Coef coef_of(const Resolved& r, int64_t it) {
  const mf_params& p = r.p;
  Coef k;
  k.alpha = (float)p.alpha;
  k.inv_c = (float)(1.0 / p.c);
  k.c = (float)p.c;
  const bool eb = p.method == MF_RPADMM_EB;
  const double rho = eb ? rho_at(p, it) : 1.0;
  k.rho = (float)rho;
  k.omr = (float)(1.0 - rho);
  k.ku = eb ? (float)p.c : (float)(p.relax * p.c);
  k.inv_a = (float)(1.0 / p.a);
  if (p.model == MF_TWO_LABEL) {
    k.inv_a1 = (float)(1.0 / p.a_tilde);
    k.inv_a2 = (float)(1.0 / p.a_tilde);
  } else {
    k.inv_a1 = (float)(1.0 / p.a1);
    k.inv_a2 = (float)(1.0 / p.a2);
  }
  return k;
}

// State buffer of iterate k (rpADMM ping-pong).  A depth-1 sweep writes
// iterate k+1 into the other buffer; a depth-2 pass writes iterate k+2 into
// the other buffer and flips `off`.
int buf_of(const mf_solver* s, int64_t k) { return (int)((k + s->off) & 1); }

// The gap of the input iterate rides on the fused sweep: every fused rpADMM
// pass except 3-D Potts (which runs the per-operator kernels).
bool fused_gap(const mf_solver* s) {
  return s->r.p.variant == MF_FUSED && s->r.p.method != MF_RPDRQ &&
         (s->r.p.model == MF_TWO_LABEL || s->r.g.ndim == 2);
}

// One rpADMM sweep from iterate k (buffer k%2) to k+1.
hipError_t admm_sweep(mf_solver* s, int64_t k, bool check, bool write, const int* done) {
  SweepDesc d;
  d.g = s->r.g;
  d.nl = s->r.nl;
  d.two = s->r.p.model == MF_TWO_LABEL;
  d.bf16 = s->r.p.storage == MF_BF16;
  d.iso = s->r.p.tv == MF_TV_ISO;
  d.check = check;
  d.write = write;
  d.tile_rows = s->r.p.tile_rows;
  // the gap-carrying 3-D sweep runs 8-row tiles: at 16 rows its FP64 terms
  // and u staging take 214 VGPRs and 55 KB of LDS (two workgroups per CU),
  // at 8 rows 128 VGPRs and 32 KB (four).  The tile height never changes
  // the iterate.
  if (check && s->r.g.ndim == 3) d.tile_rows = 8;
  d.slab_depth = s->r.p.slab_depth;
  d.cap = s->cap;
  d.in = s->st[buf_of(s, k)];
  d.out = s->st[buf_of(s, k) ^ 1];
  d.wbuf = s->wbuf;
  d.k = coef_of(s->r, k);
  d.acc = &s->ctrl->acc[0][0];
  d.done = done;
  d.scheme = s->r.p.method == MF_PADMM_TY ? 1 : (s->r.p.method == MF_CP_ALG1 ? 2 : 0);
  d.sigma = (float)s->r.p.sigma;
  d.tau = (float)s->r.p.tau;
  d.cg = s->r.cg;
  d.stream = s->L.total > kStreamBytes;
  // Potts 3-D has no fused pass: it always runs the per-operator kernels
  if (s->r.p.variant == MF_UNFUSED || (s->r.g.ndim == 3 && s->r.p.model == MF_POTTS))
    return launch_unfused(d, s->stream);
  return launch_fused(d, s->stream);
}

// Depth-2 pass from iterate k to k+2 (two-label 2-D fused sweep); `flip`
// records that iterate k+2 now lives in the other buffer.
hipError_t admm_pass2(mf_solver* s, int64_t k, bool check, const int* done, bool flip = true) {
  SweepDesc d;
  d.g = s->r.g;
  d.nl = s->r.nl;
  d.two = true;
  d.bf16 = s->r.p.storage == MF_BF16;
  d.iso = s->r.p.tv == MF_TV_ISO;
  d.check = check;
  d.write = true;
  d.tile_rows = s->r.p.tile_rows;
  d.cap = s->cap;
  d.in = s->st[buf_of(s, k)];
  d.out = s->st[buf_of(s, k) ^ 1];
  d.wbuf = s->wbuf;
  d.k = coef_of(s->r, k);
  d.cg = s->r.cg;
  d.stream = s->L.total > kStreamBytes;
  d.acc = &s->ctrl->acc[0][0];
  d.done = done;
  const hipError_t e = launch_fused2d_d2(d, s->stream);
  if (e == hipSuccess && flip) s->off ^= 1;
  return e;
}

hipError_t dr_iter(mf_solver* s, int64_t k, bool keep_z, const int* done) {
  PdrqDesc d;
  d.g = s->r.g;
  d.nl = s->r.nl;
  d.two = s->r.p.model == MF_TWO_LABEL;
  d.bf16 = s->r.p.storage == MF_BF16;
  d.iso = s->r.p.tv == MF_TV_ISO;
  d.cap = s->cap;
  d.st = s->st[buf_of(s, k)];
  d.out = s->st[buf_of(s, k) ^ 1];   // the same buffer for the in-place launches
  d.z = s->z;
  d.b = s->wbuf;
  d.fused = dr_fused(s->r);
  d.tile_rows = s->r.p.tile_rows;
  d.sigma = (float)s->r.p.sigma;
  d.tau = (float)s->r.p.tau;
  d.rho = (float)s->r.p.relax;
  d.inv_st = (float)(1.0 / (s->r.p.sigma * s->r.p.tau));
  d.alpha = (float)s->r.p.alpha;
  d.keep_z = keep_z;
  d.sweeps = s->r.p.gs_sweeps;
  d.done = done;
  d.cg = s->r.cg;
  d.stream = s->L.total > kStreamBytes;
  return launch_pdrq_iter(d, s->stream);
}

// Standalone gap of the current iterate into ctrl->acc.
hipError_t gap_of(mf_solver* s, int64_t k, const int* done) {
  GapDesc d;
  d.g = s->r.g;
  d.nl = s->r.nl;
  d.two = s->r.p.model == MF_TWO_LABEL;
  d.bf16 = s->r.p.storage == MF_BF16;
  d.iso = s->r.p.tv == MF_TV_ISO;
  d.cap = s->cap;
  if (s->r.p.method == MF_RPDRQ) {
    d.st = s->z;
    d.st.u = s->st[buf_of(s, k)].u;
  } else {
    d.st = s->st[buf_of(s, k)];
  }
  d.acc = &s->ctrl->acc[0][0];
  d.done = done;
  d.cg = s->r.cg;
  return launch_gap(d, s->stream);
}

long long nres(const mf_solver* s) { return s->r.g.npix() * s->r.nl; }
double neg_tol(const mf_solver* s) { return neg_gap_tol(s->r.p.storage == MF_BF16); }

// Two-label fused rpADMM with capacity planes and depth-1 sweeps: a solve's
// first iteration from the initial point runs pointwise (k_first_two) and
// needs neither iterate 0 in memory nor a sweep.
bool first_pointwise(const mf_solver* s) {
  const mf_params& p = s->r.p;
  return p.model == MF_TWO_LABEL && p.variant == MF_FUSED &&
         (p.method == MF_RPADMM_FG || p.method == MF_RPADMM_EB) && !s->r.cg.img && p.depth != 2;
}

// Store iterate 0 if init_state left it out.
mf_status materialize(mf_solver* s) {
  if (!s->pending) return MF_OK;
  HIP_TRY(launch_init(s->r.g, s->r.nl, s->r.p.model == MF_TWO_LABEL, s->r.p.storage == MF_BF16, s->cap,
                      s->r.cg, s->st[0], s->stream));
  s->pending = false;
  return MF_OK;
}

// The initial point.  Where a solve's first iteration runs pointwise, iterate
// 0 is stored only when something else needs it (any entry point but a
// solve, or a solve that stops at iterate 0): the 256^3 solve then skips a
// 105 us pass.
mf_status init_state(mf_solver* s) {
  s->pending = first_pointwise(s);
  if (!s->pending)
    HIP_TRY(launch_init(s->r.g, s->r.nl, s->r.p.model == MF_TWO_LABEL, s->r.p.storage == MF_BF16, s->cap,
                        s->r.cg, s->st[0], s->stream));
  if (s->r.p.method == MF_RPDRQ) {
    if (s->L.wbuf_bytes < (size_t)s->r.nl * (size_t)s->r.g.plane * 4)
      return fail(MF_EDEVICE, "internal: rPDRQ layout without its scratch planes");
    StateView z = s->z;
    // resolvent outputs of "iteration 0" := the initial flows
    HIP_TRY(launch_init(s->r.g, s->r.nl, s->r.p.model == MF_TWO_LABEL, s->r.p.storage == MF_BF16, s->cap,
                        s->r.cg, StateView{s->wbuf, z.q, z.ps, z.p}, s->stream));
  }
  if (s->r.p.method == MF_CP_ALG1)   // u-bar^0 = u^0 = 0
    HIP_TRY(hipMemsetAsync(s->st[0].ub, 0, (size_t)s->r.nl * (size_t)s->r.g.plane * 4, s->stream));
  HIP_TRY(launch_ctrl_reset(s->ctrl, s->stream));
  s->iter = 0;
  s->off = 0;
  s->fresh = true;
  return MF_OK;
}

void fill_gap(const Ctrl& c, int64_t iter, mf_gap* out, int32_t status) {
  if (!out) return;
  out->iter = iter;
  out->primal = c.last[0];
  out->dual = c.last[1];
  out->rel_gap = c.last[2];
  out->resid_rms = c.last[3];
  out->flow = c.last[4];
  out->status = status;
}

// Checked iterates whose decision the host has not seen yet, with the buffer
// offset in effect at each (depth-2 passes flip it): once the solve has
// stopped, the accepted iterate's offset is looked up here.  The host keeps
// at most a few chunks unobserved, so a short ring suffices.
struct OffRing {
  static constexpr int kN = 32;
  int64_t k[kN];
  int off[kN];
  int n = 0;
  void push(int64_t kk, int o) {
    k[n % kN] = kk;
    off[n % kN] = o;
    n++;
  }
  bool find(int64_t kk, int& o) const {
    for (int i = 0; i < kN && i < n; i++) {
      const int j = (n - 1 - i) % kN;
      if (k[j] == kk) {
        o = off[j];
        return true;
      }
    }
    return false;
  }
};

// Chunks between the synchronous polls of the allocation-free solve.
constexpr int kSyncPollChunks = 4;

// The solve loop behind maxflow_solve and maxflow_solve_static: chunks of
// check_every iterations, each opened by the gap check of its first iterate
// and the on-GPU decision; later sweeps of a stopped solve exit at once.  The
// host follows the decisions either through pinned slots and events (at
// most `lookahead` unobserved chunks queued) or, with `sync_poll`, through a
// synchronous 4-byte read every kSyncPollChunks chunks (no pinned memory and
// no events: nothing is allocated).
mf_status solve_loop(mf_solver* s, mf_gap* out, bool sync_poll) {
  const mf_params& p = s->r.p;
  const int64_t max_iter = std::max<int64_t>(p.max_iter, s->iter);
  const int ce = p.check_every;
  const bool dr = p.method == MF_RPDRQ;
  const int* done = &s->ctrl->done;
  // iterate 0 must be in memory unless the first check runs pointwise
  if (!(s->fresh && s->iter == 0 && max_iter > 0 && first_pointwise(s))) {
    const mf_status ms = materialize(s);
    if (ms != MF_OK) return ms;
  }
  HIP_TRY(launch_ctrl_reset(s->ctrl, s->stream));
  int64_t k = s->iter;
  const bool d2 = p.depth == 2;
  OffRing off_at;
  // polling ring: the decision of each chunk's check sits in pinned slot
  // (chunk & 7), its copy marked by an event
  int issued = 0, observed = 0;
  // Each chunk's decision is copied out right after its gap-carrying sweep,
  // ahead of the chunk's other sweeps.  Unobserved decisions kept in
  // flight: enough that the GPU still has queued work while the host turns
  // around to launch the next chunk, and no more, since every sweep queued
  // past the stop still dispatches its grid (to exit at once, ~10 us for a
  // 256^3 sweep).  A chunk's length is estimated from its state traffic (one
  // state read and write per iteration, ~5 TB/s): from ~0.2 ms per chunk the
  // host waits for the current chunk's decision while the GPU runs the
  // chunk's other sweeps; from ~60 us it keeps one decision more in flight,
  // below that three.
  const double chunk_us = (double)ce * 2.0 * (double)s->L.state_bytes / 5.0e6;
  const int lookahead = chunk_us >= 200.0 ? 0 : (chunk_us >= 60.0 ? 1 : 3);
  bool stop = false;
  while (!stop) {
    // ---- gap of iterate k and the decision
    const bool final_check = k >= max_iter;
    const int64_t n = final_check ? 0 : std::min<int64_t>(ce, max_iter - k);
    // the solve's first check on the initial point of a two-label rpADMM
    // solve with capacity planes runs pointwise (see k_first_two): 256^3
    // solve 4.30 -> 4.22 ms.  Not with depth-2 passes, where it would replace
    // a two-iteration pass and add a launch (2048^2 0.572 -> 0.583 ms).
    const bool first = k == 0 && s->fresh && first_pointwise(s) && !final_check;
    s->fresh = false;
    off_at.push(k, s->off);
    int64_t j = 1;   // iterations of the chunk issued with the check
    if (dr) {
      HIP_TRY(gap_of(s, k, done));
    } else if (first) {
      // the first iteration from the initial point is pointwise (q stays 0)
      HIP_TRY(launch_first_two(s->r.g, p.storage == MF_BF16, s->cap, s->st[buf_of(s, k) ^ 1], coef_of(s->r, k),
                               &s->ctrl->acc[0][0], s->stream));
    } else if (fused_gap(s)) {
      if (d2 && n >= 2 && same_coef(p, k)) {
        HIP_TRY(admm_pass2(s, k, true, done));
        j = 2;
      } else {
        HIP_TRY(admm_sweep(s, k, true, !final_check, done));
      }
    } else {
      HIP_TRY(gap_of(s, k, done));
      if (!final_check) HIP_TRY(admm_sweep(s, k, false, true, done));
    }
    HIP_TRY(launch_bookkeep(s->ctrl, k, p.alpha, p.tol, neg_tol(s), nres(s), final_check ? 1 : 0, 1, s->stream));
    if (final_check) break;
    issued++;
    if (!sync_poll) {
      // the decision at k, copied into pinned slot (chunk & 7) and marked by
      // an event (no kernel of this library stores into host memory: only
      // the runtime's copies write there)
      const int slot = (issued - 1) & 7;
      HIP_TRY(hipMemcpyAsync(s->host_done + slot, done, sizeof(int), hipMemcpyDeviceToHost, s->stream));
      HIP_TRY(hipEventRecord(s->ev[slot], s->stream));
    }
    // ---- the rest of the chunk
    if (dr) {
      for (int64_t i = 0; i < n; i++) HIP_TRY(dr_iter(s, k + i, i == n - 1, done));
    } else {
      while (j < n) {
        if (d2 && n - j >= 2 && same_coef(p, k + j)) {
          HIP_TRY(admm_pass2(s, k + j, false, done));
          j += 2;
        } else {
          HIP_TRY(admm_sweep(s, k + j, false, true, done));
          j += 1;
        }
      }
    }
    k += n;
    if (sync_poll) {
      if (issued % kSyncPollChunks == 0) {
        int flag = 0;
        HIP_TRY(hipMemcpyAsync(&flag, done, sizeof(int), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        if (flag) stop = true;
      }
      continue;
    }
    // ---- follow the decisions without stalling the queue
    while (observed < issued) {
      const int os = observed & 7;
      const hipError_t q =
          (issued - observed > lookahead) ? hipEventSynchronize(s->ev[os]) : hipEventQuery(s->ev[os]);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return fail(MF_EDEVICE, "event", hipGetErrorString(q));
      if (s->host_done[os]) stop = true;
      observed++;
    }
  }
  Ctrl c;
  HIP_TRY(hipMemcpyAsync(&c, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (!c.done) return fail(MF_EDEVICE, "solve ended without a decision");
  int off = s->off;
  if (!off_at.find(c.iter, off)) return fail(MF_EDEVICE, "internal: accepted iterate outside the polling window");
  s->iter = c.iter;
  s->off = off;
  if (s->pending) {   // a stop at iterate 0 keeps it; any later one has overwritten its buffer
    if (c.iter == 0) {
      const mf_status ms = materialize(s);
      if (ms != MF_OK) return ms;
      HIP_TRY(hipStreamSynchronize(s->stream));
    }
    s->pending = false;
  }
  const mf_status st = (mf_status)c.status;
  fill_gap(c, s->iter, out, st);
  if (st == MF_EDIVERGED) return fail(MF_EDIVERGED, "non-finite or negative gap");
  return st;
}

}  // namespace

extern "C" {

const char* maxflow_last_error(void) { return g_err; }

size_t maxflow_workspace_bytes(const mf_params* p) {
  Resolved r;
  const char* e = resolve(p, r);
  if (*e) {
    set_err(e);
    return 0;
  }
  return plan(r).total;
}

mf_status maxflow_create(const mf_params* p, const float* cap, void* workspace, size_t ws_bytes,
                         void* hip_stream, mf_solver** out) {
  if (!out) return fail(MF_EINVAL, "out is null");
  *out = nullptr;
  Resolved r;
  const char* e = resolve(p, r);
  if (*e) return fail(MF_EINVAL, e);
  if (!cap || !workspace) return fail(MF_EINVAL, "cap and workspace must be device pointers");
  if (((uintptr_t)workspace) & 255) return fail(MF_EINVAL, "workspace must be 256-byte aligned");
  const Layout L = plan(r);
  if (ws_bytes < L.total)
    return fail(MF_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes (maxflow_workspace_bytes)");
  mf_solver* s = new (std::nothrow) mf_solver();
  if (!s) return fail(MF_ENOMEM, "host allocation failed");
  s->r = r;
  s->L = L;
  s->ws = (char*)workspace;
  s->stream = (hipStream_t)hip_stream;
  s->ctrl = (Ctrl*)(s->ws + L.ctrl);
  s->cap = s->ws + L.cap;
  s->st[0] = view(s->ws, L.state[0], r);
  s->st[1] = view(s->ws, L.state[1], r);
  s->z = view(s->ws, L.stz, r);
  s->wbuf = (float*)(s->ws + L.wbuf);
  if (hipGetDevice(&s->dev) != hipSuccess) {
    delete s;
    return fail(MF_EDEVICE, "hipGetDevice failed");
  }
  if (hipHostMalloc((void**)&s->host_done, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    delete s;
    return fail(MF_EDEVICE, "pinned host allocation failed");
  }
  for (int i = 0; i < 8; i++) {
    if (hipEventCreateWithFlags(&s->ev[i], hipEventDisableTiming) != hipSuccess) {
      for (int j = 0; j < i; j++) hipEventDestroy(s->ev[j]);
      hipHostFree(s->host_done);
      delete s;
      return fail(MF_EDEVICE, "event creation failed");
    }
  }
  hipError_t he = launch_pitch_copy(cap, false, r.g.npix(), r.g.W, s->cap, r.p.storage == MF_BF16, r.g.plane,
                                    r.g.pitch, r.g.W, (long long)r.g.H * r.g.D, r.ncp, s->stream);
  if (he != hipSuccess) {
    maxflow_destroy(s);
    return fail(MF_EDEVICE, "capacity copy", hipGetErrorString(he));
  }
  mf_status st = init_state(s);
  if (st != MF_OK) {
    maxflow_destroy(s);
    return st;
  }
  // the caller may free `cap` on return: make the copy complete
  if (hipStreamSynchronize(s->stream) != hipSuccess) {
    maxflow_destroy(s);
    return fail(MF_EDEVICE, "stream synchronize failed");
  }
  *out = s;
  return MF_OK;
}

mf_status maxflow_reset(mf_solver* s) {
  if (!s) return fail(MF_EINVAL, "null solver");
  return init_state(s);
}

int64_t maxflow_iter(const mf_solver* s) { return s ? s->iter : -1; }

mf_status maxflow_step(mf_solver* s, int32_t iters) {
  if (!s) return fail(MF_EINVAL, "null solver");
  if (iters < 0) return fail(MF_EINVAL, "iters must be >= 0");
  {
    const mf_status ms = materialize(s);
    if (ms != MF_OK) return ms;
  }
  if (iters > 0) s->fresh = false;
  const bool d2 = s->r.p.depth == 2;
  for (int32_t i = 0; i < iters;) {
    if (s->r.p.method == MF_RPDRQ) {
      HIP_TRY(dr_iter(s, s->iter, i == iters - 1, nullptr));
    } else if (d2 && iters - i >= 2 && same_coef(s->r.p, s->iter)) {
      HIP_TRY(admm_pass2(s, s->iter, false, nullptr));
      s->iter += 1;
      i += 1;
    } else {
      HIP_TRY(admm_sweep(s, s->iter, false, true, nullptr));
    }
    s->iter += 1;
    i += 1;
  }
  return MF_OK;
}

mf_status maxflow_gap(mf_solver* s, mf_gap* out) {
  if (!s) return fail(MF_EINVAL, "null solver");
  {
    const mf_status ms = materialize(s);
    if (ms != MF_OK) return ms;
  }
  HIP_TRY(launch_ctrl_reset(s->ctrl, s->stream));
  HIP_TRY(gap_of(s, s->iter, nullptr));
  HIP_TRY(launch_bookkeep(s->ctrl, s->iter, s->r.p.alpha, 0.0, neg_tol(s), nres(s), 0, 0, s->stream));
  Ctrl c;
  HIP_TRY(hipMemcpyAsync(&c, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  const bool bad = !std::isfinite(c.last[0]) || !std::isfinite(c.last[1]) || !std::isfinite(c.last[3]) ||
                   c.last[2] < -neg_tol(s);
  fill_gap(c, s->iter, out, bad ? MF_EDIVERGED : MF_OK);
  return bad ? fail(MF_EDIVERGED, "non-finite or negative gap") : MF_OK;
}

mf_status maxflow_solve(mf_solver* s, mf_gap* out) {
  if (!s) return fail(MF_EINVAL, "null solver");
  return solve_loop(s, out, false);
}

mf_status maxflow_read_u(mf_solver* s, float* dst) { return maxflow_read_field(s, 0, dst); }

mf_status maxflow_labels(mf_solver* s, int32_t* dst) {
  if (!s || !dst) return fail(MF_EINVAL, "null argument");
  {
    const mf_status ms = materialize(s);
    if (ms != MF_OK) return ms;
  }
  const StateView& v = s->st[buf_of(s, s->iter)];
  HIP_TRY(launch_labels(s->r.g, s->r.nl, s->r.p.model == MF_TWO_LABEL, v.u, dst, s->stream, s->r.g.pitch));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MF_OK;
}

static mf_status field_ptr(mf_solver* s, int32_t field, void** ptr, int* np, bool* is_u) {
  const bool dr = s->r.p.method == MF_RPDRQ;
  const StateView& v = s->st[buf_of(s, s->iter)];
  *is_u = false;
  switch (field) {
    case 0: *ptr = v.u; *np = s->r.nl; *is_u = true; return MF_OK;
    case 1: *ptr = v.q; *np = s->r.nq; return MF_OK;
    case 2: *ptr = v.ps; *np = 1; return MF_OK;
    case 3: *ptr = v.p; *np = s->r.nl; return MF_OK;
    case 4: case 5: case 6:
      if (!dr) return fail(MF_EINVAL, "resolvent fields exist only for rPDRQ");
      *ptr = field == 4 ? s->z.q : (field == 5 ? s->z.ps : s->z.p);
      *np = field == 4 ? s->r.nq : (field == 5 ? 1 : s->r.nl);
      return MF_OK;
    default: return fail(MF_EINVAL, "unknown field");
  }
}

mf_status maxflow_read_field(mf_solver* s, int32_t field, float* dst) {
  if (!s || !dst) return fail(MF_EINVAL, "null argument");
  {
    const mf_status ms = materialize(s);
    if (ms != MF_OK) return ms;
  }
  void* ptr;
  int np;
  bool is_u;
  mf_status e = field_ptr(s, field, &ptr, &np, &is_u);
  if (e != MF_OK) return e;
  const Geom& g = s->r.g;
  HIP_TRY(launch_pitch_copy(ptr, is_u ? false : s->r.p.storage == MF_BF16, g.plane, g.pitch, dst, false, g.npix(),
                            g.W, g.W, (long long)g.H * g.D, np, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MF_OK;
}

mf_status maxflow_write_field(mf_solver* s, int32_t field, const float* src) {
  if (!s || !src) return fail(MF_EINVAL, "null argument");
  {
    const mf_status ms = materialize(s);
    if (ms != MF_OK) return ms;
  }
  s->fresh = false;
  void* ptr;
  int np;
  bool is_u;
  mf_status e = field_ptr(s, field, &ptr, &np, &is_u);
  if (e != MF_OK) return e;
  const Geom& g = s->r.g;
  HIP_TRY(launch_pitch_copy(src, false, g.npix(), g.W, ptr, is_u ? false : s->r.p.storage == MF_BF16, g.plane,
                            g.pitch, g.W, (long long)g.H * g.D, np, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MF_OK;
}

size_t maxflow_state_bytes(const mf_solver* s) {
  if (!s) return 0;
  return s->r.p.method == MF_RPDRQ ? 2 * s->L.state_bytes : s->L.state_bytes;
}

mf_status maxflow_export_state(mf_solver* s, void* dst) {
  if (!s || !dst) return fail(MF_EINVAL, "null argument");
  {
    const mf_status ms = materialize(s);
    if (ms != MF_OK) return ms;
  }
  const bool dr = s->r.p.method == MF_RPDRQ;
  const size_t off = s->L.state[buf_of(s, s->iter)];
  HIP_TRY(hipMemcpyAsync(dst, s->ws + off, s->L.state_bytes, hipMemcpyDeviceToDevice, s->stream));
  if (dr)
    HIP_TRY(hipMemcpyAsync((char*)dst + s->L.state_bytes, s->ws + s->L.stz, s->L.state_bytes,
                           hipMemcpyDeviceToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MF_OK;
}

mf_status maxflow_import_state(mf_solver* s, const void* src, int64_t iter) {
  if (!s || !src) return fail(MF_EINVAL, "null argument");
  if (iter < 0) return fail(MF_EINVAL, "iter must be >= 0");
  s->fresh = false;
  s->pending = false;   // the import overwrites the state it would have held
  const bool dr = s->r.p.method == MF_RPDRQ;
  s->iter = iter;
  const size_t off = s->L.state[buf_of(s, iter)];
  HIP_TRY(hipMemcpyAsync(s->ws + off, src, s->L.state_bytes, hipMemcpyDeviceToDevice, s->stream));
  if (dr)
    HIP_TRY(hipMemcpyAsync(s->ws + s->L.stz, (const char*)src + s->L.state_bytes, s->L.state_bytes,
                           hipMemcpyDeviceToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MF_OK;
}

mf_status maxflow_tune(mf_solver* s, int32_t sweeps, int32_t what, mf_tuning* out) {
  if (!s || !out) return fail(MF_EINVAL, "null solver or out");
  {
    const mf_status ms = materialize(s);
    if (ms != MF_OK) return ms;
  }
  if (sweeps < 1 || sweeps > 10000) return fail(MF_EINVAL, "sweeps must be in 1..10000");
  mf_params& p = s->r.p;
  *out = mf_tuning{};
  const bool dr = p.method == MF_RPDRQ;
  const bool fused = p.variant == MF_FUSED;
  const bool two = p.model == MF_TWO_LABEL;
  const bool d3 = s->r.g.ndim == 3;
  // the candidate list: the free knobs range over their values, the others
  // keep the solver's
  std::vector<mf_tune_cand> cand;
  const std::vector<int> rows_all = {8, 16, 32}, depth_all = {1, 2}, slab_all = {4, 8, 16, 32};
  const std::vector<int> rows_l = (what & MF_TUNE_TILE) ? rows_all : std::vector<int>{p.tile_rows};
  const std::vector<int> depth_l = (what & MF_TUNE_DEPTH) ? depth_all : std::vector<int>{p.depth};
  int shape_kind = 0;   // 0: no launch-shape choice
  if (dr && dr_fused(s->r) && p.gs_sweeps == 1) shape_kind = 1;   // fused rPDRQ, one sweep: 16 or 32 rows
  else if (!dr && fused && !d3 && two) shape_kind = 2;   // depth 1: 8/16/32 rows; depth 2: 16/32
  else if (!dr && fused && !d3) shape_kind = 3;          // Potts: 8/16/32 rows (8/16 for n > 4)
  else if (!dr && fused && d3 && two) shape_kind = 4;    // 3-D: 8/16 rows x slab depths
  // the slab depth only shapes the 3-D sweep
  const std::vector<int> slab_l =
      (shape_kind == 4 && (what & MF_TUNE_SLAB)) ? slab_all : std::vector<int>{p.slab_depth};
  for (int rows : rows_l)
    for (int depth : depth_l)
      for (int slab : slab_l) {
        bool ok = false;
        switch (shape_kind) {
          case 1: ok = (rows == 16 || rows == 32) && depth == 1; break;
          case 2: ok = depth == 1 || rows != 8; break;
          case 3: ok = depth == 1 && !(rows == 32 && p.nlabels > 4); break;
          case 4: ok = rows != 32 && depth == 1; break;
          default: ok = false;
        }
        if (ok) cand.push_back(mf_tune_cand{rows, depth, slab, 0.0});
      }
  if (cand.empty() && !(dr && !dr_fused(s->r)))   // the one configuration
    cand.push_back(mf_tune_cand{p.tile_rows, p.depth, p.slab_depth, 0.0});
  if ((int)cand.size() > 16) cand.resize(16);
  out->tile_rows = p.tile_rows;
  out->depth = p.depth;
  out->slab_depth = p.slab_depth;
  if (cand.empty()) return MF_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(MF_EDEVICE, "event creation failed");
  }
  const mf_params keep = p;
  int best = -1;
  hipError_t he = hipSuccess;
  for (size_t c = 0; c < cand.size() && he == hipSuccess; c++) {
    p.tile_rows = cand[c].tile_rows;
    p.depth = cand[c].depth;
    p.slab_depth = cand[c].slab_depth;
    const bool d2 = p.depth == 2;
    float ms = 0.f;
    // iterate k -> k+1 (or k+2) repeatedly: the buffer of iterate k is only
    // read, the other one is scratch until the next real pass
    for (int w = 0; w < 2 + sweeps && he == hipSuccess; w++) {
      if (w == 2) he = hipEventRecord(e0, s->stream);
      if (he != hipSuccess) break;
      if (dr) he = dr_iter(s, s->iter, false, nullptr);
      else if (d2) he = admm_pass2(s, s->iter, false, nullptr, false);
      else he = admm_sweep(s, s->iter, false, true, nullptr);
    }
    if (he == hipSuccess) he = hipEventRecord(e1, s->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) break;
    cand[c].us_per_iter = 1e3 * (double)ms / sweeps / (d2 ? 2 : 1);
    if (best < 0 || cand[c].us_per_iter < cand[best].us_per_iter) best = (int)c;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  p = keep;
  if (he != hipSuccess) return fail(MF_EDEVICE, "tuning pass", hipGetErrorString(he));
  p.tile_rows = cand[best].tile_rows;
  p.depth = cand[best].depth;
  p.slab_depth = cand[best].slab_depth;
  out->tile_rows = p.tile_rows;
  out->depth = p.depth;
  out->slab_depth = p.slab_depth;
  out->ncand = (int32_t)cand.size();
  for (size_t c = 0; c < cand.size(); c++) out->cand[c] = cand[c];
  return MF_OK;
}

mf_status maxflow_destroy(mf_solver* s) {
  if (!s) return MF_OK;
  hipStreamSynchronize(s->stream);
  for (int i = 0; i < 8; i++)
    if (s->ev[i]) hipEventDestroy(s->ev[i]);
  if (s->host_done) hipHostFree(s->host_done);
  delete s;
  return MF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free solve: the workspace is a static device array, one per
// device the library runs on (held until the process ends).  In host code
// `scratch` names a host-side stand-in, not a device address: host code uses
// only the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[MF_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (current), looked up once per
// device and kept.
hipError_t scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" mf_status maxflow_solve_static(const mf_params* p, const float* cap, float* u_dst, int32_t* labels_dst,
                                          mf_gap* out, void* hip_stream) {
  Resolved r;
  const char* e = resolve(p, r);
  if (*e) return fail(MF_EINVAL, e);
  if (!cap) return fail(MF_EINVAL, "cap must be a device pointer");
  const Layout L = plan(r);
  if (L.total > (size_t)MF_STATIC_SCRATCH_BYTES) {
    snprintf(g_err, sizeof(g_err),
             "problem needs %zu bytes of workspace; the static scratch holds %zu (use maxflow_create)", L.total,
             (size_t)MF_STATIC_SCRATCH_BYTES);
    return MF_ENOMEM;
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  void* ws = nullptr;
  HIP_TRY(scratch_ptr(dev, &ws));
  // the solver lives on this stack frame: no pinned polling slots, no events
  mf_solver s{};
  s.r = r;
  s.L = L;
  s.ws = (char*)ws;
  s.stream = (hipStream_t)hip_stream;
  s.ctrl = (Ctrl*)(s.ws + L.ctrl);
  s.cap = s.ws + L.cap;
  s.st[0] = view(s.ws, L.state[0], r);
  s.st[1] = view(s.ws, L.state[1], r);
  s.z = view(s.ws, L.stz, r);
  s.wbuf = (float*)(s.ws + L.wbuf);
  s.host_done = nullptr;
  s.dev = dev;
  HIP_TRY(launch_pitch_copy(cap, false, r.g.npix(), r.g.W, s.cap, r.p.storage == MF_BF16, r.g.plane, r.g.pitch,
                            r.g.W, (long long)r.g.H * r.g.D, r.ncp, s.stream));
  mf_status st = init_state(&s);
  if (st != MF_OK) return st;
  st = solve_loop(&s, out, true);
  if (st != MF_OK && st != MF_ENOTCONV && st != MF_EDIVERGED) return st;
  const StateView& v = s.st[buf_of(&s, s.iter)];
  const Geom& g = r.g;
  if (u_dst)
    HIP_TRY(launch_pitch_copy(v.u, false, g.plane, g.pitch, u_dst, false, g.npix(), g.W, g.W, (long long)g.H * g.D,
                              r.nl, s.stream));
  if (labels_dst)
    HIP_TRY(launch_labels(g, r.nl, r.p.model == MF_TWO_LABEL, v.u, labels_dst, s.stream, g.pitch));
  HIP_TRY(hipStreamSynchronize(s.stream));
  return st;
}
