// Kernel launch descriptors shared by the host runtime (capi.cpp) and the
// kernel translation units.  Only plain pointers and sizes cross this line.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_device.h"

namespace mf {

// Device control block of one solve: gap accumulators, the last evaluated
// gap and the convergence decision.  Written only by the bookkeeping kernel
// (decision) and by the gap reductions (atomics into acc); sweeps read `done`.
constexpr int kAccSlots = 64;   // blocks spread their atomics over this many slots

struct Ctrl {
  double acc[kAccSlots][8];  // per slot: data, tv, dual, residual^2, flow (FP64 partial sums)
  double last[8];    // primal, dual, rel_gap, resid_rms, flow, iter
  long long iter;    // iterate at which the solve stopped
  int done;          // 0 running, 1 stopped
  int status;        // MF_OK / MF_ENOTCONV / MF_EDIVERGED when done
  long long checks;  // number of gap evaluations so far
  int pad[6];
};

struct Geom {
  int ndim;
  int W, H, D;       // D = 1 in 2-D
  int pitch;         // row stride in elements (>= W; padded layouts round W up to 4)
  long long plane;   // element stride between planes (>= pitch * H * D)
  long long npix() const { return (long long)W * H * D; }
  long long nstore() const { return (long long)pitch * H * D; }
};

// Element stride between the planes of a workspace: the stored plane rounded
// up to 128 elements, plus a pad.  Without it a 1024^2, 4096^2 or 256^3 FP32
// plane has a large power-of-two stride, so the same pixel of the 7 to 41
// planes a sweep reads and writes at once sits at addresses that differ only
// in high bits, and the DRAM accesses of the planes collide.  The pads are
// measured ones (fused FP32 sweeps, µs per sweep, no pad -> pad): 2-D 2176
// elements, two-label 4096^2 depth 1 158.9 -> 151.9, Potts n = 8 1024^2
// 67.8 -> 66.9, n = 4 26.5 -> 25.9; 3-D 128 elements, 256^3 204.0 -> 201.2.
// Not every pad helps (256 elements: 162 and 208).  The layout changes no
// value.
inline long long plane_stride(long long nstore, int ndim) {
  return (nstore + 127) / 128 * 128 + (ndim == 3 ? 128 : 2176);
}

// One state buffer (all planes of one iterate).
struct StateView {
  float* u;    // NL planes (FP32 always)
  void* q;     // NL * ndim planes (storage type)
  void* ps;    // 1 plane
  void* p;     // NL planes
  float* ub = nullptr;   // ALG1 only: extrapolated u-bar, NL planes FP32
};

struct SweepDesc {
  Geom g;
  int nl;          // 1 for the two-label model, n for Potts
  bool two;        // two-label model (p = p_t, extra clip of p_s at C_s)
  bool bf16;       // storage type of flows and capacities
  bool iso;        // isotropic projection
  bool check;      // accumulate the gap of the input iterate (fused only)
  bool write;      // write the output iterate
  int tile_rows;   // fused 2-D tile height
  int slab_depth = 0;   // fused 3-D: planes per z-slab (0: one wave of workgroups)
  const void* cap;
  StateView in, out;
  float* wbuf;     // unfused: NL planes of w
  Coef k;
  double* acc;     // Ctrl::acc of this solve
  const int* done; // Ctrl::done of this solve, or nullptr
  int scheme = 0;  // element-wise passes: 0 rpADMM, 1 pADMM-TY, 2 ALG1
  float sigma = 0.f, tau = 0.f;   // ALG1 step sizes
  CapGen cg;       // cg.img: `cap` is one image plane
  bool stream = false;   // working set beyond the last-level cache: strip tile order, non-temporal stores
};

struct GapDesc {
  Geom g;
  int nl;
  bool two, bf16, iso;
  const void* cap;
  StateView st;    // iterate (for rPDRQ: u plus the resolvent outputs)
  double* acc;
  const int* done;
  CapGen cg;
};

struct PdrqDesc {
  Geom g;
  int nl;
  bool two, bf16, iso;
  const void* cap;
  StateView st;        // u and the reflected variables (q-bar, p_s-bar, p-bar) of iterate k
  StateView out;       // iterate k+1: = st for the in-place launches, the other buffer when fused
  StateView z;         // resolvent outputs (written when `keep_z`)
  float* b;            // NL planes of the right-hand side b^k
  float sigma, tau, rho, inv_st, alpha;
  bool keep_z;
  bool fused;          // one tiled pass (2-D, padded rows, 1 to 4 sweeps; tile_rows 16 or 32 for one)
  int tile_rows;
  int sweeps = 1;      // symmetric red-black GS sweeps (in-place launches; the fused pass runs 1)
  const int* done;
  CapGen cg;
  bool stream = false;   // as in SweepDesc
};

// Working sets (capacities and both state buffers) above this many bytes do
// not stay in the 256 MB last-level cache between sweeps: their sweeps take
// the strip tile order and non-temporal stores (measured faster there and
// slower on smaller working sets).
#ifndef MF_STREAM_MIB
#define MF_STREAM_MIB 384
#endif
constexpr size_t kStreamBytes = (size_t)MF_STREAM_MIB << 20;

hipError_t launch_fused(const SweepDesc& d, hipStream_t s);
hipError_t launch_fused2d_d2(const SweepDesc& d, hipStream_t s);
hipError_t launch_unfused(const SweepDesc& d, hipStream_t s);
hipError_t launch_gap(const GapDesc& d, hipStream_t s);
hipError_t launch_pdrq_iter(const PdrqDesc& d, hipStream_t s);

// misc kernels
hipError_t launch_init(const Geom& g, int nl, bool two, bool bf16, const void* cap, const CapGen& cg,
                       StateView st, hipStream_t s);
hipError_t launch_first_two(const Geom& g, bool bf16, const void* cap, const StateView& out, const Coef& k,
                            double* acc, hipStream_t s);
hipError_t launch_convert_caps(const float* src, void* dst, long long n_per_plane, int nplanes,
                               long long plane, bool bf16, hipStream_t s);
hipError_t launch_labels(const Geom& g, int nl, bool two, const float* u, int32_t* lab,
                         hipStream_t s, int pitch = 0);
hipError_t launch_pitch_copy(const void* src, bool src_bf16, long long src_plane, int src_pitch, void* dst,
                             bool dst_bf16, long long dst_plane, int dst_pitch, int W, long long rows, int nplanes,
                             hipStream_t s);
hipError_t launch_read_planes(const void* src, bool bf16, float* dst, long long n, int nplanes,
                              long long plane, hipStream_t s);
hipError_t launch_write_planes(const float* src, void* dst, bool bf16, long long n, int nplanes,
                               long long plane, hipStream_t s);
hipError_t launch_convert_planes(const void* src, bool src_bf16, void* dst, bool dst_bf16, long long n, int nplanes,
                                 long long src_stride, long long dst_stride, hipStream_t s);
hipError_t launch_ctrl_reset(Ctrl* c, hipStream_t s);
hipError_t launch_bookkeep(Ctrl* c, long long k, double alpha, double tol, double neg_tol, long long nres,
                           int final_check, int decide, hipStream_t s);

// Largest negative relative gap that rounding of the stored flows explains.
// Weak duality P(u) >= D(q) holds whenever |q| <= alpha; after P_alpha in
// FP32 (reciprocal square root, a few ulp) |q| exceeds alpha by at most
// ~1e-6 relative, and BF16 storage rounds q (and a clamped alpha) by at most
// 2^-8 relative, so P - D >= -(excess) alpha TV(u) >= -(excess) max(|P|,|D|).
// A gap below minus this bound cannot come from rounding: the solve is
// reported as diverged.
__host__ __device__ inline double neg_gap_tol(bool bf16) { return bf16 ? 8e-3 : 1e-5; }

}  // namespace mf
