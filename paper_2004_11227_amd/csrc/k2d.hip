// 2-D rpADMM sweep: the fused LDS-tiled pass (one tile per workgroup), and
// the depth-2 pass of the two-label model (two iterations per launch).  The
// CHECK variants also accumulate the FP64 gap of their input iterate
// (two-label and Potts).
#include "tile2d.h"
#include "tile2d_d2.h"

namespace mf {

template <int NL, bool TWO, typename TS, bool CHECK, int TY, bool IMG>
__global__ __launch_bounds__(256) void k_fused2d(const K2<TS> A) {
  __shared__ Smem2<TY, CHECK, CHECK && !TWO> S;
  if (A.done && *A.done) return;
  int tx, ty;
  strip_tile(xcd_tile(blockIdx.x, gridDim.x), A.tiles_x, (A.H + TY - 1) / TY, A.strip, tx, ty);
  const int x0 = tx * 64;
  const int y0 = ty * TY;
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (d1_interior<TY>(x0, y0, A.W, A.H)) tile2d<NL, TWO, TS, CHECK, TY, true, CHECK, IMG, false>(A, x0, y0, S, g);
  else tile2d<NL, TWO, TS, CHECK, TY, true, CHECK, IMG, true>(A, x0, y0, S, g);
  if (CHECK) block_accumulate<5, 4>(g, A.acc, S.sred);
}

template <typename TS, bool CHECK, int TY, bool IMG>
__global__ __launch_bounds__(256) void k_fused2d_d2(const K2<TS> A) {
  __shared__ Smem2d2<TY> S;
  if (A.done && *A.done) return;
  int tx, ty;
  strip_tile(xcd_tile(blockIdx.x, gridDim.x), A.tiles_x, (A.H + TY - 1) / TY, A.strip, tx, ty);
  const int x0 = tx * 64;
  const int y0 = ty * TY;
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (d2_interior<TY>(x0, y0, A.W, A.H)) tile2d_d2<TS, CHECK, TY, IMG, false>(A, x0, y0, S, g);
  else tile2d_d2<TS, CHECK, TY, IMG, true>(A, x0, y0, S, g);
  if (CHECK) block_accumulate<5, 4>(g, A.acc, S.sred);
}

// ------------------------------------------------------------------ launchers
template <typename TS>
static K2<TS> make_k2(const SweepDesc& d) {
  K2<TS> a;
  a.W = d.g.W;
  a.H = d.g.H;
  a.pitch = d.g.pitch;
  a.P = d.g.plane;
  a.tiles_x = (d.g.W + 63) / 64;
  a.cap = (const TS*)d.cap;
  a.u_in = d.in.u;
  a.u_out = d.out.u;
  a.q_in = (const TS*)d.in.q;
  a.q_out = (TS*)d.out.q;
  a.ps_in = (const TS*)d.in.ps;
  a.ps_out = (TS*)d.out.ps;
  a.p_in = (const TS*)d.in.p;
  a.p_out = (TS*)d.out.p;
  a.wbuf = d.wbuf;
  a.k = d.k;
  a.cg = d.cg;
  a.acc = d.acc;
  a.done = d.done;
  a.write = d.write ? 1 : 0;
  a.iso = d.iso ? 1 : 0;
  a.strip = d.stream ? kStripTiles : (1 << 30);
  a.nt = d.stream ? 1 : 0;
  return a;
}

// Rows are padded to a multiple of 4 elements, so every owned group is one
// vector access.
template <int NL, bool TWO, typename TS, bool CHECK, int TY>
static hipError_t fused_launch(const K2<TS>& a, int H, hipStream_t s) {
  const int nb = a.tiles_x * ((H + TY - 1) / TY);
  if (a.pitch % 4 != 0) return hipErrorInvalidValue;
  if (a.cg.img)
    hipLaunchKernelGGL((k_fused2d<NL, TWO, TS, CHECK, TY, true>), dim3(nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_fused2d<NL, TWO, TS, CHECK, TY, false>), dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int NL, bool TWO, typename TS, bool CHECK>
static hipError_t fused_ty(const SweepDesc& d, hipStream_t s) {
  const K2<TS> a = make_k2<TS>(d);
  const int tr = d.tile_rows;
  if (tr == 8) return fused_launch<NL, TWO, TS, CHECK, 8>(a, d.g.H, s);
  if (tr == 32 && NL <= 4) return fused_launch<NL, TWO, TS, CHECK, (NL <= 4 ? 32 : 16)>(a, d.g.H, s);
  return fused_launch<NL, TWO, TS, CHECK, 16>(a, d.g.H, s);
}

template <int NL, bool TWO, typename TS>
static hipError_t fused_nl(const SweepDesc& d, hipStream_t s) {
  if (d.check) return fused_ty<NL, TWO, TS, true>(d, s);
  return fused_ty<NL, TWO, TS, false>(d, s);
}

template <typename TS>
static hipError_t fused_ts(const SweepDesc& d, hipStream_t s) {
  if (d.two) return fused_nl<1, true, TS>(d, s);
  switch (d.nl) {
    case 2: return fused_nl<2, false, TS>(d, s);
    case 3: return fused_nl<3, false, TS>(d, s);
    case 4: return fused_nl<4, false, TS>(d, s);
    case 8: return fused_nl<8, false, TS>(d, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fused2d(const SweepDesc& d, hipStream_t s) {
  return d.bf16 ? fused_ts<bf16_t>(d, s) : fused_ts<float>(d, s);
}

template <typename TS, bool CHECK, bool IMG>
static hipError_t fused_d2_img(const K2<TS>& a, const SweepDesc& d, hipStream_t s) {
  if (d.tile_rows == 32) {
    const int nb = a.tiles_x * ((d.g.H + 31) / 32);
    hipLaunchKernelGGL((k_fused2d_d2<TS, CHECK, 32, IMG>), dim3(nb), dim3(256), 0, s, a);
  } else {
    const int nb = a.tiles_x * ((d.g.H + 15) / 16);
    hipLaunchKernelGGL((k_fused2d_d2<TS, CHECK, 16, IMG>), dim3(nb), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <typename TS, bool CHECK>
static hipError_t fused_d2_ts(const SweepDesc& d, hipStream_t s) {
  const K2<TS> a = make_k2<TS>(d);
  return d.cg.img ? fused_d2_img<TS, CHECK, true>(a, d, s) : fused_d2_img<TS, CHECK, false>(a, d, s);
}

// Two iterations (d.in = iterate k, d.out = iterate k+2) of the two-label 2-D
// model; rows padded to a multiple of 4; tile height 16 (8 is taken as 16) or 32.
hipError_t launch_fused2d_d2(const SweepDesc& d, hipStream_t s) {
  if (!d.two || d.g.ndim != 2 || d.g.pitch % 4 != 0 || !d.write) return hipErrorInvalidValue;
  if (d.bf16) return d.check ? fused_d2_ts<bf16_t, true>(d, s) : fused_d2_ts<bf16_t, false>(d, s);
  return d.check ? fused_d2_ts<float, true>(d, s) : fused_d2_ts<float, false>(d, s);
}

}  // namespace mf
