// 3-D fused rpADMM sweep (two-label model): one xy tile and z-slab per workgroup.
#include "tile3d.h"

namespace mf {

// The gap-carrying 8-row sweep is held to 128 VGPRs (four workgroups per
// CU, as its LDS allows), which it meets without spills.
template <typename TS, bool CHECK, int TY, bool IMG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CHECK && TY == 8 ? 4 : 1)))
void k_fused3d(const K3<TS> A) {
  __shared__ Smem3<CHECK, TY> S;
  if (A.done && *A.done) return;
  const int nxy = A.tiles_x * A.tiles_y;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int slab = tile / nxy;
  const int txy = tile % nxy;
  const int x0 = (txy % A.tiles_x) * 64;
  const int y0 = (txy / A.tiles_x) * TY;
  const int z0 = slab * A.tz;
  const int z1 = min(z0 + A.tz, A.D);
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  tile3d<TS, CHECK, true, CHECK, TY, IMG>(A, x0, y0, z0, z1, S, g);
  if (CHECK) block_accumulate<5, 4>(g, A.acc, S.sred);
}

// Rows are padded to a multiple of 4 elements, so every owned group is one
// vector access.
template <typename TS, bool CHECK, int TY>
static hipError_t fused3d_ty(const SweepDesc& d, hipStream_t s) {
  if (d.g.pitch % 4 != 0) return hipErrorInvalidValue;
  K3<TS> a;
  a.W = d.g.W;
  a.H = d.g.H;
  a.D = d.g.D;
  a.pitch = d.g.pitch;
  a.P = d.g.plane;
  a.SZ = (long long)d.g.pitch * d.g.H;
  a.tiles_x = (d.g.W + 63) / 64;
  a.tiles_y = (d.g.H + TY - 1) / TY;
  // Slab depth: each slab re-reads 3 warm-up planes, but a launch needs
  // enough workgroups to keep every CU busy to the end: the deepest of 16
  // and 8 planes that still gives at least 2048 workgroups (8 per CU), else
  // 4.  Measured (FP32, µs per sweep, slabs of 4 / 8 / 16 planes): 256^3
  // 205.9 / 194.1 / 196.5; 128^3 31.6 / 33.8 / 52.9; 128 x 512^2 452.6 /
  // 406.5 / 390.3; 64 x 1024^2 924 / 836 / 797; 200 x 300 x 260 255.8 /
  // 264.6 / 279.7; the rule's choice is the fastest or within 3% of it, for
  // BF16 (8-row tiles) as well.  Depths that give a slab count off a
  // multiple of the 8 XCDs are slower (256^3: 12 planes 210.9, 20 planes
  // 231.3), as each XCD's run of workgroups then splits slabs.  slab_depth
  // overrides the rule.
  const long long nxy = (long long)a.tiles_x * a.tiles_y;
  int tz = d.slab_depth;
  if (tz <= 0) {
    tz = 4;
    for (int c = 16; c >= 8; c /= 2)
      if (nxy * ((d.g.D + c - 1) / c) >= 2048) {
        tz = c;
        break;
      }
  }
  if (tz > d.g.D) tz = d.g.D;
  a.tz = tz;
  a.cap = (const TS*)d.cap;
  a.u_in = d.in.u;
  a.u_out = d.out.u;
  a.q_in = (const TS*)d.in.q;
  a.q_out = (TS*)d.out.q;
  a.ps_in = (const TS*)d.in.ps;
  a.ps_out = (TS*)d.out.ps;
  a.p_in = (const TS*)d.in.p;
  a.p_out = (TS*)d.out.p;
  a.k = d.k;
  a.cg = d.cg;
  a.acc = d.acc;
  a.done = d.done;
  a.write = d.write ? 1 : 0;
  a.iso = d.iso ? 1 : 0;
  a.strip = 1 << 30;
  a.nt = d.stream ? 1 : 0;
  const long long nb = nxy * ((d.g.D + tz - 1) / tz);
  if (d.cg.img)
    hipLaunchKernelGGL((k_fused3d<TS, CHECK, TY, true>), dim3((unsigned)nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_fused3d<TS, CHECK, TY, false>), dim3((unsigned)nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

// xy tile height: 16 rows when tile_rows asks for 16 or more, else 8.
template <typename TS, bool CHECK>
static hipError_t fused3d_ts(const SweepDesc& d, hipStream_t s) {
  return d.tile_rows >= 16 ? fused3d_ty<TS, CHECK, 16>(d, s) : fused3d_ty<TS, CHECK, 8>(d, s);
}

hipError_t launch_fused3d(const SweepDesc& d, hipStream_t s) {
  if (!d.two) return hipErrorNotSupported;   // Potts 3-D runs the unfused passes
  if (d.bf16) return d.check ? fused3d_ts<bf16_t, true>(d, s) : fused3d_ts<bf16_t, false>(d, s);
  return d.check ? fused3d_ts<float, true>(d, s) : fused3d_ts<float, false>(d, s);
}

}  // namespace mf
