// 3-D fused rpADMM sweep (two-label model): one xy tile and z-slab per workgroup.
#include "tile3d.h"

namespace mf {

template <typename TS, bool CHECK, bool VEC>
__global__ __launch_bounds__(256) void k_fused3d(const K3<TS> A) {
  __shared__ Smem3<CHECK> S;
  if (A.done && *A.done) return;
  const int nxy = A.tiles_x * A.tiles_y;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int slab = tile / nxy;
  const int txy = tile % nxy;
  const int x0 = (txy % A.tiles_x) * 64;
  const int y0 = (txy / A.tiles_x) * 8;
  const int z0 = slab * A.tz;
  const int z1 = min(z0 + A.tz, A.D);
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  tile3d<TS, CHECK, VEC, CHECK>(A, x0, y0, z0, z1, S, g);
  if (CHECK) block_accumulate<5, 4>(g, A.acc, S.sred);
}

// Workgroups of k_fused3d resident at once on the current device.
template <typename TS, bool CHECK>
static long long resident_blocks3(bool vec) {
  static int cached[2] = {0, 0};
  int& c = cached[vec ? 1 : 0];
  if (c == 0) {
    int per_cu = 0, dev = 0, cus = 0;
    const void* f = vec ? (const void*)k_fused3d<TS, CHECK, true> : (const void*)k_fused3d<TS, CHECK, false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    c = per_cu * cus;
  }
  return c;
}

template <typename TS, bool CHECK>
static hipError_t fused3d_ts(const SweepDesc& d, hipStream_t s) {
  K3<TS> a;
  a.W = d.g.W;
  a.H = d.g.H;
  a.D = d.g.D;
  a.pitch = d.g.pitch;
  a.P = d.g.plane;
  a.SZ = (long long)d.g.pitch * d.g.H;
  a.tiles_x = (d.g.W + 63) / 64;
  a.tiles_y = (d.g.H + 7) / 8;
  // Slab depth: each slab re-reads 3 warm-up planes, so slabs should be
  // deep, but the grid must fill the chip.  Cut the volume into as many
  // slabs as make one full wave of resident workgroups (occupancy x CUs):
  // a partial second wave would run on a fraction of the chip.
  const long long nxy = (long long)a.tiles_x * a.tiles_y;
  const long long resident = resident_blocks3<TS, CHECK>(d.g.pitch % 2 == 0);
  long long nslab = resident / nxy;
  if (nslab < 1) nslab = 1;
  int tz = (int)((d.g.D + nslab - 1) / nslab);
  if (tz < 8) tz = d.g.D < 8 ? d.g.D : 8;
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
  a.acc = d.acc;
  a.done = d.done;
  a.write = d.write ? 1 : 0;
  a.iso = d.iso ? 1 : 0;
  const long long nb = nxy * ((d.g.D + tz - 1) / tz);
  if (d.g.pitch % 2 == 0)
    hipLaunchKernelGGL((k_fused3d<TS, CHECK, true>), dim3((unsigned)nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_fused3d<TS, CHECK, false>), dim3((unsigned)nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fused3d(const SweepDesc& d, hipStream_t s) {
  if (!d.two) return hipErrorNotSupported;   // Potts 3-D runs the unfused passes
  if (d.bf16) return d.check ? fused3d_ts<bf16_t, true>(d, s) : fused3d_ts<bf16_t, false>(d, s);
  return d.check ? fused3d_ts<float, true>(d, s) : fused3d_ts<float, false>(d, s);
}

}  // namespace mf
