// rPDRQ: relaxed, preconditioned Douglas-Rachford with one symmetric
// red-black Gauss-Seidel sweep as preconditioner (eq. iteration:quadratic:seg
// for two labels, eq. pdrq:4labels for n labels with T_0 of Lemma 1), or n
// sweeps (the preconditioner M_n: n preconditioned steps for T u = b).
//
// The u-step u^{k+1} = u^k + M^{-1}(b^k - st T u^k), M the symmetric GS
// matrix of st T = st(-Delta + m I) in red-black order, is one in-place
// red, black, red sweep of
//     u(x) <- (b(x)/st + sum_{y ~ x} u(y)) / (|N(x)| + m),
// m = 2 (two-label) or n + 1 (Potts, per label).  Each colour needs every
// update of the other colour, so an iteration is four launches:
//   R1 : b^k at every cell (-> b planes), red cells updated in place
//   B  : black cells updated in place
//   (n sweeps: then n - 1 more red, black pairs of half-sweep launches)
//   R  : red cells updated in place from the final black cells
//   F  : the flows y = y-bar + tau K u and the relaxed reflection
//        y-bar += rho (prox(2y - y-bar) - y) in place (each cell touches only
//        its own flows).
// 2-D solves (two-label and Potts, 1 to 4 sweeps) also have a fused tiled
// pass (tiledr.h) that runs the same per-cell arithmetic with the state read
// once and written once into the other ping-pong buffer.
#include "mf_kernels.h"
#include "tiledr.h"

namespace mf {

// Threads of a workgroup: 256 for 64 x 16 tiles, 512 for 64 x 32 (the
// larger tile amortises each barrier-separated phase over twice the cells
// and shrinks the halo from 1.41 to 1.25 times the tile).
template <int TY>
constexpr int dr_threads() { return TY == 32 ? 512 : 256; }

// Occupancy: a one-sweep tile of 64 x 16 (256 threads) or 64 x 32 (512)
// keeps its LDS within a quarter or a half of a CU's 160 KiB, so four or
// two workgroups can share a CU if the registers allow it; the kernel is
// latency bound (barrier-separated LDS phases), so those instantiations are
// held to 128 VGPRs (four waves per SIMD).
template <int TY, int NS, int NT>
constexpr int dr_waves_per_eu() { return (TY * 256 == 16 * NT && NS == 1) ? 4 : 1; }

template <typename TS, int TY, int NL, bool TWO, int NS, int NT = dr_threads<TY>()>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(dr_waves_per_eu<TY, NS, NT>())))
void k_dr_fused2d(const KDF<TS> A) {
  __shared__ SmemDR<TY, TWO, NS> S;
  if (A.done && *A.done) return;
  int tx, ty;
  strip_tile(xcd_tile(blockIdx.x, gridDim.x), A.tiles_x, (A.H + TY - 1) / TY, A.strip, tx, ty);
  const int x0 = tx * 64;
  const int y0 = ty * TY;
  if (dr_interior<TY, NS>(x0, y0, A.W, A.H)) tile_dr2d<TS, TY, NL, TWO, false, NS, NT>(A, x0, y0, S);
  else tile_dr2d<TS, TY, NL, TWO, true, NS, NT>(A, x0, y0, S);
}

template <typename TS, int NL, bool TWO>
static hipError_t dr_fused_nl(const PdrqDesc& d, hipStream_t s) {
  KDF<TS> a;
  a.W = d.g.W;
  a.H = d.g.H;
  a.pitch = d.g.pitch;
  a.P = d.g.plane;
  a.tiles_x = (d.g.W + 63) / 64;
  a.cap = (const TS*)d.cap;
  a.u_in = d.st.u;
  a.u_out = d.out.u;
  a.qb_in = (const TS*)d.st.q;
  a.qb_out = (TS*)d.out.q;
  a.psb_in = (const TS*)d.st.ps;
  a.psb_out = (TS*)d.out.ps;
  a.pb_in = (const TS*)d.st.p;
  a.pb_out = (TS*)d.out.p;
  a.zq = (TS*)d.z.q;
  a.zs = (TS*)d.z.ps;
  a.zp = (TS*)d.z.p;
  a.sigma = d.sigma;
  a.tau = d.tau;
  a.rho = d.rho;
  a.inv_st = d.inv_st;
  a.alpha = d.alpha;
  set_rden(a.rden, TWO ? 2.f : (float)(NL + 1));
  a.iso = d.iso ? 1 : 0;
  a.keep_z = d.keep_z ? 1 : 0;
  a.strip = d.stream ? kStripTiles : (1 << 30);
  a.nt = d.stream ? 1 : 0;
  a.done = d.done;
  a.cg = d.cg;
  // one sweep: 64 x 32 or 64 x 16 tiles; M_2 .. M_4: 64 x 16 tiles
  const dim3 g16(a.tiles_x * ((d.g.H + 15) / 16));
  switch (d.sweeps) {
    case 1:
      if (d.tile_rows == 32)
        hipLaunchKernelGGL((k_dr_fused2d<TS, 32, NL, TWO, 1>), dim3(a.tiles_x * ((d.g.H + 31) / 32)),
                           dim3(dr_threads<32>()), 0, s, a);
      else
        hipLaunchKernelGGL((k_dr_fused2d<TS, 16, NL, TWO, 1>), g16, dim3(256), 0, s, a);
      break;
    case 2: hipLaunchKernelGGL((k_dr_fused2d<TS, 16, NL, TWO, 2>), g16, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_dr_fused2d<TS, 16, NL, TWO, 3>), g16, dim3(256), 0, s, a); break;
    case 4:   // two labels only (resolve)
      if (!TWO) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_dr_fused2d<TS, 16, NL, TWO, TWO ? 4 : 1>), g16, dim3(256), 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TS>
static hipError_t dr_fused_ts(const PdrqDesc& d, hipStream_t s) {
  if (d.two) return dr_fused_nl<TS, 1, true>(d, s);
  switch (d.nl) {
    case 2: return dr_fused_nl<TS, 2, false>(d, s);
    case 3: return dr_fused_nl<TS, 3, false>(d, s);
    case 4: return dr_fused_nl<TS, 4, false>(d, s);
    case 8: return dr_fused_nl<TS, 8, false>(d, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename TS>
struct KD {
  int W, H, D;
  long long P, n;
  const TS* cap;
  float* u;
  TS* qb;
  TS* psb;
  TS* pb;
  TS* zq;
  TS* zs;
  TS* zp;
  float* b;
  float sigma, tau, rho, inv_st, alpha;
  Rden rden;            // 1 / (|N(x)| + m) for |N(x)| = 0 .. 6, rounded once on the host
  int iso, keep_z;
  const int* done;
  CapGen cg;            // cg.img: `cap` is one image plane
};

struct Cell {
  int x, y, z;
};

__device__ __forceinline__ bool is_red(const Cell& c) { return ((c.x + c.y + c.z) & 1) == 0; }

// Row-wise visit of the cells of the dense layout: each wavefront takes one
// row (y, z) at a time and the block's four wavefronts four rows, strided
// over the launch's y dimension; 64-cell chunks of a row go along x.  The
// row and its coordinates are uniform across the wavefront, so no cell
// needs an index division.
template <typename F>
__device__ __forceinline__ void for_rows(int H, int D, F&& f) {
  const long long nrows = (long long)H * D;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (long long row = (long long)blockIdx.y * 4 + wv; row < nrows; row += (long long)gridDim.y * 4)
    f(row, (int)(row % H), (int)(row / H));
}

// Gauss-Seidel value at one cell from its neighbours in `u` (one label).
// (b / (sigma tau) + sum of the neighbours) / (|N(x)| + m), the division as a
// product with the reciprocal of the denominator.
template <int NDIM>
__device__ __forceinline__ float gs_value(const float* u, const float* b, long long idx, const Cell& c, int W,
                                          int H, int D, float inv_st, const Rden rden) {
  const long long sz = (long long)W * H;
  float s = 0.f;
  int nb = 0;
  if (c.x > 0) { s += u[idx - 1]; nb++; }
  if (c.x + 1 < W) { s += u[idx + 1]; nb++; }
  if (c.y > 0) { s += u[idx - W]; nb++; }
  if (c.y + 1 < H) { s += u[idx + W]; nb++; }
  if (NDIM == 3) {
    if (c.z > 0) { s += u[idx - sz]; nb++; }
    if (c.z + 1 < D) { s += u[idx + sz]; nb++; }
  }
  return (b[idx] * inv_st + s) * rden_at(rden, nb);
}

// R1: b^k at every cell, then the red cells updated in place.
template <int NL, bool TWO, int NDIM, typename TS>
__global__ __launch_bounds__(256) void k_dr_r1(const KD<TS> A) {
  if (A.done && *A.done) return;
  const long long sz = (long long)A.W * A.H;
  const int lane = threadIdx.x & 63;
  for_rows(A.H, A.D, [&](long long row, int y, int z) {
    for (int x = blockIdx.x * 64 + lane; x < A.W; x += gridDim.x * 64) {
      const long long idx = row * A.W + x;
      const Cell c{x, y, z};
      const float psb = ld(A.psb, idx);
      float usum = 0.f;
      float uk[NL];
#pragma unroll
      for (int l = 0; l < NL; l++) {
        uk[l] = A.u[(long long)l * A.P + idx];
        usum += uk[l];
      }
#pragma unroll
      for (int l = 0; l < NL; l++) {
        const TS* q = A.qb + (long long)(NDIM * l) * A.P;
        float d = (ldz(q, idx, c.x + 1 < A.W) - ldz(q, idx - 1, c.x > 0)) +
                  (ldz(q + A.P, idx, c.y + 1 < A.H) - ldz(q + A.P, idx - A.W, c.y > 0));
        if (NDIM == 3)
          d += ldz(q + 2 * A.P, idx, c.z + 1 < A.D) - ldz(q + 2 * A.P, idx - sz, c.z > 0);
        float bl = -A.sigma * ((d + ld(A.pb + (long long)l * A.P, idx)) - psb);
        // Potts: + st ((n-1) u_i - sum_{j != i} u_j) = st (n u_i - sum_j u_j)
        if (!TWO) bl += (A.sigma * A.tau) * ((float)NL * uk[l] - usum);
        float* bp = A.b + (long long)l * A.P;
        bp[idx] = bl;
      }
      if (is_red(c)) {
#pragma unroll
        for (int l = 0; l < NL; l++) {
          float* ul = A.u + (long long)l * A.P;
          ul[idx] = gs_value<NDIM>(ul, A.b + (long long)l * A.P, idx, c, A.W, A.H, A.D, A.inv_st, A.rden);
        }
      }
    }
  });
}

// Half-sweep over the cells of one colour (RED: the red cells, else the
// black ones), in place; the lanes of a row take that colour's cells only
// (every other column).
template <int NL, int NDIM, typename TS, bool RED>
__global__ __launch_bounds__(256) void k_dr_half(const KD<TS> A) {
  if (A.done && *A.done) return;
  const int lane = threadIdx.x & 63;
  for_rows(A.H, A.D, [&](long long row, int y, int z) {
    const int par = (y + z + (RED ? 0 : 1)) & 1;   // column parity of this colour in the row
    for (int x = 2 * (blockIdx.x * 64 + lane) + par; x < A.W; x += 2 * gridDim.x * 64) {
      const long long idx = row * A.W + x;
      const Cell c{x, y, z};
#pragma unroll
      for (int l = 0; l < NL; l++) {
        float* ul = A.u + (long long)l * A.P;
        ul[idx] = gs_value<NDIM>(ul, A.b + (long long)l * A.P, idx, c, A.W, A.H, A.D, A.inv_st, A.rden);
      }
    }
  });
}

// F: the flows y = y-bar + tau K u^{k+1} from the final u, and the relaxed
// reflection y-bar += rho (prox(2y - y-bar) - y) in place (each cell
// touches only its own flows).
template <int NL, bool TWO, int NDIM, typename TS>
__global__ __launch_bounds__(256) void k_dr_flow(const KD<TS> A) {
  if (A.done && *A.done) return;
  const long long sz = (long long)A.W * A.H;
  const float tau = A.tau, rho = A.rho;
  const int lane = threadIdx.x & 63;
  for_rows(A.H, A.D, [&](long long row, int y, int z) {
    for (int x = blockIdx.x * 64 + lane; x < A.W; x += gridDim.x * 64) {
      const long long idx = row * A.W + x;
      float usum = 0.f;
#pragma unroll
      for (int l = 0; l < NL; l++) {
        const float* ul = A.u + (long long)l * A.P;
        const float u0 = ul[idx];
        usum += u0;
        // grad u^{k+1}: forward differences, zero across the boundary
        float g[3] = {0.f, 0.f, 0.f};
        if (x + 1 < A.W) g[0] = ul[idx + 1] - u0;
        if (y + 1 < A.H) g[1] = ul[idx + A.W] - u0;
        if (NDIM == 3 && z + 1 < A.D) g[2] = ul[idx + sz] - u0;
        // q = q-bar - tau grad u;  z_q = P_alpha(2q - q-bar);  q-bar += rho (z_q - q)
        TS* q = A.qb + (long long)(NDIM * l) * A.P;
        float qbv[3], qv[3], zv[3];
#pragma unroll
        for (int k = 0; k < NDIM; k++) {
          qbv[k] = ld(q + (long long)k * A.P, idx);
          qv[k] = qbv[k] - tau * g[k];
          zv[k] = 2.f * qv[k] - qbv[k];
        }
        if (NDIM == 2) {
          if (A.iso) proj2<true>(zv[0], zv[1], A.alpha);
          else proj2<false>(zv[0], zv[1], A.alpha);
        } else {
          if (A.iso) proj3<true>(zv[0], zv[1], zv[2], A.alpha);
          else proj3<false>(zv[0], zv[1], zv[2], A.alpha);
        }
#pragma unroll
        for (int k = 0; k < NDIM; k++) {
          st(q + (long long)k * A.P, idx, qbv[k] + rho * (zv[k] - qv[k]));
          if (A.keep_z) st(A.zq + (long long)(NDIM * l + k) * A.P, idx, zv[k]);
        }
        // p_i = p-bar_i + tau u_i;  z = min(C_i, 2 p_i - p-bar_i);  p-bar_i += rho (z - p_i)
        TS* pbl = A.pb + (long long)l * A.P;
        const float pbv = ld(pbl, idx);
        const float pv = pbv + tau * u0;
        const float zpv = fminf(cap_ld(A.cap, A.P, TWO ? 1 : l, idx, A.cg), 2.f * pv - pbv);
        st(pbl, idx, pbv + rho * (zpv - pv));
        if (A.keep_z) st(A.zp + (long long)l * A.P, idx, zpv);
      }
      // p_s = p-bar_s - tau sum_i u_i;  z_s = (min(C_s,) 2 p_s - p-bar_s + tau)
      const float psbv = ld(A.psb, idx);
      const float psv = psbv - tau * usum;
      float zsv = (2.f * psv - psbv) + tau;
      if (TWO) zsv = fminf(cap_ld(A.cap, A.P, 0, idx, A.cg), zsv);
      st(A.psb, idx, psbv + rho * (zsv - psv));
      if (A.keep_z) st(A.zs, idx, zsv);
    }
  });
}

template <int NL, bool TWO, int NDIM, typename TS>
static hipError_t dr_nl(const PdrqDesc& d, hipStream_t s) {
  KD<TS> a;
  a.W = d.g.W;
  a.H = d.g.H;
  a.D = d.g.D;
  a.P = d.g.plane;
  a.n = d.g.npix();
  a.cap = (const TS*)d.cap;
  a.u = d.st.u;
  a.qb = (TS*)d.st.q;
  a.psb = (TS*)d.st.ps;
  a.pb = (TS*)d.st.p;
  a.zq = (TS*)d.z.q;
  a.zs = (TS*)d.z.ps;
  a.zp = (TS*)d.z.p;
  a.b = d.b;
  a.sigma = d.sigma;
  a.tau = d.tau;
  a.rho = d.rho;
  a.inv_st = d.inv_st;
  a.alpha = d.alpha;
  set_rden(a.rden, TWO ? 2.f : (float)(NL + 1));
  a.iso = d.iso ? 1 : 0;
  a.keep_z = d.keep_z ? 1 : 0;
  a.done = d.done;
  a.cg = d.cg;
  // x: 64-cell chunks of a row (128 for the one-colour half-sweeps); y: four
  // rows per block, strided beyond 65535 blocks
  const long long rows4 = ((long long)d.g.H * d.g.D + 3) / 4;
  const int gy = (int)(rows4 < 65535 ? rows4 : 65535);
  const dim3 g_all((d.g.W + 63) / 64, gy), g_half(((d.g.W + 1) / 2 + 63) / 64, gy);
  // n symmetric sweeps = red, black, (red, black) x (n - 1), red: a red
  // half-sweep right after a red one would repeat it exactly
  hipLaunchKernelGGL((k_dr_r1<NL, TWO, NDIM, TS>), g_all, dim3(256), 0, s, a);
  hipLaunchKernelGGL((k_dr_half<NL, NDIM, TS, false>), g_half, dim3(256), 0, s, a);
  for (int sw = 1; sw < d.sweeps; sw++) {
    hipLaunchKernelGGL((k_dr_half<NL, NDIM, TS, true>), g_half, dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_dr_half<NL, NDIM, TS, false>), g_half, dim3(256), 0, s, a);
  }
  hipLaunchKernelGGL((k_dr_half<NL, NDIM, TS, true>), g_half, dim3(256), 0, s, a);
  hipLaunchKernelGGL((k_dr_flow<NL, TWO, NDIM, TS>), g_all, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int NDIM, typename TS>
static hipError_t dr_ts(const PdrqDesc& d, hipStream_t s) {
  if (d.two) return dr_nl<1, true, NDIM, TS>(d, s);
  switch (d.nl) {
    case 2: return dr_nl<2, false, NDIM, TS>(d, s);
    case 3: return dr_nl<3, false, NDIM, TS>(d, s);
    case 4: return dr_nl<4, false, NDIM, TS>(d, s);
    case 8: return dr_nl<8, false, NDIM, TS>(d, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pdrq_iter(const PdrqDesc& d, hipStream_t s) {
  if (d.sweeps < 1) return hipErrorInvalidValue;
  if (d.fused) {
    if (d.g.ndim != 2 || d.g.pitch % 4 != 0 || d.sweeps > 4) return hipErrorInvalidValue;
    return d.bf16 ? dr_fused_ts<bf16_t>(d, s) : dr_fused_ts<float>(d, s);
  }
  if (d.g.pitch != d.g.W) return hipErrorInvalidValue;   // element-wise sweeps use the dense layout
  if (d.g.ndim == 2) return d.bf16 ? dr_ts<2, bf16_t>(d, s) : dr_ts<2, float>(d, s);
  return d.bf16 ? dr_ts<3, bf16_t>(d, s) : dr_ts<3, float>(d, s);
}

}  // namespace mf
