// Per-pixel FP64 primal-dual gap terms, shared by the standalone gap
// reduction and the pool's per-tile gap kernel.
#pragma once
#include "mf_kernels.h"

namespace mf {

template <typename TS>
struct KG {
  int W, H, D;
  int pitch;          // row stride (>= W)
  long long P, n;
  const TS* cap;
  const float* u;
  const TS* q;
  const TS* ps;
  const TS* p;
  double* acc;
  const int* done;
  int iso;
  CapGen cg;          // cg.img: `cap` is one image plane
};

__device__ __forceinline__ double clip01(float v) { return fmin(1.0, fmax(0.0, (double)v)); }

// Adds to g the terms of pixel (x, y, z) at storage index idx: primal data and TV at the
// projected u (clip to [0,1] for two labels, pointwise simplex projection for
// Potts: relaxed min-cut eq. seg:chanvese / relaxed Potts eq. relaxed-potts),
// the dual term (min(C_s, C_t + div q) or min_i(C_i + div q_i): the max-flow
// objectives eqs. two-label-mf, potts-mf maximised over p for fixed q), the
// squared conservation residual and p_s.
template <int NL, bool TWO, int NDIM, typename TS>
__device__ __forceinline__ void gap_px(const KG<TS>& A, long long idx, int x, int y, int z, double (&g)[5]) {
  const long long sz = (long long)A.pitch * A.H;
  const long long sy = A.pitch;
  const bool hx = x + 1 < A.W, hy = y + 1 < A.H, hz = NDIM == 3 && z + 1 < A.D;
  const double ps = (double)ld(A.ps, idx);
  double dq[NL];
#pragma unroll
  for (int l = 0; l < NL; l++) {
    const TS* q = A.q + (long long)(NDIM * l) * A.P;
    double d = ((double)ldz(q, idx, hx) - (double)ldz(q, idx - 1, x > 0)) +
               ((double)ldz(q + A.P, idx, hy) - (double)ldz(q + A.P, idx - sy, y > 0));
    if (NDIM == 3)
      d += (double)ldz(q + 2 * A.P, idx, hz) - (double)ldz(q + 2 * A.P, idx - sz, z > 0);
    dq[l] = d;
  }
  if (TWO) {
    const double Cs = (double)cap_ld(A.cap, A.P, 0, idx, A.cg), Ct = (double)cap_ld(A.cap, A.P, 1, idx, A.cg);
    const double u0 = clip01(A.u[idx]);
    const double gx = hx ? clip01(ldz(A.u, idx + 1, hx)) - u0 : 0.0;
    const double gy = hy ? clip01(ldz(A.u, idx + sy, hy)) - u0 : 0.0;
    const double gz = hz ? clip01(ldz(A.u, idx + sz, hz)) - u0 : 0.0;
    g[0] += (1.0 - u0) * Cs + u0 * Ct;
    g[1] += A.iso ? sqrt((gx * gx + gy * gy) + gz * gz) : (fabs(gx) + fabs(gy)) + fabs(gz);
    g[2] += fmin(Cs, Ct + dq[0]);
    const double r = ((double)ld(A.p, idx) - ps) + dq[0];
    g[3] += r * r;
  } else {
    double v[NL], w0[NL], wx[NL], wy[NL], wz[NL];
#pragma unroll
    for (int l = 0; l < NL; l++) v[l] = (double)A.u[(long long)l * A.P + idx];
    simplex_proj<NL>(v, w0);
#pragma unroll
    for (int l = 0; l < NL; l++) v[l] = (double)ldz(A.u, (long long)l * A.P + idx + 1, hx);
    simplex_proj<NL>(v, wx);
#pragma unroll
    for (int l = 0; l < NL; l++) v[l] = (double)ldz(A.u, (long long)l * A.P + idx + sy, hy);
    simplex_proj<NL>(v, wy);
    if (NDIM == 3) {
#pragma unroll
      for (int l = 0; l < NL; l++) v[l] = (double)ldz(A.u, (long long)l * A.P + idx + sz, hz);
      simplex_proj<NL>(v, wz);
    }
    double mn = 1e300;
#pragma unroll
    for (int l = 0; l < NL; l++) {
      const double C = (double)cap_ld(A.cap, A.P, l, idx, A.cg);
      g[0] += w0[l] * C;
      const double gx = hx ? wx[l] - w0[l] : 0.0;
      const double gy = hy ? wy[l] - w0[l] : 0.0;
      const double gz = (NDIM == 3 && hz) ? wz[l] - w0[l] : 0.0;
      g[1] += A.iso ? sqrt((gx * gx + gy * gy) + gz * gz) : (fabs(gx) + fabs(gy)) + fabs(gz);
      const double t = C + dq[l];
      mn = t < mn ? t : mn;
      const double r = (dq[l] + (double)ld(A.p + (long long)l * A.P, idx)) - ps;
      g[3] += r * r;
    }
    g[2] += mn;
  }
  g[4] += ps;
}

}  // namespace mf
