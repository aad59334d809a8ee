// Unfused rpADMM baseline (2-D and 3-D): one kernel per operator,
//   K_w : w_i = div q_i^k + (p_i - p_s) - u_i/c          -> HBM (FP32 planes)
//   K_q : q_i' = P_alpha(q_i^k + grad(w_i)/a)             -> HBM
//   K_pu: d_i = div q_i', then the pointwise p, p_s, u updates
// The arithmetic is the same sequence of device functions as the fused
// passes, so both produce the same bits.
//
// The same element-wise machinery runs the paper's comparison methods:
//   pADMM-TY (eqs. ADMM:Tai_yuan, mADMM:Tai_yuan): K_w and K_q as above,
//     then block-sequential flow updates (K_ty);
//   ALG1 (Chambolle-Pock, eqs. iteration:pd:seg, alg1:4labels): K_cpd, the
//     dual step q' = P_alpha(q - sigma grad u-bar), p' = min(C, p + sigma
//     u-bar), p_s' = (min(C_s,) p_s - sigma sum u-bar + sigma); then K_cpp,
//     the primal step u' = u - tau (div q' + p' - p_s') and u-bar' = 2u' - u.
#include "mf_kernels.h"

namespace mf {

template <typename TS>
struct KU {
  int W, H, D;
  long long P, n;
  const TS* cap;
  const float* u_in;
  float* u_out;
  const TS* q_in;
  TS* q_out;
  const TS* ps_in;
  TS* ps_out;
  const TS* p_in;
  TS* p_out;
  float* wbuf;
  Coef k;
  const int* done;
  int iso;
  const float* ub_in;   // ALG1
  float* ub_out;
  float sigma, tau;
  CapGen cg;            // cg.img: `cap` is one image plane
};

template <int NDIM, typename TS>
__device__ __forceinline__ float div_at(const TS* q, long long P, long long idx, int x, int y, int z,
                                        int W, int H, int D) {
  const long long sz = (long long)W * H;
  if (NDIM == 2) {
    return div2(ld(q, idx), ldz(q, idx - 1, x > 0), ld(q + P, idx),
                ldz(q + P, idx - W, y > 0), x + 1 < W, x > 0, y + 1 < H, y > 0);
  }
  return div3(ld(q, idx), ldz(q, idx - 1, x > 0), ld(q + P, idx), ldz(q + P, idx - W, y > 0),
              ld(q + 2 * P, idx), ldz(q + 2 * P, idx - sz, z > 0), x + 1 < W, x > 0, y + 1 < H,
              y > 0, z + 1 < D, z > 0);
}

template <int NL, int NDIM, typename TS>
__global__ __launch_bounds__(256) void k_uf_w(const KU<TS> A) {
  if (A.done && *A.done) return;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < A.n; idx += (long long)gridDim.x * 256) {
    const int x = (int)(idx % A.W);
    const int y = (int)((idx / A.W) % A.H);
    const int z = (int)(idx / ((long long)A.W * A.H));
    const float ps = ld(A.ps_in, idx);
#pragma unroll
    for (int l = 0; l < NL; l++) {
      const float d = div_at<NDIM>(A.q_in + (long long)(NDIM * l) * A.P, A.P, idx, x, y, z, A.W, A.H, A.D);
      const float v = vterm(ld(A.p_in + (long long)l * A.P, idx), ps, A.u_in[(long long)l * A.P + idx],
                            A.k.inv_c);
      A.wbuf[(long long)l * A.P + idx] = wterm(d, v);
    }
  }
}

template <int NL, int NDIM, typename TS>
__global__ __launch_bounds__(256) void k_uf_q(const KU<TS> A) {
  if (A.done && *A.done) return;
  const long long sz = (long long)A.W * A.H;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < A.n; idx += (long long)gridDim.x * 256) {
    const int x = (int)(idx % A.W);
    const int y = (int)((idx / A.W) % A.H);
    const int z = (int)(idx / sz);
#pragma unroll
    for (int l = 0; l < NL; l++) {
      const float* w = A.wbuf + (long long)l * A.P;
      const float w0 = w[idx];
      const TS* qi = A.q_in + (long long)(NDIM * l) * A.P;
      TS* qo = A.q_out + (long long)(NDIM * l) * A.P;
      float qx = qstep(ld(qi, idx), ldz(w, idx + 1, x + 1 < A.W), w0, x + 1 < A.W, A.k.inv_a);
      float qy = qstep(ld(qi + A.P, idx), ldz(w, idx + A.W, y + 1 < A.H), w0, y + 1 < A.H, A.k.inv_a);
      if (NDIM == 2) {
        if (A.iso) proj2<true>(qx, qy, A.k.alpha);
        else proj2<false>(qx, qy, A.k.alpha);
      } else {
        float qz = qstep(ld(qi + 2 * A.P, idx), ldz(w, idx + sz, z + 1 < A.D), w0, z + 1 < A.D, A.k.inv_a);
        if (A.iso) proj3<true>(qx, qy, qz, A.k.alpha);
        else proj3<false>(qx, qy, qz, A.k.alpha);
        st(qo + 2 * A.P, idx, qz);
      }
      st(qo, idx, qx);
      st(qo + A.P, idx, qy);
    }
  }
}

template <int NL, bool TWO, int NDIM, typename TS>
__global__ __launch_bounds__(256) void k_uf_pu(const KU<TS> A) {
  if (A.done && *A.done) return;
  const Coef k = A.k;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < A.n; idx += (long long)gridDim.x * 256) {
    const int x = (int)(idx % A.W);
    const int y = (int)((idx / A.W) % A.H);
    const int z = (int)(idx / ((long long)A.W * A.H));
    const float ps = ld(A.ps_in, idx);
    float t[NL];
    float sumd = 0.f, sumr = 0.f;
#pragma unroll
    for (int l = 0; l < NL; l++) {
      const float d = div_at<NDIM>(A.q_out + (long long)(NDIM * l) * A.P, A.P, idx, x, y, z, A.W, A.H, A.D);
      const float C = cap_ld(A.cap, A.P, TWO ? 1 : l, idx, A.cg);
      float pn;
      label_update(k, A.u_in[(long long)l * A.P + idx], ld(A.p_in + (long long)l * A.P, idx), ps, d, C, pn,
                   t[l], sumd, sumr);
      st(A.p_out + (long long)l * A.P, idx, pn);
    }
    const float psn = finish_ps(k, ps, sumd, sumr, TWO, TWO ? cap_ld(A.cap, A.P, 0, idx, A.cg) : 0.f);
    st(A.ps_out, idx, psn);
#pragma unroll
    for (int l = 0; l < NL; l++) A.u_out[(long long)l * A.P + idx] = finish_u(k, t[l], psn);
  }
}

// pADMM-TY flows and multiplier from d_i = div q_i' (blocks in sequence).
// Two labels: p_s' with p_t^k, then p_t' with p_s'; n labels: p_i' with
// p_s^k, then p_s' with the new p_i', then u_i' = u_i - c (p_i' - p_s' + d_i).
template <int NL, bool TWO, int NDIM, typename TS>
__global__ __launch_bounds__(256) void k_ty(const KU<TS> A) {
  if (A.done && *A.done) return;
  const float c = A.k.c, inv_c = A.k.inv_c;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < A.n; idx += (long long)gridDim.x * 256) {
    const int x = (int)(idx % A.W);
    const int y = (int)((idx / A.W) % A.H);
    const int z = (int)(idx / ((long long)A.W * A.H));
    const float ps = ld(A.ps_in, idx);
    if (TWO) {
      const float d = div_at<NDIM>(A.q_out, A.P, idx, x, y, z, A.W, A.H, A.D);
      const float u = A.u_in[idx];
      const float psn = fminf(cap_ld(A.cap, A.P, 0, idx, A.cg), ((ld(A.p_in, idx) + d) - u * inv_c) + inv_c);
      const float ptn = fminf(cap_ld(A.cap, A.P, 1, idx, A.cg), (psn - d) + u * inv_c);
      st(A.ps_out, idx, psn);
      st(A.p_out, idx, ptn);
      A.u_out[idx] = u - c * ((ptn - psn) + d);
    } else {
      float d[NL], pn[NL];
      float s = 0.f;
#pragma unroll
      for (int l = 0; l < NL; l++) {
        d[l] = div_at<NDIM>(A.q_out + (long long)(NDIM * l) * A.P, A.P, idx, x, y, z, A.W, A.H, A.D);
        const float u = A.u_in[(long long)l * A.P + idx];
        pn[l] = fminf(cap_ld(A.cap, A.P, l, idx, A.cg), (ps - d[l]) + u * inv_c);
        s += (pn[l] + d[l]) - u * inv_c;
      }
      const float psn = s / (float)NL + inv_c / (float)NL;
      st(A.ps_out, idx, psn);
#pragma unroll
      for (int l = 0; l < NL; l++) {
        st(A.p_out + (long long)l * A.P, idx, pn[l]);
        const float u = A.u_in[(long long)l * A.P + idx];
        A.u_out[(long long)l * A.P + idx] = u - c * ((pn[l] - psn) + d[l]);
      }
    }
  }
}

// ALG1 dual step at every cell: q_i' from the forward differences of u-bar_i,
// then the flows.
template <int NL, bool TWO, int NDIM, typename TS>
__global__ __launch_bounds__(256) void k_cpd(const KU<TS> A) {
  if (A.done && *A.done) return;
  const long long sz = (long long)A.W * A.H;
  const float sg = A.sigma;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < A.n; idx += (long long)gridDim.x * 256) {
    const int x = (int)(idx % A.W);
    const int y = (int)((idx / A.W) % A.H);
    const int z = (int)(idx / sz);
    float sub = 0.f;
#pragma unroll
    for (int l = 0; l < NL; l++) {
      const float* ub = A.ub_in + (long long)l * A.P;
      const float b0 = ub[idx];
      const TS* qi = A.q_in + (long long)(NDIM * l) * A.P;
      TS* qo = A.q_out + (long long)(NDIM * l) * A.P;
      // neighbour loads guarded by their own conditions (ldz loads element 0 otherwise)
      const bool hx = x + 1 < A.W, hy = y + 1 < A.H;
      float qx = ld(qi, idx) - sg * (hx ? ldz(ub, idx + 1, hx) - b0 : 0.f);
      float qy = ld(qi + A.P, idx) - sg * (hy ? ldz(ub, idx + A.W, hy) - b0 : 0.f);
      if (NDIM == 2) {
        if (A.iso) proj2<true>(qx, qy, A.k.alpha);
        else proj2<false>(qx, qy, A.k.alpha);
      } else {
        const bool hz = z + 1 < A.D;
        float qz = ld(qi + 2 * A.P, idx) - sg * (hz ? ldz(ub, idx + sz, hz) - b0 : 0.f);
        if (A.iso) proj3<true>(qx, qy, qz, A.k.alpha);
        else proj3<false>(qx, qy, qz, A.k.alpha);
        st(qo + 2 * A.P, idx, qz);
      }
      st(qo, idx, qx);
      st(qo + A.P, idx, qy);
      const float C = cap_ld(A.cap, A.P, TWO ? 1 : l, idx, A.cg);
      st(A.p_out + (long long)l * A.P, idx, fminf(C, ld(A.p_in + (long long)l * A.P, idx) + sg * b0));
      sub += b0;
    }
    float psn = (ld(A.ps_in, idx) - sg * sub) + sg;
    if (TWO) psn = fminf(cap_ld(A.cap, A.P, 0, idx, A.cg), psn);
    st(A.ps_out, idx, psn);
  }
}

// ALG1 primal step and extrapolation (after K_cpd has finished everywhere).
template <int NL, bool TWO, int NDIM, typename TS>
__global__ __launch_bounds__(256) void k_cpp(const KU<TS> A) {
  if (A.done && *A.done) return;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < A.n; idx += (long long)gridDim.x * 256) {
    const int x = (int)(idx % A.W);
    const int y = (int)((idx / A.W) % A.H);
    const int z = (int)(idx / ((long long)A.W * A.H));
    const float psn = ld(A.ps_out, idx);
#pragma unroll
    for (int l = 0; l < NL; l++) {
      const float d = div_at<NDIM>(A.q_out + (long long)(NDIM * l) * A.P, A.P, idx, x, y, z, A.W, A.H, A.D);
      const float u = A.u_in[(long long)l * A.P + idx];
      const float un = u - A.tau * ((d + ld(A.p_out + (long long)l * A.P, idx)) - psn);
      A.u_out[(long long)l * A.P + idx] = un;
      A.ub_out[(long long)l * A.P + idx] = 2.f * un - u;
    }
  }
}

template <int NL, bool TWO, int NDIM, typename TS>
static hipError_t unfused_nl(const SweepDesc& d, hipStream_t s) {
  KU<TS> a;
  a.W = d.g.W;
  a.H = d.g.H;
  a.D = d.g.D;
  a.P = d.g.plane;
  a.n = d.g.npix();
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
  a.done = d.done;
  a.iso = d.iso ? 1 : 0;
  a.ub_in = d.in.ub;
  a.ub_out = d.out.ub;
  a.sigma = d.sigma;
  a.tau = d.tau;
  a.cg = d.cg;
  long long nb = (a.n + 255) / 256;
  if (nb > 16384) nb = 16384;
  if (d.scheme == 2) {
    if (!a.ub_in || !a.ub_out) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_cpd<NL, TWO, NDIM, TS>), dim3((int)nb), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_cpp<NL, TWO, NDIM, TS>), dim3((int)nb), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_uf_w<NL, NDIM, TS>), dim3((int)nb), dim3(256), 0, s, a);
  hipLaunchKernelGGL((k_uf_q<NL, NDIM, TS>), dim3((int)nb), dim3(256), 0, s, a);
  if (d.scheme == 1)
    hipLaunchKernelGGL((k_ty<NL, TWO, NDIM, TS>), dim3((int)nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_uf_pu<NL, TWO, NDIM, TS>), dim3((int)nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int NDIM, typename TS>
static hipError_t unfused_ts(const SweepDesc& d, hipStream_t s) {
  if (d.two) return unfused_nl<1, true, NDIM, TS>(d, s);
  switch (d.nl) {
    case 2: return unfused_nl<2, false, NDIM, TS>(d, s);
    case 3: return unfused_nl<3, false, NDIM, TS>(d, s);
    case 4: return unfused_nl<4, false, NDIM, TS>(d, s);
    case 8: return unfused_nl<8, false, NDIM, TS>(d, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_unfused(const SweepDesc& d, hipStream_t s) {
  if (d.g.pitch != d.g.W) return hipErrorInvalidValue;   // element-wise passes use the dense layout
  if (d.g.ndim == 2) return d.bf16 ? unfused_ts<2, bf16_t>(d, s) : unfused_ts<2, float>(d, s);
  return d.bf16 ? unfused_ts<3, bf16_t>(d, s) : unfused_ts<3, float>(d, s);
}

}  // namespace mf
