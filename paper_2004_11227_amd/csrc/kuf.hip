// Unfused rpADMM baseline (2-D and 3-D): one kernel per operator,
//   K_w : w_i = div q_i^k + (p_i - p_s) - u_i/c          -> HBM (FP32 planes)
//   K_q : q_i' = P_alpha(q_i^k + grad(w_i)/a)             -> HBM
//   K_pu: d_i = div q_i', then the pointwise p, p_s, u updates
// The arithmetic is the same sequence of device functions as the fused
// passes, so both produce the same bits.
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
      float qx = qstep(ld(qi, idx), x + 1 < A.W ? w[idx + 1] : 0.f, w0, x + 1 < A.W, A.k.inv_a);
      float qy = qstep(ld(qi + A.P, idx), y + 1 < A.H ? w[idx + A.W] : 0.f, w0, y + 1 < A.H, A.k.inv_a);
      if (NDIM == 2) {
        if (A.iso) proj2<true>(qx, qy, A.k.alpha);
        else proj2<false>(qx, qy, A.k.alpha);
      } else {
        float qz = qstep(ld(qi + 2 * A.P, idx), z + 1 < A.D ? w[idx + sz] : 0.f, w0, z + 1 < A.D, A.k.inv_a);
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
      const float C = ld(A.cap + (long long)(TWO ? 1 : l) * A.P, idx);
      float pn;
      label_update(k, A.u_in[(long long)l * A.P + idx], ld(A.p_in + (long long)l * A.P, idx), ps, d, C, pn,
                   t[l], sumd, sumr);
      st(A.p_out + (long long)l * A.P, idx, pn);
    }
    const float psn = finish_ps(k, ps, sumd, sumr, TWO, TWO ? ld(A.cap, idx) : 0.f);
    st(A.ps_out, idx, psn);
#pragma unroll
    for (int l = 0; l < NL; l++) A.u_out[(long long)l * A.P + idx] = finish_u(k, t[l], psn);
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
  long long nb = (a.n + 255) / 256;
  if (nb > 16384) nb = 16384;
  hipLaunchKernelGGL((k_uf_w<NL, NDIM, TS>), dim3((int)nb), dim3(256), 0, s, a);
  hipLaunchKernelGGL((k_uf_q<NL, NDIM, TS>), dim3((int)nb), dim3(256), 0, s, a);
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
