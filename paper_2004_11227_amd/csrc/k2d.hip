// 2-D rpADMM sweep: the fused LDS-tiled pass.
//
// One iteration of rpADMMI / rpADMMII (two-label and Potts) is, per label i,
//   w_i   = div q_i^k + (p_i^k - p_s^k) - u_i^k / c
//   q_i'  = P_alpha(q_i^k + grad(w_i) / a)
//   d_i   = div q_i'
// followed by the pointwise p, p_s and u updates (label_update/finish_*).
// q_i'(x) depends on q^k up to two cells behind x and one ahead, so a tile of
// 64 x TY outputs stages q^k on (TY+3) x 67 cells, w on (TY+2) x 66 and
// produces q' on (TY+1) x 65 cells in LDS.
#include "mf_kernels.h"

namespace mf {

template <typename TS>
__device__ __forceinline__ float quant(float v);
template <>
__device__ __forceinline__ float quant<float>(float v) { return v; }
template <>
__device__ __forceinline__ float quant<bf16_t>(float v) {
  return __uint_as_float(((uint32_t)f2bf(v)) << 16);
}

template <typename TS>
struct K2 {
  int W, H;
  long long P;        // plane stride
  int tiles_x;
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
  double* acc;
  const int* done;
  int write;
  int iso;
};

__device__ __forceinline__ void proj(float& x, float& y, float alpha, int iso) {
  if (iso) proj2<true>(x, y, alpha);
  else proj2<false>(x, y, alpha);
}

// FP64 gap terms of the two-label model at one pixel:
// data (1-u)C_s + u C_t and TV at u = clip(u,0,1), dual min(C_s, C_t + div q),
// residual p_t - p_s + div q, flow p_s.
__device__ __forceinline__ void gap_two_px(double (&g)[5], float u0f, float uxf, float uyf,
                                           bool hx, bool hy, double dq, float Cs, float Ct,
                                           float ps, float pt, int iso) {
  const double u0 = fmin(1.0, fmax(0.0, (double)u0f));
  const double gx = hx ? fmin(1.0, fmax(0.0, (double)uxf)) - u0 : 0.0;
  const double gy = hy ? fmin(1.0, fmax(0.0, (double)uyf)) - u0 : 0.0;
  g[0] += (1.0 - u0) * (double)Cs + u0 * (double)Ct;
  g[1] += iso ? sqrt(gx * gx + gy * gy) : fabs(gx) + fabs(gy);
  g[2] += fmin((double)Cs, (double)Ct + dq);
  const double r = ((double)pt - (double)ps) + dq;
  g[3] += r * r;
  g[4] += (double)ps;
}

template <int NL, bool TWO, typename TS, bool CHECK, int TY>
__global__ __launch_bounds__(256) void k_fused2d(const K2<TS> A) {
  constexpr int TX = 64, BY = 4, RY = TY / BY;
  constexpr int SW = TX + 4;   // cols -2 .. TX+1
  constexpr int SH = TY + 3;   // rows -2 .. TY
  __shared__ float sqx[SH][SW];
  __shared__ float sqy[SH][SW];
  __shared__ float sw[SH][SW];
  __shared__ float su[CHECK ? SH : 1][CHECK ? SW : 1];
  __shared__ double sred[4 * 5];

  if (A.done && *A.done) return;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % A.tiles_x) * TX;
  const int y0 = (tile / A.tiles_x) * TY;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
  const int W = A.W, H = A.H;
  const long long P = A.P;
  const int gx = x0 + tx;
  const bool colin = gx < W;
  const Coef k = A.k;

  float t[RY][NL];
  float ps[RY], sumd[RY], sumr[RY];
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < RY; j++) {
    const int gy = y0 + ty + BY * j;
    const bool in = colin && gy < H;
    ps[j] = in ? ld(A.ps_in, (long long)gy * W + gx) : 0.f;
    sumd[j] = 0.f;
    sumr[j] = 0.f;
  }

#pragma unroll
  for (int l = 0; l < NL; l++) {
    const TS* qx_in = A.q_in + (long long)(2 * l) * P;
    const TS* qy_in = qx_in + P;
    const float* u_in = A.u_in + (long long)l * P;
    const TS* p_in = A.p_in + (long long)l * P;
    float ul[RY], pl[RY];
    // ---- stage q^k and v = (p - p_s) - u/c: interior by the owning threads
#pragma unroll
    for (int j = 0; j < RY; j++) {
      const int r = ty + BY * j;
      const int gy = y0 + r;
      const bool in = colin && gy < H;
      const long long idx = (long long)gy * W + gx;
      sqx[r + 2][tx + 2] = in ? ld(qx_in, idx) : 0.f;
      sqy[r + 2][tx + 2] = in ? ld(qy_in, idx) : 0.f;
      ul[j] = in ? u_in[idx] : 0.f;
      pl[j] = in ? ld(p_in, idx) : 0.f;
      sw[r + 2][tx + 2] = vterm(pl[j], ps[j], ul[j], k.inv_c);
      if (CHECK) su[r + 2][tx + 2] = ul[j];
    }
    // q halo: rows {-2,-1,TY} x cols -2..TX, then cols {-2,-1,TX} x rows 0..TY-1
    for (int h = tid; h < 3 * (TX + 3) + 3 * TY; h += 256) {
      int r, c;
      if (h < 3 * (TX + 3)) {
        const int rr = h / (TX + 3);
        r = rr == 0 ? -2 : (rr == 1 ? -1 : TY);
        c = h % (TX + 3) - 2;
      } else {
        const int hh = h - 3 * (TX + 3);
        r = hh / 3;
        const int cc = hh % 3;
        c = cc == 0 ? -2 : (cc == 1 ? -1 : TX);
      }
      const int hx = x0 + c, hy = y0 + r;
      const bool in = hx >= 0 && hx < W && hy >= 0 && hy < H;
      const long long idx = (long long)hy * W + hx;
      sqx[r + 2][c + 2] = in ? ld(qx_in, idx) : 0.f;
      sqy[r + 2][c + 2] = in ? ld(qy_in, idx) : 0.f;
    }
    // v halo: rows {-1,TY} x cols -1..TX, then cols {-1,TX} x rows 0..TY-1
    for (int h = tid; h < 2 * (TX + 2) + 2 * TY; h += 256) {
      int r, c;
      if (h < 2 * (TX + 2)) {
        r = h < TX + 2 ? -1 : TY;
        c = h % (TX + 2) - 1;
      } else {
        const int hh = h - 2 * (TX + 2);
        r = hh >> 1;
        c = (hh & 1) ? TX : -1;
      }
      const int hx = x0 + c, hy = y0 + r;
      const bool in = hx >= 0 && hx < W && hy >= 0 && hy < H;
      const long long idx = (long long)hy * W + hx;
      const float uu = in ? u_in[idx] : 0.f;
      const float pp = in ? ld(p_in, idx) : 0.f;
      const float ss = in ? ld(A.ps_in, idx) : 0.f;
      sw[r + 2][c + 2] = vterm(pp, ss, uu, k.inv_c);
      if (CHECK) su[r + 2][c + 2] = uu;
    }
    __syncthreads();
    // ---- gap of the input iterate (two-label; q^k is still intact in LDS)
    if (CHECK) {
#pragma unroll
      for (int j = 0; j < RY; j++) {
        const int r = ty + BY * j;
        const int gy = y0 + r;
        if (colin && gy < H) {
          const long long idx = (long long)gy * W + gx;
          const double dq =
              (((gx + 1 < W) ? (double)sqx[r + 2][tx + 2] : 0.0) - ((gx > 0) ? (double)sqx[r + 2][tx + 1] : 0.0)) +
              (((gy + 1 < H) ? (double)sqy[r + 2][tx + 2] : 0.0) - ((gy > 0) ? (double)sqy[r + 1][tx + 2] : 0.0));
          gap_two_px(g, su[r + 2][tx + 2], su[r + 2][tx + 3], su[r + 3][tx + 2], gx + 1 < W,
                     gy + 1 < H, dq, ld(A.cap, idx), ld(A.cap + P, idx), ps[j], pl[j], A.iso);
        }
      }
    }
    // ---- w = div q^k + v on rows -1..TY, cols -1..TX
    for (int h = tid; h < (TY + 2) * (TX + 2); h += 256) {
      const int r = h / (TX + 2) - 1, c = h % (TX + 2) - 1;
      const int hx = x0 + c, hy = y0 + r;
      const float d = div2(sqx[r + 2][c + 2], sqx[r + 2][c + 1], sqy[r + 2][c + 2],
                           sqy[r + 1][c + 2], hx + 1 < W, hx > 0, hy + 1 < H, hy > 0);
      sw[r + 2][c + 2] = wterm(d, sw[r + 2][c + 2]);
    }
    __syncthreads();
    // ---- q^{k+1} = P_alpha(q^k + grad(w)/a) on rows -1..TY-1, cols -1..TX-1 (in place)
    for (int h = tid; h < (TY + 1) * (TX + 1); h += 256) {
      const int r = h / (TX + 1) - 1, c = h % (TX + 1) - 1;
      const int hx = x0 + c, hy = y0 + r;
      const float w0 = sw[r + 2][c + 2];
      float qx = qstep(sqx[r + 2][c + 2], sw[r + 2][c + 3], w0, hx + 1 < W, k.inv_a);
      float qy = qstep(sqy[r + 2][c + 2], sw[r + 3][c + 2], w0, hy + 1 < H, k.inv_a);
      proj(qx, qy, k.alpha, A.iso);
      sqx[r + 2][c + 2] = quant<TS>(qx);
      sqy[r + 2][c + 2] = quant<TS>(qy);
    }
    __syncthreads();
    // ---- interior: d = div q^{k+1}, store q^{k+1}, per-label p and u parts
    {
      TS* qx_out = A.q_out + (long long)(2 * l) * P;
      TS* qy_out = qx_out + P;
      TS* p_out = A.p_out + (long long)l * P;
      const TS* capl = A.cap + (long long)(TWO ? 1 : l) * P;
#pragma unroll
      for (int j = 0; j < RY; j++) {
        const int r = ty + BY * j;
        const int gy = y0 + r;
        const bool in = colin && gy < H;
        const long long idx = (long long)gy * W + gx;
        const float qx = sqx[r + 2][tx + 2], qy = sqy[r + 2][tx + 2];
        const float d = div2(qx, sqx[r + 2][tx + 1], qy, sqy[r + 1][tx + 2], gx + 1 < W, gx > 0,
                             gy + 1 < H, gy > 0);
        const float C = in ? ld(capl, idx) : 0.f;
        float pn;
        label_update(k, ul[j], pl[j], ps[j], d, C, pn, t[j][l], sumd[j], sumr[j]);
        if (A.write && in) {
          st(qx_out, idx, qx);
          st(qy_out, idx, qy);
          st(p_out, idx, pn);
        }
      }
    }
    if (NL > 1) __syncthreads();
  }
  // ---- p_s and u
#pragma unroll
  for (int j = 0; j < RY; j++) {
    const int gy = y0 + ty + BY * j;
    const bool in = colin && gy < H;
    const long long idx = (long long)gy * W + gx;
    const float Cs = (TWO && in) ? ld(A.cap, idx) : 0.f;
    const float psn = finish_ps(k, ps[j], sumd[j], sumr[j], TWO, Cs);
    if (A.write && in) {
      st(A.ps_out, idx, psn);
#pragma unroll
      for (int l = 0; l < NL; l++) A.u_out[(long long)l * P + idx] = finish_u(k, t[j][l], psn);
    }
  }
  if (CHECK) block_accumulate<5, 4>(g, A.acc, sred);
}

// ------------------------------------------------------------------ launchers
template <typename TS>
static K2<TS> make_k2(const SweepDesc& d) {
  K2<TS> a;
  a.W = d.g.W;
  a.H = d.g.H;
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
  a.acc = d.acc;
  a.done = d.done;
  a.write = d.write ? 1 : 0;
  a.iso = d.iso ? 1 : 0;
  return a;
}

template <int NL, bool TWO, typename TS, bool CHECK>
static hipError_t fused_ty(const SweepDesc& d, hipStream_t s) {
  const K2<TS> a = make_k2<TS>(d);
  const dim3 blk(64, 4);
  const int tr = d.tile_rows;
  if (tr == 8) {
    const int nb = a.tiles_x * ((d.g.H + 7) / 8);
    hipLaunchKernelGGL((k_fused2d<NL, TWO, TS, CHECK, 8>), dim3(nb), blk, 0, s, a);
  } else if (tr == 32 && NL <= 4) {
    const int nb = a.tiles_x * ((d.g.H + 31) / 32);
    hipLaunchKernelGGL((k_fused2d<NL, TWO, TS, CHECK, (NL <= 4 ? 32 : 8)>), dim3(nb), blk, 0, s, a);
  } else {
    const int nb = a.tiles_x * ((d.g.H + 15) / 16);
    hipLaunchKernelGGL((k_fused2d<NL, TWO, TS, CHECK, 16>), dim3(nb), blk, 0, s, a);
  }
  return hipGetLastError();
}

template <int NL, bool TWO, typename TS>
static hipError_t fused_nl(const SweepDesc& d, hipStream_t s) {
  if (d.check) {
    if constexpr (TWO) return fused_ty<NL, TWO, TS, true>(d, s);
    return hipErrorInvalidValue;   // Potts gaps use the standalone reduction
  }
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

}  // namespace mf
