// Gap reduction, initial point, labels, field copies and the per-solve
// bookkeeping kernel.
#include "gap.h"

namespace mf {

hipError_t launch_fused2d(const SweepDesc& d, hipStream_t s);
hipError_t launch_fused3d(const SweepDesc& d, hipStream_t s);

hipError_t launch_fused(const SweepDesc& d, hipStream_t s) {
  return d.g.ndim == 2 ? launch_fused2d(d, s) : launch_fused3d(d, s);
}

// ------------------------------------------------------------------ gap

// Standalone FP64 gap of an iterate (grid-stride over pixels).
template <int NL, bool TWO, int NDIM, typename TS>
__global__ __launch_bounds__(256) void k_gap(const KG<TS> A) {
  __shared__ double sred[4 * 5];
  if (A.done && *A.done) return;
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const long long sz = (long long)A.W * A.H;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < A.n; idx += (long long)gridDim.x * 256) {
    const int x = (int)(idx % A.W);
    const int y = (int)((idx / A.W) % A.H);
    const int z = (int)(idx / sz);
    gap_px<NL, TWO, NDIM, TS>(A, ((long long)z * A.H + y) * A.pitch + x, x, y, z, g);
  }
  block_accumulate<5, 4>(g, A.acc, sred);
}

template <int NL, bool TWO, int NDIM, typename TS>
static hipError_t gap_nl(const GapDesc& d, hipStream_t s) {
  KG<TS> a;
  a.W = d.g.W;
  a.H = d.g.H;
  a.D = d.g.D;
  a.pitch = d.g.pitch;
  a.P = d.g.plane;
  a.n = d.g.npix();
  a.cap = (const TS*)d.cap;
  a.u = d.st.u;
  a.q = (const TS*)d.st.q;
  a.ps = (const TS*)d.st.ps;
  a.p = (const TS*)d.st.p;
  a.acc = d.acc;
  a.done = d.done;
  a.iso = d.iso ? 1 : 0;
  a.cg = d.cg;
  long long nb = (a.n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL((k_gap<NL, TWO, NDIM, TS>), dim3((int)nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int NDIM, typename TS>
static hipError_t gap_ts(const GapDesc& d, hipStream_t s) {
  if (d.two) return gap_nl<1, true, NDIM, TS>(d, s);
  switch (d.nl) {
    case 2: return gap_nl<2, false, NDIM, TS>(d, s);
    case 3: return gap_nl<3, false, NDIM, TS>(d, s);
    case 4: return gap_nl<4, false, NDIM, TS>(d, s);
    case 8: return gap_nl<8, false, NDIM, TS>(d, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gap(const GapDesc& d, hipStream_t s) {
  if (d.g.ndim == 2) return d.bf16 ? gap_ts<2, bf16_t>(d, s) : gap_ts<2, float>(d, s);
  return d.bf16 ? gap_ts<3, bf16_t>(d, s) : gap_ts<3, float>(d, s);
}

// ------------------------------------------------------------------ init
// q = 0, u = 0, p_s and every p_i (p_t) at the pointwise minimum capacity
// (0 in the padding of the rows, pitch > W).
template <typename TS>
__global__ __launch_bounds__(256) void k_init(int nl, int ncap, int ndim, long long n, long long P, int pitch,
                                              int W, const TS* cap, const CapGen cg, float* u, TS* q, TS* ps,
                                              TS* p) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    float m = cap_ld(cap, P, 0, i, cg);
#pragma unroll
    for (int c = 1; c < 8; c++)
      if (c < ncap) m = fminf(m, cap_ld(cap, P, c, i, cg));
    m = (int)(i % pitch) < W ? m : 0.f;
    st(ps, i, m);
    for (int l = 0; l < nl; l++) {
      u[(long long)l * P + i] = 0.f;
      st(p + (long long)l * P, i, m);
      for (int k = 0; k < ndim; k++) st(q + (long long)(l * ndim + k) * P, i, 0.f);
    }
  }
}

static int blocks_for(long long n) {
  long long nb = (n + 255) / 256;
  return (int)(nb > 8192 ? 8192 : (nb < 1 ? 1 : nb));
}

hipError_t launch_init(const Geom& g, int nl, bool two, bool bf16, const void* cap, const CapGen& cg,
                       StateView st, hipStream_t s) {
  const int ncap = two ? 2 : nl;
  if (ncap > 8) return hipErrorInvalidValue;
  const long long n = g.nstore();   // pads included
  if (bf16)
    hipLaunchKernelGGL(k_init<bf16_t>, dim3(blocks_for(n)), dim3(256), 0, s, nl, ncap, g.ndim, n, g.plane, g.pitch,
                       g.W, (const bf16_t*)cap, cg, st.u, (bf16_t*)st.q, (bf16_t*)st.ps, (bf16_t*)st.p);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(blocks_for(n)), dim3(256), 0, s, nl, ncap, g.ndim, n, g.plane, g.pitch,
                       g.W, (const float*)cap, cg, st.u, (float*)st.q, (float*)st.ps, (float*)st.p);
  return hipGetLastError();
}

// The first rpADMM iteration of the two-label model from the initial point
// as k_init stores it (u = 0, q = 0, p_s = p_t): v = (p_t - p_s) - u/c and
// div q are both +0, so w = 0 and q^1 = P_alpha(0 + 0) = +0 exactly, and the
// iteration is pointwise.  It runs the sweeps' device functions on those
// values (div q^1 = +0, u = +0, p_t and p_s as k_init stores them), so
// iterate 1 has the sweeps' bits, and adds the FP64 gap terms of iterate 0 (u = 0: data C_s,
// TV 0, dual min(C_s, C_t), residual (p_t - p_s)^2, flow p_s) to the gap
// accumulators as the gap-carrying sweep does.  Pad columns are neither
// written nor counted.
template <typename TS>
__global__ __launch_bounds__(256) void k_first_two(long long n, long long P, int pitch, int W, int ndim,
                                                   const TS* cap, Coef k, float* u_out, TS* q_out, TS* ps_out,
                                                   TS* p_out, double* acc) {
  __shared__ double sred[4 * 5];
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    if ((int)(i % pitch) >= W) continue;
    const float cs = ld(cap, i), ct = ld(cap + P, i);
    // p_t^0 = p_s^0 = min(C_s, C_t) in the storage type, as k_init stores
    // them (iterate 0 itself need not be in memory)
    const float m = fminf(cs, ct);
    const float ps = sizeof(TS) == 2 ? __uint_as_float((uint32_t)__builtin_bit_cast(uint16_t, f2bf(m)) << 16) : m;
    const float pt = ps;
    float pn, t, sd = 0.f, sr = 0.f;
    label_update(k, 0.f, pt, ps, 0.f, ct, pn, t, sd, sr);
    const float psn = finish_ps(k, ps, sd, sr, true, cs);
    u_out[i] = finish_u(k, t, psn);
    st(p_out, i, pn);
    st(ps_out, i, psn);
    for (int c = 0; c < ndim; c++) st(q_out + (long long)c * P, i, 0.f);
    g[0] += (double)cs;
    g[2] += fmin((double)cs, (double)ct);
    const double r = (double)pt - (double)ps;
    g[3] += r * r;
    g[4] += (double)ps;
  }
  block_accumulate<5, 4>(g, acc, sred);
}

hipError_t launch_first_two(const Geom& g, bool bf16, const void* cap, const StateView& out, const Coef& k,
                            double* acc, hipStream_t s) {
  const long long n = g.nstore();
  if (bf16)
    hipLaunchKernelGGL(k_first_two<bf16_t>, dim3(blocks_for(n)), dim3(256), 0, s, n, g.plane, g.pitch, g.W, g.ndim,
                       (const bf16_t*)cap, k, out.u, (bf16_t*)out.q, (bf16_t*)out.ps, (bf16_t*)out.p, acc);
  else
    hipLaunchKernelGGL(k_first_two<float>, dim3(blocks_for(n)), dim3(256), 0, s, n, g.plane, g.pitch, g.W, g.ndim,
                       (const float*)cap, k, out.u, (float*)out.q, (float*)out.ps, (float*)out.p, acc);
  return hipGetLastError();
}

// ------------------------------------------------------------------ copies
template <typename TS>
__global__ __launch_bounds__(256) void k_to_storage(const float* src, TS* dst, long long n, int np,
                                                    long long psrc, long long pdst) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    for (int c = 0; c < np; c++) st(dst + (long long)c * pdst, i, src[(long long)c * psrc + i]);
}
template <typename TS>
__global__ __launch_bounds__(256) void k_from_storage(const TS* src, float* dst, long long n, int np,
                                                      long long psrc, long long pdst) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    for (int c = 0; c < np; c++) dst[(long long)c * pdst + i] = ld(src + (long long)c * psrc, i);
}

hipError_t launch_convert_caps(const float* src, void* dst, long long n, int np, long long plane,
                               bool bf16, hipStream_t s) {
  if (bf16)
    hipLaunchKernelGGL(k_to_storage<bf16_t>, dim3(blocks_for(n)), dim3(256), 0, s, src, (bf16_t*)dst, n, np, n,
                       plane);
  else
    hipLaunchKernelGGL(k_to_storage<float>, dim3(blocks_for(n)), dim3(256), 0, s, src, (float*)dst, n, np, n,
                       plane);
  return hipGetLastError();
}
hipError_t launch_write_planes(const float* src, void* dst, bool bf16, long long n, int np, long long plane,
                               hipStream_t s) {
  return launch_convert_caps(src, dst, n, np, plane, bf16, s);
}
hipError_t launch_read_planes(const void* src, bool bf16, float* dst, long long n, int np, long long plane,
                              hipStream_t s) {
  if (bf16)
    hipLaunchKernelGGL(k_from_storage<bf16_t>, dim3(blocks_for(n)), dim3(256), 0, s, (const bf16_t*)src, dst, n,
                       np, plane, n);
  else
    hipLaunchKernelGGL(k_from_storage<float>, dim3(blocks_for(n)), dim3(256), 0, s, (const float*)src, dst, n,
                       np, plane, n);
  return hipGetLastError();
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_convert(const TI* src, TO* dst, long long n, int np, long long ss,
                                                 long long ds) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    for (int c = 0; c < np; c++) st(dst + (long long)c * ds, i, ld(src + (long long)c * ss, i));
}

hipError_t launch_convert_planes(const void* src, bool sb, void* dst, bool db, long long n, int np, long long ss,
                                 long long ds, hipStream_t s) {
  const dim3 g(blocks_for(n)), b(256);
  if (sb && db) hipLaunchKernelGGL((k_convert<bf16_t, bf16_t>), g, b, 0, s, (const bf16_t*)src, (bf16_t*)dst, n, np, ss, ds);
  else if (sb) hipLaunchKernelGGL((k_convert<bf16_t, float>), g, b, 0, s, (const bf16_t*)src, (float*)dst, n, np, ss, ds);
  else if (db) hipLaunchKernelGGL((k_convert<float, bf16_t>), g, b, 0, s, (const float*)src, (bf16_t*)dst, n, np, ss, ds);
  else hipLaunchKernelGGL((k_convert<float, float>), g, b, 0, s, (const float*)src, (float*)dst, n, np, ss, ds);
  return hipGetLastError();
}

// ------------------------------------------------------------------ labels
__global__ __launch_bounds__(256) void k_labels(int nl, int two, long long n, long long P, const float* u,
                                                int32_t* lab, int W, int pitch) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const long long j = (i / W) * pitch + i % W;   // storage index of dense pixel i
    if (two) {
      lab[i] = u[j] > 0.5f ? 1 : 0;
    } else {
      int best = 0;
      float bv = u[j];
      for (int l = 1; l < nl; l++) {
        const float v = u[(long long)l * P + j];
        if (v > bv) {
          bv = v;
          best = l;
        }
      }
      lab[i] = best;
    }
  }
}

hipError_t launch_labels(const Geom& g, int nl, bool two, const float* u, int32_t* lab, hipStream_t s, int pitch) {
  const long long n = g.npix();
  hipLaunchKernelGGL(k_labels, dim3(blocks_for(n)), dim3(256), 0, s, nl, two ? 1 : 0, n, g.plane, u, lab, g.W,
                     pitch > 0 ? pitch : g.W);
  return hipGetLastError();
}

// Copy `np` planes of `rows` x W elements between row strides (and storage
// types); destination pads (columns W .. dpitch-1) are set to 0.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_pitch_copy(const TI* src, long long sp, int spitch, TO* dst, long long dp,
                                                    int dpitch, int W, long long rows, int np) {
  const long long n = rows * dpitch;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const long long r = i / dpitch;
    const int x = (int)(i % dpitch);
    for (int c = 0; c < np; c++)
      st(dst + (long long)c * dp, i, x < W ? ld(src + (long long)c * sp, r * spitch + x) : 0.f);
  }
}

hipError_t launch_pitch_copy(const void* src, bool sb, long long sp, int spitch, void* dst, bool db, long long dp,
                             int dpitch, int W, long long rows, int np, hipStream_t s) {
  const dim3 g(blocks_for(rows * dpitch)), b(256);
  if (sb && db) hipLaunchKernelGGL((k_pitch_copy<bf16_t, bf16_t>), g, b, 0, s, (const bf16_t*)src, sp, spitch, (bf16_t*)dst, dp, dpitch, W, rows, np);
  else if (sb) hipLaunchKernelGGL((k_pitch_copy<bf16_t, float>), g, b, 0, s, (const bf16_t*)src, sp, spitch, (float*)dst, dp, dpitch, W, rows, np);
  else if (db) hipLaunchKernelGGL((k_pitch_copy<float, bf16_t>), g, b, 0, s, (const float*)src, sp, spitch, (bf16_t*)dst, dp, dpitch, W, rows, np);
  else hipLaunchKernelGGL((k_pitch_copy<float, float>), g, b, 0, s, (const float*)src, sp, spitch, (float*)dst, dp, dpitch, W, rows, np);
  return hipGetLastError();
}

// ------------------------------------------------------------------ control
__global__ void k_ctrl_reset(Ctrl* c) {
  const int t = threadIdx.x;
  for (int j = t; j < kAccSlots * 8; j += blockDim.x) c->acc[j / 8][j % 8] = 0.0;
  if (t < 8) c->last[t] = 0.0;
  if (t == 0) {
    c->iter = 0;
    c->done = 0;
    c->status = 0;
    c->checks = 0;
  }
}

hipError_t launch_ctrl_reset(Ctrl* c, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, c);
  return hipGetLastError();
}

// Turns the accumulated sums into the gap at iterate k, decides (when
// `decide`) whether the solve stops there, and clears the accumulators.
// Status codes follow mf_status: 0 converged, 1 cap reached, -4 diverged
// (a non-finite gap or residual, or a gap below -neg_tol).
// One wavefront, lane t reading and clearing accumulator slot t.
static_assert(kAccSlots == 64, "one lane per accumulator slot");
__global__ __launch_bounds__(64) void k_bookkeep(Ctrl* c, long long k, double alpha, double tol, double neg_tol,
                                                 long long nres, int final_check, int decide) {
  const int t = threadIdx.x;
  double tot[5];
#pragma unroll
  for (int j = 0; j < 5; j++) tot[j] = c->acc[t][j];   // issued together with the read of done
  if (c->done) return;
#pragma unroll
  for (int j = 0; j < 5; j++) tot[j] = wave_total(tot[j]);
#pragma unroll
  for (int j = 0; j < 8; j++) c->acc[t][j] = 0.0;
  if (t != 0) return;
  const double P = tot[0] + alpha * tot[1];
  const double D = tot[2];
  const double m = fmax(fmax(fabs(P), fabs(D)), 1e-300);
  const double rel = (P - D) / m;
  c->last[0] = P;
  c->last[1] = D;
  c->last[2] = rel;
  c->last[3] = sqrt(tot[3] / (double)nres);
  c->last[4] = tot[4];
  c->last[5] = (double)k;
  c->checks += 1;
  if (decide) {
    const bool bad = !isfinite(P) || !isfinite(D) || !isfinite(tot[3]) || rel < -neg_tol;
    if (bad) {
      c->done = 1;
      c->status = -4;
      c->iter = k;
    } else if (rel <= tol) {
      c->done = 1;
      c->status = 0;
      c->iter = k;
    } else if (final_check) {
      c->done = 1;
      c->status = 1;
      c->iter = k;
    }
  }
}

hipError_t launch_bookkeep(Ctrl* c, long long k, double alpha, double tol, double neg_tol, long long nres,
                           int final_check, int decide, hipStream_t s) {
  hipLaunchKernelGGL(k_bookkeep, dim3(1), dim3(64), 0, s, c, k, alpha, tol, neg_tol, nres, final_check, decide);
  return hipGetLastError();
}

}  // namespace mf
