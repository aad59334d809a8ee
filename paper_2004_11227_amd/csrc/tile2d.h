// Fused 2-D rpADMM tile: the body shared by the single-solve kernel and the
// persistent pool kernel.
//
// One iteration of rpADMMI / rpADMMII (two-label and Potts) is, per label i,
//   w_i   = div q_i^k + (p_i^k - p_s^k) - u_i^k / c
//   q_i'  = P_alpha(q_i^k + grad(w_i) / a)
//   d_i   = div q_i'
// followed by the pointwise p, p_s and u updates (label_update/finish_*).
// q_i'(x) depends on q^k up to two cells behind x and one ahead, so a tile of
// 64 x TY outputs stages q^k on (TY+3) x 67 cells, w on (TY+2) x 66 and
// produces q' on (TY+1) x 65 cells in LDS.
#pragma once
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
  int pitch;          // row stride in elements (>= W; multiple of 4 in padded layouts)
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
  CapGen cg;          // with IMG: `cap` is one image plane
  double* acc;
  const int* done;
  int write;
  int iso;
  int strip;          // 2-D tile order: tiles per column strip (see strip_tile)
  int nt;             // non-temporal stores of the new iterate
};

__device__ __forceinline__ void proj(float& x, float& y, float alpha, int iso) {
  if (iso) proj2<true>(x, y, alpha);
  else proj2<false>(x, y, alpha);
}

// proj with selects in place of the isotropic case's branch (the same
// operations on the same values), so a loop over several cells stays one
// basic block.
__device__ __forceinline__ void projs(float& x, float& y, float alpha, int iso) {
  if (iso) {
    const float n2 = x * x + y * y;
    const bool out = n2 > alpha * alpha;
    const float sc = alpha * rsq(n2);
    x = out ? x * sc : x;
    y = out ? y * sc : y;
  } else {
    proj2<false>(x, y, alpha);
  }
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

// Tile of 64 x TY outputs, 256 threads (1-D block).  Owner mapping: thread t
// owns V consecutive columns c0 = (t % (64/V)) * V of rows t / (64/V) + j *
// (4V), j < RPT, so every interior global access is one V-wide vector
// access per lane (16 B for FP32 and V = 4).  LDS column c of the tile is
// stored at index c + 4 so those groups stay 16-byte aligned.
// TH (Potts gap): the simplex threshold of the projected u at every cell of
// rows 0..TY, cols 0..64 (the owned cells and their +x / +y neighbours).
template <int TY, bool CHECK, bool TH = false>
struct Smem2 {
  static constexpr int SW = 64 + 8;   // cols -4 .. 67
  static constexpr int SH = TY + 3;   // rows -2 .. TY
  __align__(16) float sqx[SH][SW];
  __align__(16) float sqy[SH][SW];
  __align__(16) float sw[SH][SW];
  __align__(16) float su[CHECK ? SH : 1][CHECK ? SW : 1];
  double sth[TH ? TY + 1 : 1][TH ? 65 : 1];
  double sred[4 * 5];
};

// Loads of one label ahead of its use: the owned groups of q_x, q_y, u, p
// (and the label's capacities for Potts), and this thread's xy-halo entries.
// Raw values: entries outside the grid load element 0 of their plane and are
// zeroed when the label is staged, so the loads of label l+1 stay in flight
// across the LDS phases of label l.
template <int RPT, int V, int KQ, int KW>
struct Lab2 {
  float qx[RPT][V], qy[RPT][V], u[RPT][V], p[RPT][V], C[RPT][V];
  float hqx[KQ], hqy[KQ], hu[KW], hp[KW];
};

// A tile whose cells and halo cells (rows -1 .. TY, cols -1 .. 64) all have
// their four neighbours inside the grid.
template <int TY>
__device__ __forceinline__ bool d1_interior(int x0, int y0, int W, int H) {
  return x0 > 0 && y0 > 0 && x0 + 64 + 1 < W && y0 + TY + 1 < H;
}

// IMG: the capacities are computed from one image plane (A.cg), which is
// read once per pixel instead of 2 (two-label) or NL capacity planes.
// EDGE false: an interior tile (d1_interior), whose every boundary test is
// true and folds away; the arithmetic is unchanged.
template <int NL, bool TWO, typename TS, bool CHECK, int TY, bool VEC, bool SU, bool IMG = false, bool EDGE = true,
          bool TH = false>
__device__ __forceinline__ void tile2d(const K2<TS>& A, int x0, int y0, Smem2<TY, SU, TH>& S, double (&g)[5]) {
  static_assert(!CHECK || SU, "the gap needs the u staging array");
  static_assert(!CHECK || TWO || TH, "the Potts gap needs the simplex thresholds");
  constexpr int TX = 64;
  constexpr int V = TY >= 16 ? 4 : 2;
  constexpr int TPR = TX / V;        // threads per tile row
  constexpr int RSTEP = 256 / TPR;   // tile rows covered by one pass of the block
  constexpr int RPT = TY / RSTEP;    // rows per thread
  constexpr int OX = 4;              // LDS column offset
  constexpr int NHQ = 3 * (TX + 3) + 3 * TY;   // q halo: rows {-2,-1,TY} x cols -2..TX, cols {-2,-1,TX} x rows 0..TY-1
  constexpr int NHW = 2 * (TX + 2) + 2 * TY;   // v halo: rows {-1,TY} x cols -1..TX, cols {-1,TX} x rows 0..TY-1
  constexpr int KQ = (NHQ + 255) / 256, KW = (NHW + 255) / 256;
  // Potts with n = 8, and n = 3 on 16- and 32-row tiles, forms each
  // phase's cells in a batch (see the w and q phases below): n = 8 1024^2
  // FP32 67.3 -> 65.8 us, BF16 41.3 -> 39.3 us, n = 3 2% faster.  Elsewhere
  // the batch's registers cost a wave per SIMD (FP32 n = 4: 11% slower) or
  // gain nothing (two labels, n = 2).
  constexpr bool BATCH = !TWO && (NL == 8 || (NL == 3 && TY >= 16));
  auto& sqx = S.sqx;
  auto& sqy = S.sqy;
  auto& sw = S.sw;
  auto& su = S.su;
  const int tid = threadIdx.x;
  const int W = A.W, H = A.H, pitch = A.pitch;
  const long long P = A.P;
  const int c0 = (tid % TPR) * V;
  const int rr0 = tid / TPR;
  const int gx0 = x0 + c0;
  const int nvx = W - gx0 < 0 ? 0 : (W - gx0 > V ? V : W - gx0);
  constexpr bool vec = VEC;   // W % V == 0: interior groups are whole vectors
  const Coef k = A.k;
  // neighbour-inside-the-grid tests of the stencils (zero flux outside)
  auto xp = [&](int x) { return !EDGE || x + 1 < W; };
  auto xm = [&](int x) { return !EDGE || x > 0; };
  auto yp = [&](int y) { return !EDGE || y + 1 < H; };
  auto ym = [&](int y) { return !EDGE || y > 0; };

  // owned groups: valid element counts and storage offsets
  int nvj[RPT];
  long long oj[RPT];
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    const int gy = y0 + rr0 + RSTEP * j;
    nvj[j] = gy < H ? nvx : 0;
    oj[j] = (long long)gy * pitch + gx0;
  }
  // this thread's halo entries: tile coordinates, inside flags, offsets
  int hq_r[KQ], hq_c[KQ], hw_r[KW], hw_c[KW];
  bool hq_in[KQ], hw_in[KW];
  long long hq_o[KQ], hw_o[KW];
#pragma unroll
  for (int m = 0; m < KQ; m++) {
    const int h = tid + 256 * m;
    int r = 0, c = 0;
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
    hq_r[m] = r;
    hq_c[m] = c;
    hq_in[m] = h < NHQ && x0 + c >= 0 && x0 + c < W && y0 + r >= 0 && y0 + r < H;
    hq_o[m] = hq_in[m] ? (long long)(y0 + r) * pitch + (x0 + c) : 0;
  }
#pragma unroll
  for (int m = 0; m < KW; m++) {
    const int h = tid + 256 * m;
    int r = 0, c = 0;
    if (h < 2 * (TX + 2)) {
      r = h < TX + 2 ? -1 : TY;
      c = h % (TX + 2) - 1;
    } else {
      const int hh = h - 2 * (TX + 2);
      r = hh >> 1;
      c = (hh & 1) ? TX : -1;
    }
    hw_r[m] = r;
    hw_c[m] = c;
    hw_in[m] = h < NHW && x0 + c >= 0 && x0 + c < W && y0 + r >= 0 && y0 + r < H;
    hw_o[m] = hw_in[m] ? (long long)(y0 + r) * pitch + (x0 + c) : 0;
  }

  // raw group load (element 0 of the plane for groups outside the grid)
  auto ldr = [&](auto* p, int j, float (&o)[V]) {
    if (vec) {
      ldv<V>(p, nvj[j] > 0 ? oj[j] : 0, o);
    } else {
#pragma unroll
      for (int e = 0; e < V; e++) o[e] = ld(p, e < nvj[j] ? oj[j] + e : 0);
    }
  };
  auto zmask = [&](int j, float (&o)[V]) {
#pragma unroll
    for (int e = 0; e < V; e++) o[e] = e < nvj[j] ? o[e] : 0.f;
  };
  using LabT = Lab2<RPT, V, KQ, KW>;
  auto fetch = [&](int l, LabT& F) {
    const TS* qx_in = A.q_in + (long long)(2 * l) * P;
    const TS* qy_in = qx_in + P;
    const float* u_in = A.u_in + (long long)l * P;
    const TS* p_in = A.p_in + (long long)l * P;
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      ldr(qx_in, j, F.qx[j]);
      ldr(qy_in, j, F.qy[j]);
      ldr(u_in, j, F.u[j]);
      ldr(p_in, j, F.p[j]);
      if (!TWO && !IMG) ldr(A.cap + (long long)l * P, j, F.C[j]);
    }
#pragma unroll
    for (int m = 0; m < KQ; m++) {
      F.hqx[m] = ld(qx_in, hq_o[m]);
      F.hqy[m] = ld(qy_in, hq_o[m]);
    }
#pragma unroll
    for (int m = 0; m < KW; m++) {
      F.hu[m] = ld(u_in, hw_o[m]);
      F.hp[m] = ld(p_in, hw_o[m]);
    }
  };

  // label-independent loads: p_s (owned and halo), two-label capacities or
  // the image
  float t[RPT][NL][V];
  float ps[RPT][V], sumd[RPT][V], sumr[RPT][V];
  float capt[RPT][V], caps[RPT][V], im[RPT][V];
  float hps[KW];
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    ldr(A.ps_in, j, ps[j]);
    if (IMG) {
      ldr(A.cap, j, im[j]);
    } else if (TWO) {
      ldr(A.cap, j, caps[j]);
      ldr(A.cap + P, j, capt[j]);
    }
#pragma unroll
    for (int e = 0; e < V; e++) {
      sumd[j][e] = 0.f;
      sumr[j][e] = 0.f;
    }
  }
#pragma unroll
  for (int m = 0; m < KW; m++) hps[m] = ld(A.ps_in, hw_o[m]);
  // C_s (two-label) and the capacity of label l at owned element (j, e)
  auto cap_s = [&](int j, int e) { return IMG ? cap_from(im[j][e], A.cg.lv[0], A.cg.pw) : caps[j][e]; };
  auto cap_l = [&](int j, int e, int l, const LabT& F) {
    if (IMG) return cap_from(im[j][e], A.cg.lv[TWO ? 1 : l], A.cg.pw);
    return TWO ? capt[j][e] : F.C[j][e];
  };
  // Potts gap of the input iterate: the simplex threshold of u^k at the
  // owned cells and their +x / +y neighbours (FP64, as the standalone gap)
  double mn[RPT][V];
  if (CHECK && !TWO) {
#pragma unroll
    for (int j = 0; j < RPT; j++)
#pragma unroll
      for (int e = 0; e < V; e++) mn[j][e] = 1e300;
    for (int h = tid; h < (TY + 1) * (TX + 1); h += 256) {
      const int r = h / (TX + 1), c = h % (TX + 1);
      const int gx = x0 + c, gy = y0 + r;
      const bool in = gx < W && gy < H;
      const long long o = (long long)gy * pitch + gx;
      double v[NL];
#pragma unroll
      for (int l = 0; l < NL; l++) v[l] = (double)ldz(A.u_in + (long long)l * P, o, in);
      S.sth[r][c] = simplex_theta<NL>(v);
    }
  }
  LabT F;
  fetch(0, F);
#pragma unroll
  for (int j = 0; j < RPT; j++) zmask(j, ps[j]);
#pragma unroll
  for (int m = 0; m < KW; m++) hps[m] = hw_in[m] ? hps[m] : 0.f;

#pragma unroll
  for (int l = 0; l < NL; l++) {
    float ul[RPT][V], pl[RPT][V], Cl[RPT][V];
    // ---- stage q^k and v = (p - p_s) - u/c of label l from the registers
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      const int r = rr0 + RSTEP * j;
      zmask(j, F.qx[j]);
      zmask(j, F.qy[j]);
      zmask(j, F.u[j]);
      zmask(j, F.p[j]);
#pragma unroll
      for (int e = 0; e < V; e++) {
        ul[j][e] = F.u[j][e];
        pl[j][e] = F.p[j][e];
        Cl[j][e] = cap_l(j, e, l, F);
        sqx[r + 2][c0 + OX + e] = F.qx[j][e];
        sqy[r + 2][c0 + OX + e] = F.qy[j][e];
        sw[r + 2][c0 + OX + e] = vterm(pl[j][e], ps[j][e], ul[j][e], k.inv_c);
        if (CHECK) su[r + 2][c0 + OX + e] = ul[j][e];
      }
    }
#pragma unroll
    for (int m = 0; m < KQ; m++) {
      if (tid + 256 * m < NHQ) {
        sqx[hq_r[m] + 2][hq_c[m] + OX] = hq_in[m] ? F.hqx[m] : 0.f;
        sqy[hq_r[m] + 2][hq_c[m] + OX] = hq_in[m] ? F.hqy[m] : 0.f;
      }
    }
#pragma unroll
    for (int m = 0; m < KW; m++) {
      if (tid + 256 * m < NHW) {
        const float uu = hw_in[m] ? F.hu[m] : 0.f;
        const float pp = hw_in[m] ? F.hp[m] : 0.f;
        sw[hw_r[m] + 2][hw_c[m] + OX] = vterm(pp, hps[m], uu, k.inv_c);
        if (CHECK) su[hw_r[m] + 2][hw_c[m] + OX] = uu;
      }
    }
    // ---- issue the loads of label l+1
    if (l + 1 < NL) fetch(l + 1, F);
    lds_barrier();
    // ---- gap of the input iterate (q^k is still intact in LDS).  Potts:
    // label l's part of the primal (data and TV at the projected u), its
    // residual and its term of the dual minimum; the rest after the labels.
    if (CHECK) {
#pragma unroll
      for (int j = 0; j < RPT; j++) {
        const int r = rr0 + RSTEP * j;
        const int gy = y0 + r;
        const int nv = nvj[j];
#pragma unroll
        for (int e = 0; e < V; e++) {
          if (e < nv) {
            const int gx = gx0 + e, c = c0 + OX + e;
            const double dq =
                ((xp(gx) ? (double)sqx[r + 2][c] : 0.0) - (xm(gx) ? (double)sqx[r + 2][c - 1] : 0.0)) +
                ((yp(gy) ? (double)sqy[r + 2][c] : 0.0) - (ym(gy) ? (double)sqy[r + 1][c] : 0.0));
            if (TWO) {
              gap_two_px(g, su[r + 2][c], su[r + 2][c + 1], su[r + 3][c], xp(gx), yp(gy), dq,
                         cap_s(j, e), Cl[j][e], ps[j][e], pl[j][e], A.iso);
            } else {
              const int cc = c0 + e;
              const double w0 = simplex_part((double)su[r + 2][c], S.sth[r][cc]);
              const double wx = simplex_part((double)su[r + 2][c + 1], S.sth[r][cc + 1]);
              const double wy = simplex_part((double)su[r + 3][c], S.sth[r + 1][cc]);
              const double C = (double)Cl[j][e];
              g[0] += w0 * C;
              const double ddx = xp(gx) ? wx - w0 : 0.0;
              const double ddy = yp(gy) ? wy - w0 : 0.0;
              g[1] += A.iso ? sqrt(ddx * ddx + ddy * ddy) : fabs(ddx) + fabs(ddy);
              const double tt = C + dq;
              mn[j][e] = tt < mn[j][e] ? tt : mn[j][e];
              const double rr = (dq + (double)pl[j][e]) - (double)ps[j][e];
              g[3] += rr * rr;
            }
          }
        }
      }
    }
    if constexpr (BATCH) {
      // ---- w = div q^k + v on rows -1..TY, cols -1..TX; then q^{k+1} =
      // P_alpha(q^k + grad(w)/a) on rows -1..TY-1, cols -1..TX-1 in place.
      // Each thread takes cells tid + 256 k and forms all of them before
      // writing any (a cell reads no other cell's output of the same
      // phase), so their LDS reads are in flight together; the last,
      // partial round forms a copy of the last cell in its idle threads and
      // stores nothing.
      {
        constexpr int NC = (TY + 2) * (TX + 2), KC = (NC + 255) / 256;
        float wv[KC];
#pragma unroll
        for (int kk = 0; kk < KC; kk++) {
          int h = tid + 256 * kk;
          if (kk == KC - 1) h = h < NC ? h : NC - 1;
          const int r = h / (TX + 2) - 1, c = h % (TX + 2) - 1;
          const int hx = x0 + c, hy = y0 + r;
          const float d = div2(sqx[r + 2][c + OX], sqx[r + 2][c + OX - 1], sqy[r + 2][c + OX],
                               sqy[r + 1][c + OX], xp(hx), xm(hx), yp(hy), ym(hy));
          wv[kk] = wterm(d, sw[r + 2][c + OX]);
        }
#pragma unroll
        for (int kk = 0; kk < KC; kk++) {
          const int h = tid + 256 * kk;
          if (kk < KC - 1 || h < NC) sw[h / (TX + 2) + 1][h % (TX + 2) - 1 + OX] = wv[kk];
        }
      }
      lds_barrier();
      {
        constexpr int NC = (TY + 1) * (TX + 1), KC = (NC + 255) / 256;
        float qxv[KC], qyv[KC];
#pragma unroll
        for (int kk = 0; kk < KC; kk++) {
          int h = tid + 256 * kk;
          if (kk == KC - 1) h = h < NC ? h : NC - 1;
          const int r = h / (TX + 1) - 1, c = h % (TX + 1) - 1;
          const int hx = x0 + c, hy = y0 + r;
          const float w0 = sw[r + 2][c + OX];
          float qx = qstep(sqx[r + 2][c + OX], sw[r + 2][c + OX + 1], w0, xp(hx), k.inv_a);
          float qy = qstep(sqy[r + 2][c + OX], sw[r + 3][c + OX], w0, yp(hy), k.inv_a);
          projs(qx, qy, k.alpha, A.iso);
          qxv[kk] = quant<TS>(qx);
          qyv[kk] = quant<TS>(qy);
        }
#pragma unroll
        for (int kk = 0; kk < KC; kk++) {
          const int h = tid + 256 * kk;
          if (kk < KC - 1 || h < NC) {
            const int r = h / (TX + 1) - 1, c = h % (TX + 1) - 1;
            sqx[r + 2][c + OX] = qxv[kk];
            sqy[r + 2][c + OX] = qyv[kk];
          }
        }
      }
      lds_barrier();
    } else {
      // ---- w = div q^k + v on rows -1..TY, cols -1..TX
      for (int h = tid; h < (TY + 2) * (TX + 2); h += 256) {
        const int r = h / (TX + 2) - 1, c = h % (TX + 2) - 1;
        const int hx = x0 + c, hy = y0 + r;
        const float d = div2(sqx[r + 2][c + OX], sqx[r + 2][c + OX - 1], sqy[r + 2][c + OX],
                             sqy[r + 1][c + OX], xp(hx), xm(hx), yp(hy), ym(hy));
        sw[r + 2][c + OX] = wterm(d, sw[r + 2][c + OX]);
      }
      lds_barrier();
      // ---- q^{k+1} = P_alpha(q^k + grad(w)/a) on rows -1..TY-1, cols -1..TX-1 (in place)
      for (int h = tid; h < (TY + 1) * (TX + 1); h += 256) {
        const int r = h / (TX + 1) - 1, c = h % (TX + 1) - 1;
        const int hx = x0 + c, hy = y0 + r;
        const float w0 = sw[r + 2][c + OX];
        float qx = qstep(sqx[r + 2][c + OX], sw[r + 2][c + OX + 1], w0, xp(hx), k.inv_a);
        float qy = qstep(sqy[r + 2][c + OX], sw[r + 3][c + OX], w0, yp(hy), k.inv_a);
        proj(qx, qy, k.alpha, A.iso);
        sqx[r + 2][c + OX] = quant<TS>(qx);
        sqy[r + 2][c + OX] = quant<TS>(qy);
      }
      lds_barrier();
    }
    // ---- owned groups: d = div q^{k+1}, store q^{k+1}, per-label p and u parts
    {
      TS* qx_out = A.q_out + (long long)(2 * l) * P;
      TS* qy_out = qx_out + P;
      TS* p_out = A.p_out + (long long)l * P;
#pragma unroll
      for (int j = 0; j < RPT; j++) {
        const int r = rr0 + RSTEP * j;
        const int gy = y0 + r;
        const int nv = nvj[j];
        const long long idx = oj[j];
        float qxv[V], qyv[V], pn[V];
#pragma unroll
        for (int e = 0; e < V; e++) {
          const int gx = gx0 + e, c = c0 + OX + e;
          qxv[e] = sqx[r + 2][c];
          qyv[e] = sqy[r + 2][c];
          const float d = div2(qxv[e], sqx[r + 2][c - 1], qyv[e], sqy[r + 1][c], xp(gx), xm(gx),
                               yp(gy), ym(gy));
          label_update(k, ul[j][e], pl[j][e], ps[j][e], d, Cl[j][e], pn[e], t[j][l][e], sumd[j][e], sumr[j][e]);
        }
        if (A.write) {
          stg<V>(qx_out, idx, nv, vec, qxv, A.nt != 0);
          stg<V>(qy_out, idx, nv, vec, qyv, A.nt != 0);
          stg<V>(p_out, idx, nv, vec, pn, A.nt != 0);
        }
      }
    }
    if (NL > 1) lds_barrier();
  }
  if (CHECK && !TWO) {   // Potts gap: the dual minimum over the labels and the flow
#pragma unroll
    for (int j = 0; j < RPT; j++)
#pragma unroll
      for (int e = 0; e < V; e++)
        if (e < nvj[j]) {
          g[2] += mn[j][e];
          g[4] += (double)ps[j][e];
        }
  }
  // ---- p_s and u
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    const int nv = nvj[j];
    const long long idx = oj[j];
    float psn[V];
#pragma unroll
    for (int e = 0; e < V; e++) psn[e] = finish_ps(k, ps[j][e], sumd[j][e], sumr[j][e], TWO, TWO ? cap_s(j, e) : 0.f);
    if (A.write) {
      stg<V>(A.ps_out, idx, nv, vec, psn, A.nt != 0);
#pragma unroll
      for (int l = 0; l < NL; l++) {
        float un[V];
#pragma unroll
        for (int e = 0; e < V; e++) un[e] = finish_u(k, t[j][l][e], psn[e]);
        stg<V>(A.u_out + (long long)l * P, idx, nv, vec, un, A.nt != 0);
      }
    }
  }
}

}  // namespace mf
