// Depth-2 fused 2-D rpADMM pass (two-label model): iterations k -> k+1 ->
// k+2 of one 64 x TY tile in one workgroup, with iterate k+1 kept in LDS.
//
// Write T+[a,b] for the tile grown by a cells on its low sides and b cells on
// its high sides.  Iterate k+2 on T needs iterate k+1 with q on T+[-2,+1] and
// u, p_t, p_s on T+[-1,+1]; that needs w^k on T+[-2,+2] and so iterate k on
// T+[-3,+2].  The pass
//   1. stages iterate k on T+[-3,+2] (one read of the state; the staged
//      rectangle is widened to whole 4-element groups, columns -4 .. 67),
//   2. iteration k+1: w on T+[-2,+2], q' on T+[-2,+1] in place, the
//      pointwise p_t, p_s, u updates on T+[-1,+1] in place,
//   3. iteration k+2: w' on T+[-1,+1], q'' on T+[-1,0] in place, the
//      divergence and pointwise updates on the tile, and one write of the
//      state,
// so HBM moves one state read and one state write per two iterations.
// Every in-grid cell runs the single-iteration operations (vterm, wterm,
// qstep, proj, div2, label_update, finish_*) in the same order as the
// depth-1 sweep, BF16 flows rounded after each iteration exactly as a store
// and reload would round them, so the iterates equal two depth-1 sweeps bit
// for bit.  Cells outside the grid are staged as zeros and never reach an
// in-grid result (the boundary flags select them out).
#pragma once
#include "tile2d.h"

namespace mf {

// A tile whose cells and halo cells (rows -2 .. TY+1, cols -2 .. 65 of the
// iterate k+1 work) all have their four neighbours inside the grid.
template <int TY>
__device__ __forceinline__ bool d2_interior(int x0, int y0, int W, int H) {
  return x0 > 0 && y0 > 0 && x0 + 64 + 2 < W && y0 + TY + 2 < H;
}

template <int TY>
struct Smem2d2 {
  static constexpr int SW = 72;       // cols -4 .. 67
  static constexpr int SH = TY + 5;   // rows -3 .. TY+1
  __align__(16) float sqx[SH][SW];
  __align__(16) float sqy[SH][SW];
  __align__(16) float su[SH][SW];
  __align__(16) float sps[SH][SW];
  __align__(16) float spt[SH][SW];
  __align__(16) float sw[SH][SW];
  double sred[4 * 5];
};

// IMG: capacities computed from one image plane (A.cg), read once per cell.
// EDGE false: an interior tile (d2_interior), whose every boundary test is
// true and folds away; the arithmetic is unchanged.
template <typename TS, bool CHECK, int TY, bool IMG = false, bool EDGE = true>
__device__ __forceinline__ void tile2d_d2(const K2<TS>& A, int x0, int y0, Smem2d2<TY>& S, double (&g)[5]) {
  constexpr int TX = 64, V = 4, TPR = TX / V, RSTEP = 256 / TPR, RPT = TY / RSTEP;
  constexpr int OX = 4, OY = 3;                    // LDS offsets of tile column / row 0
  constexpr int GPR = 18;                          // 4-element groups per staged row (cols -4 .. 67)
  constexpr int NG = (TY + 5) * GPR;               // staged groups (rows -3 .. TY+1)
  constexpr int KG = (NG + 255) / 256;
  constexpr int N1C = (TY + 2) * (TX + 2);         // cells of the k+1 pointwise update, T+[-1,+1]
  constexpr int KC = (N1C + 255) / 256;
  static_assert(RPT >= 1, "tile height must be a multiple of 16");
  auto& sqx = S.sqx;
  auto& sqy = S.sqy;
  auto& su = S.su;
  auto& sps = S.sps;
  auto& spt = S.spt;
  auto& sw = S.sw;
  const int tid = threadIdx.x;
  const int W = A.W, H = A.H, pitch = A.pitch;
  const long long P = A.P;
  const Coef k = A.k;
  const TS* qx_in = A.q_in;
  const TS* qy_in = A.q_in + P;
  // neighbour-inside-the-grid tests of the stencils (zero flux outside)
  auto xp = [&](int x) { return !EDGE || x + 1 < W; };
  auto xm = [&](int x) { return !EDGE || x > 0; };
  auto yp = [&](int y) { return !EDGE || y + 1 < H; };
  auto ym = [&](int y) { return !EDGE || y > 0; };

  // ---- 1. stage iterate k on rows -3 .. TY+1, cols -4 .. 67 (raw loads, then masks)
  float lqx[KG][V], lqy[KG][V], lu[KG][V], lps[KG][V], lpt[KG][V];
  int gnv[KG];
#pragma unroll
  for (int m = 0; m < KG; m++) {
    const int h = tid + 256 * m;
    const int r = h / GPR - OY, c = (h % GPR) * 4 - OX;
    const int gy = y0 + r, gx = x0 + c;
    const int nv = (h < NG && gy >= 0 && gy < H && gx >= 0) ? (W - gx >= V ? V : (W - gx > 0 ? W - gx : 0)) : 0;
    gnv[m] = nv;
    const long long i = nv > 0 ? (long long)gy * pitch + gx : 0;
    ldv<V>(qx_in, i, lqx[m]);
    ldv<V>(qy_in, i, lqy[m]);
    ldv<V>(A.u_in, i, lu[m]);
    ldv<V>(A.ps_in, i, lps[m]);
    ldv<V>(A.p_in, i, lpt[m]);
  }
  // capacities of the k+1 update cells (T+[-1,+1]) and of the owned groups
  // (with IMG the image values, turned into capacities where they are used)
  float c1s[KC], c1t[KC], c1i[KC];
  bool c1in[KC];
#pragma unroll
  for (int m = 0; m < KC; m++) {
    const int h = tid + 256 * m;
    const int r = h / (TX + 2) - 1, c = h % (TX + 2) - 1;
    const int gy = y0 + r, gx = x0 + c;
    const bool in = h < N1C && gx >= 0 && gx < W && gy >= 0 && gy < H;
    const long long i = in ? (long long)gy * pitch + gx : 0;
    c1in[m] = in;
    if (IMG) {
      c1i[m] = ld(A.cap, i);
    } else {
      c1s[m] = ld(A.cap, i);
      c1t[m] = ld(A.cap + P, i);
      c1s[m] = in ? c1s[m] : 0.f;
      c1t[m] = in ? c1t[m] : 0.f;
    }
  }
  const float lv0 = A.cg.lv[0], lv1 = A.cg.lv[1];
  const int pw = A.cg.pw;
  auto c1_s = [&](int m) { return IMG ? (c1in[m] ? cap_from(c1i[m], lv0, pw) : 0.f) : c1s[m]; };
  auto c1_t = [&](int m) { return IMG ? (c1in[m] ? cap_from(c1i[m], lv1, pw) : 0.f) : c1t[m]; };
  const int c0 = (tid % TPR) * V;
  const int rr0 = tid / TPR;
  const int gx0 = x0 + c0;
  const int nvx = W - gx0 < 0 ? 0 : (W - gx0 > V ? V : W - gx0);
  int nvj[RPT];
  long long oj[RPT];
  float ocs[RPT][V], oct[RPT][V], oim[RPT][V];
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    const int gy = y0 + rr0 + RSTEP * j;
    nvj[j] = gy < H ? nvx : 0;
    oj[j] = (long long)gy * pitch + gx0;
    if (IMG) {
      ldv<V>(A.cap, nvj[j] > 0 ? oj[j] : 0, oim[j]);
    } else {
      ldv<V>(A.cap, nvj[j] > 0 ? oj[j] : 0, ocs[j]);
      ldv<V>(A.cap + P, nvj[j] > 0 ? oj[j] : 0, oct[j]);
    }
  }
  auto o_s = [&](int j, int e) { return IMG ? cap_from(oim[j][e], lv0, pw) : ocs[j][e]; };
  auto o_t = [&](int j, int e) { return IMG ? cap_from(oim[j][e], lv1, pw) : oct[j][e]; };
#pragma unroll
  for (int m = 0; m < KG; m++) {
    const int h = tid + 256 * m;
    if (h < NG) {
      const int r = h / GPR, c = (h % GPR) * 4;   // LDS coordinates
#pragma unroll
      for (int e = 0; e < V; e++) {
        const bool ok = e < gnv[m];
        sqx[r][c + e] = ok ? lqx[m][e] : 0.f;
        sqy[r][c + e] = ok ? lqy[m][e] : 0.f;
        su[r][c + e] = ok ? lu[m][e] : 0.f;
        sps[r][c + e] = ok ? lps[m][e] : 0.f;
        spt[r][c + e] = ok ? lpt[m][e] : 0.f;
      }
    }
  }
  lds_barrier();
  // ---- gap of the input iterate k on the owned pixels
  if (CHECK) {
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      const int r = rr0 + RSTEP * j;
      const int gy = y0 + r;
#pragma unroll
      for (int e = 0; e < V; e++) {
        if (e < nvj[j]) {
          const int gx = gx0 + e, c = c0 + e;
          const int R = r + OY, C = c + OX;
          const double dq =
              ((xp(gx) ? (double)sqx[R][C] : 0.0) - (xm(gx) ? (double)sqx[R][C - 1] : 0.0)) +
              ((yp(gy) ? (double)sqy[R][C] : 0.0) - (ym(gy) ? (double)sqy[R - 1][C] : 0.0));
          gap_two_px(g, su[R][C], su[R][C + 1], su[R + 1][C], xp(gx), yp(gy), dq, o_s(j, e), o_t(j, e),
                     sps[R][C], spt[R][C], A.iso);
        }
      }
    }
  }
  // ---- 2a. w^k on T+[-2,+2]
  for (int h = tid; h < (TY + 4) * (TX + 4); h += 256) {
    const int r = h / (TX + 4) - 2, c = h % (TX + 4) - 2;
    const int hx = x0 + c, hy = y0 + r;
    const int R = r + OY, C = c + OX;
    const float d = div2(sqx[R][C], sqx[R][C - 1], sqy[R][C], sqy[R - 1][C], xp(hx), xm(hx), yp(hy), ym(hy));
    sw[R][C] = wterm(d, vterm(spt[R][C], sps[R][C], su[R][C], k.inv_c));
  }
  lds_barrier();
  // ---- 2b. q^{k+1} on T+[-2,+1], in place
  for (int h = tid; h < (TY + 3) * (TX + 3); h += 256) {
    const int r = h / (TX + 3) - 2, c = h % (TX + 3) - 2;
    const int hx = x0 + c, hy = y0 + r;
    const int R = r + OY, C = c + OX;
    const float w0 = sw[R][C];
    float qx = qstep(sqx[R][C], sw[R][C + 1], w0, xp(hx), k.inv_a);
    float qy = qstep(sqy[R][C], sw[R + 1][C], w0, yp(hy), k.inv_a);
    proj(qx, qy, k.alpha, A.iso);
    sqx[R][C] = quant<TS>(qx);
    sqy[R][C] = quant<TS>(qy);
  }
  lds_barrier();
  // ---- 2c. p_t, p_s, u of iterate k+1 on T+[-1,+1], in place
#pragma unroll
  for (int m = 0; m < KC; m++) {
    const int h = tid + 256 * m;
    if (h < N1C) {
      const int r = h / (TX + 2) - 1, c = h % (TX + 2) - 1;
      const int hx = x0 + c, hy = y0 + r;
      const int R = r + OY, C = c + OX;
      const float d = div2(sqx[R][C], sqx[R][C - 1], sqy[R][C], sqy[R - 1][C], xp(hx), xm(hx), yp(hy), ym(hy));
      float pn, t, sd = 0.f, sr = 0.f;
      const float ps = sps[R][C];
      label_update(k, su[R][C], spt[R][C], ps, d, c1_t(m), pn, t, sd, sr);
      const float psn = finish_ps(k, ps, sd, sr, true, c1_s(m));
      su[R][C] = finish_u(k, t, psn);
      spt[R][C] = quant<TS>(pn);
      sps[R][C] = quant<TS>(psn);
    }
  }
  lds_barrier();
  // ---- 3a. w^{k+1} on T+[-1,+1]
  for (int h = tid; h < (TY + 2) * (TX + 2); h += 256) {
    const int r = h / (TX + 2) - 1, c = h % (TX + 2) - 1;
    const int hx = x0 + c, hy = y0 + r;
    const int R = r + OY, C = c + OX;
    const float d = div2(sqx[R][C], sqx[R][C - 1], sqy[R][C], sqy[R - 1][C], xp(hx), xm(hx), yp(hy), ym(hy));
    sw[R][C] = wterm(d, vterm(spt[R][C], sps[R][C], su[R][C], k.inv_c));
  }
  lds_barrier();
  // ---- 3b. q^{k+2} on T+[-1,0], in place
  for (int h = tid; h < (TY + 1) * (TX + 1); h += 256) {
    const int r = h / (TX + 1) - 1, c = h % (TX + 1) - 1;
    const int hx = x0 + c, hy = y0 + r;
    const int R = r + OY, C = c + OX;
    const float w0 = sw[R][C];
    float qx = qstep(sqx[R][C], sw[R][C + 1], w0, xp(hx), k.inv_a);
    float qy = qstep(sqy[R][C], sw[R + 1][C], w0, yp(hy), k.inv_a);
    proj(qx, qy, k.alpha, A.iso);
    sqx[R][C] = quant<TS>(qx);
    sqy[R][C] = quant<TS>(qy);
  }
  lds_barrier();
  // ---- 3c. owned groups: divergence, updates, one write of iterate k+2
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    const int r = rr0 + RSTEP * j;
    const int gy = y0 + r;
    float qxv[V], qyv[V], pn[V], psn[V], un[V];
#pragma unroll
    for (int e = 0; e < V; e++) {
      const int gx = gx0 + e;
      const int R = r + OY, C = c0 + e + OX;
      qxv[e] = sqx[R][C];
      qyv[e] = sqy[R][C];
      const float d = div2(qxv[e], sqx[R][C - 1], qyv[e], sqy[R - 1][C], xp(gx), xm(gx), yp(gy), ym(gy));
      float t, sd = 0.f, sr = 0.f;
      const float ps = sps[R][C];
      label_update(k, su[R][C], spt[R][C], ps, d, o_t(j, e), pn[e], t, sd, sr);
      psn[e] = finish_ps(k, ps, sd, sr, true, o_s(j, e));
      un[e] = finish_u(k, t, psn[e]);
    }
    if (A.write) {
      const int nv = nvj[j];
      const long long idx = oj[j];
      stg<V>(A.q_out, idx, nv, true, qxv, A.nt != 0);
      stg<V>(A.q_out + P, idx, nv, true, qyv, A.nt != 0);
      stg<V>(A.p_out, idx, nv, true, pn, A.nt != 0);
      stg<V>(A.ps_out, idx, nv, true, psn, A.nt != 0);
      stg<V>(A.u_out, idx, nv, true, un, A.nt != 0);
    }
  }
}

}  // namespace mf
