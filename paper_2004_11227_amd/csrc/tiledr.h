// Fused rPDRQ iteration for the two-label 2-D model: one 64 x TY tile per
// workgroup, state read once and written once (ping-pong buffers).
//
// With T+[a,b] the tile grown by a cells on its low and b on its high sides:
// the flows of the tile need the final u on T+[0,+1]; the final red cells
// there need the black cells on T+[-1,+2], which need the first red cells on
// T+[-2,+3], which need the old u on T+[-3,+4] and b on T+[-2,+3]; b needs
// q-bar on T+[-3,+3] and p-bar on T+[-2,+3].  The pass stages u, q-bar,
// p-bar_s, p-bar_t on T+[-3,+4] (columns widened to whole 4-element groups,
// -4 .. 67), forms b on T+[-2,+3], runs the red, black, red half-sweeps of
// the symmetric Gauss-Seidel step on the shrinking regions in LDS, then the
// flows, the relaxed reflection and the stores on the tile.  Each cell's
// arithmetic (b, the Gauss-Seidel value with its neighbours summed in the
// order -x, +x, -y, +y, the flows and the reflection) is that of the three
// in-place launches, so both variants give the same bits.
#pragma once
#include "mf_kernels.h"

namespace mf {

template <typename TS>
struct KDF {
  int W, H, pitch;
  long long P;
  int tiles_x;
  const TS* cap;
  const float* u_in;
  float* u_out;
  const TS* qb_in;
  TS* qb_out;
  const TS* psb_in;
  TS* psb_out;
  const TS* pb_in;
  TS* pb_out;
  TS* zq;
  TS* zs;
  TS* zp;
  float sigma, tau, rho, inv_st, alpha, m;
  int iso, keep_z;
  const int* done;
  CapGen cg;            // cg.img: `cap` is one image plane (read into ocs)
};

template <int TY>
struct SmemDR {
  static constexpr int SW = 72;       // cols -4 .. 67
  static constexpr int SH = TY + 7;   // rows -3 .. TY+3
  __align__(16) float su[SH][SW];
  __align__(16) float sqx[SH][SW];
  __align__(16) float sqy[SH][SW];
  __align__(16) float sps[SH][SW];
  __align__(16) float spt[SH][SW];
  __align__(16) float sb[SH][SW];
};

template <typename TS, int TY>
__device__ __forceinline__ void tile_dr2d(const KDF<TS>& A, int x0, int y0, SmemDR<TY>& S) {
  constexpr int TX = 64, V = 4, TPR = TX / V, RSTEP = 256 / TPR, RPT = TY / RSTEP;
  constexpr int OX = 4, OY = 3;
  constexpr int GPR = 18;
  constexpr int NG = (TY + 7) * GPR;
  constexpr int KG = (NG + 255) / 256;
  static_assert(RPT >= 1, "tile height must be a multiple of 16");
  auto& su = S.su;
  auto& sqx = S.sqx;
  auto& sqy = S.sqy;
  auto& sps = S.sps;
  auto& spt = S.spt;
  auto& sb = S.sb;
  const int tid = threadIdx.x;
  const int W = A.W, H = A.H, pitch = A.pitch;
  const long long P = A.P;

  // ---- stage u, q-bar, p-bar_s, p-bar_t on rows -3 .. TY+3, cols -4 .. 67
  float lu[KG][V], lqx[KG][V], lqy[KG][V], lps[KG][V], lpt[KG][V];
  int gnv[KG];
#pragma unroll
  for (int m = 0; m < KG; m++) {
    const int h = tid + 256 * m;
    const int r = h / GPR - OY, c = (h % GPR) * 4 - OX;
    const int gy = y0 + r, gx = x0 + c;
    const int nv = (h < NG && gy >= 0 && gy < H && gx >= 0) ? (W - gx >= V ? V : (W - gx > 0 ? W - gx : 0)) : 0;
    gnv[m] = nv;
    const long long i = nv > 0 ? (long long)gy * pitch + gx : 0;
    ldv<V>(A.u_in, i, lu[m]);
    ldv<V>(A.qb_in, i, lqx[m]);
    ldv<V>(A.qb_in + P, i, lqy[m]);
    ldv<V>(A.psb_in, i, lps[m]);
    ldv<V>(A.pb_in, i, lpt[m]);
  }
  const int c0 = (tid % TPR) * V;
  const int rr0 = tid / TPR;
  const int gx0 = x0 + c0;
  const int nvx = W - gx0 < 0 ? 0 : (W - gx0 > V ? V : W - gx0);
  int nvj[RPT];
  long long oj[RPT];
  float ocs[RPT][V], oct[RPT][V];
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    const int gy = y0 + rr0 + RSTEP * j;
    nvj[j] = gy < H ? nvx : 0;
    oj[j] = (long long)gy * pitch + gx0;
    ldv<V>(A.cap, nvj[j] > 0 ? oj[j] : 0, ocs[j]);
    if (!A.cg.img) ldv<V>(A.cap + P, nvj[j] > 0 ? oj[j] : 0, oct[j]);
  }
#pragma unroll
  for (int m = 0; m < KG; m++) {
    const int h = tid + 256 * m;
    if (h < NG) {
      const int r = h / GPR, c = (h % GPR) * 4;
#pragma unroll
      for (int e = 0; e < V; e++) {
        const bool ok = e < gnv[m];
        su[r][c + e] = ok ? lu[m][e] : 0.f;
        sqx[r][c + e] = ok ? lqx[m][e] : 0.f;
        sqy[r][c + e] = ok ? lqy[m][e] : 0.f;
        sps[r][c + e] = ok ? lps[m][e] : 0.f;
        spt[r][c + e] = ok ? lpt[m][e] : 0.f;
      }
    }
  }
  lds_barrier();
  // ---- b = -sigma (div q-bar + p-bar_t - p-bar_s) on T+[-2,+3]
  for (int h = tid; h < (TY + 5) * (TX + 5); h += 256) {
    const int r = h / (TX + 5) - 2, c = h % (TX + 5) - 2;
    const int hx = x0 + c, hy = y0 + r;
    const int R = r + OY, C = c + OX;
    const float d = ((hx + 1 < W ? sqx[R][C] : 0.f) - (hx > 0 ? sqx[R][C - 1] : 0.f)) +
                    ((hy + 1 < H ? sqy[R][C] : 0.f) - (hy > 0 ? sqy[R - 1][C] : 0.f));
    sb[R][C] = -A.sigma * ((d + spt[R][C]) - sps[R][C]);
  }
  lds_barrier();
  // Gauss-Seidel value of cell (r, c) from its neighbours in su
  auto gs = [&](int r, int c) {
    const int hx = x0 + c, hy = y0 + r;
    const int R = r + OY, C = c + OX;
    float s = 0.f, nb = 0.f;
    if (hx > 0) { s += su[R][C - 1]; nb += 1.f; }
    if (hx + 1 < W) { s += su[R][C + 1]; nb += 1.f; }
    if (hy > 0) { s += su[R - 1][C]; nb += 1.f; }
    if (hy + 1 < H) { s += su[R + 1][C]; nb += 1.f; }
    return (sb[R][C] * A.inv_st + s) / (nb + A.m);
  };
  // Half-sweep over the cells of one colour (0 red, 1 black: parity of
  // x + y; x0 and y0 are even) of rows rlo .. rlo+nr-1, cols clo .. clo+nc-1:
  // threads map onto that colour's cells only.
  auto half_sweep = [&](int rlo, int nr, int clo, int nc, int colour) {
    const int nch = (nc + 1) / 2;
    for (int h = tid; h < nr * nch; h += 256) {
      const int r = rlo + h / nch;
      const int c = clo + 2 * (h % nch) + ((colour - r - clo) & 1);
      if (c < clo + nc) su[r + OY][c + OX] = gs(r, c);
    }
  };
  // ---- red cells of T+[-2,+3], black cells of T+[-1,+2], red cells of T+[0,+1]
  half_sweep(-2, TY + 5, -2, TX + 5, 0);
  lds_barrier();
  half_sweep(-1, TY + 3, -1, TX + 3, 1);
  lds_barrier();
  half_sweep(0, TY + 1, 0, TX + 1, 0);
  lds_barrier();
  // ---- flows y = y-bar + tau K u and the relaxed reflection on the owned groups
  const float tau = A.tau, rho = A.rho;
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    const int r = rr0 + RSTEP * j;
    const int gy = y0 + r;
    float un[V], qxo[V], qyo[V], zqx[V], zqy[V], pto[V], zpt[V], pso[V], zps[V];
#pragma unroll
    for (int e = 0; e < V; e++) {
      const int gx = gx0 + e;
      const int R = r + OY, C = c0 + e + OX;
      const float u0 = su[R][C];
      un[e] = u0;
      float g0 = 0.f, g1 = 0.f;
      if (gx + 1 < W) g0 = su[R][C + 1] - u0;
      if (gy + 1 < H) g1 = su[R + 1][C] - u0;
      // q = q-bar - tau grad u;  z_q = P_alpha(2q - q-bar);  q-bar += rho (z_q - q)
      const float qb0 = sqx[R][C], qb1 = sqy[R][C];
      const float q0 = qb0 - tau * g0, q1 = qb1 - tau * g1;
      float z0 = 2.f * q0 - qb0, z1 = 2.f * q1 - qb1;
      if (A.iso) proj2<true>(z0, z1, A.alpha);
      else proj2<false>(z0, z1, A.alpha);
      qxo[e] = qb0 + rho * (z0 - q0);
      qyo[e] = qb1 + rho * (z1 - q1);
      zqx[e] = z0;
      zqy[e] = z1;
      // p_t = p-bar_t + tau u;  z = min(C_t, 2 p_t - p-bar_t);  p-bar_t += rho (z - p_t)
      const float pbv = spt[R][C];
      const float pv = pbv + tau * u0;
      const float Ct = A.cg.img ? cap_from(ocs[j][e], A.cg.lv[1], A.cg.pw) : oct[j][e];
      const float zpv = fminf(Ct, 2.f * pv - pbv);
      pto[e] = pbv + rho * (zpv - pv);
      zpt[e] = zpv;
      // p_s = p-bar_s - tau u;  z_s = min(C_s, 2 p_s - p-bar_s + tau)
      const float psbv = sps[R][C];
      const float psv = psbv - tau * u0;
      const float Cs = A.cg.img ? cap_from(ocs[j][e], A.cg.lv[0], A.cg.pw) : ocs[j][e];
      const float zsv = fminf(Cs, (2.f * psv - psbv) + tau);
      pso[e] = psbv + rho * (zsv - psv);
      zps[e] = zsv;
    }
    const int nv = nvj[j];
    const long long idx = oj[j];
    stg<V>(A.u_out, idx, nv, true, un);
    stg<V>(A.qb_out, idx, nv, true, qxo);
    stg<V>(A.qb_out + P, idx, nv, true, qyo);
    stg<V>(A.pb_out, idx, nv, true, pto);
    stg<V>(A.psb_out, idx, nv, true, pso);
    if (A.keep_z) {
      stg<V>(A.zq, idx, nv, true, zqx);
      stg<V>(A.zq + P, idx, nv, true, zqy);
      stg<V>(A.zp, idx, nv, true, zpt);
      stg<V>(A.zs, idx, nv, true, zps);
    }
  }
}

}  // namespace mf
