// Fused rPDRQ iteration for the 2-D two-label and Potts models: one 64 x TY
// tile per workgroup, state read once and written once (ping-pong buffers).
//
// With T+[a,b] the tile grown by a cells on its low and b on its high sides:
// the flows of the tile need the final u on T+[0,+1]; the final red cells
// there need the black cells on T+[-1,+2], which need the first red cells on
// T+[-2,+3], which need the old u on T+[-3,+4] and b on T+[-2,+3]; b needs
// q-bar on T+[-3,+3] and p-bar on T+[-2,+3].  Per label the pass stages u,
// q-bar and p-bar of the label on T+[-3,+4] (columns widened to whole
// 4-element groups, -4 .. 67; p-bar_s, and for Potts the label sum of u,
// once for all labels), forms b on T+[-2,+3], runs the red, black, red
// half-sweeps of the symmetric Gauss-Seidel step on the shrinking regions in
// LDS, then the label's flows, relaxed reflection and stores on the tile;
// p-bar_s follows the last label.  The loads of label l+1 are issued before
// the LDS phases of label l.  With NS sweeps (the preconditioner M_NS) the
// 2 NS + 1 half-sweeps run on T+[-2NS,+2NS+1] down to T+[0,+1], b on the
// first of them and the staged rectangle is T+[-(2NS+1),+(2NS+2)].  Each
// cell's arithmetic (b with the Potts
// coupling st (n u_i - sum_j u_j), the Gauss-Seidel value with its
// neighbours summed in the order -x, +x, -y, +y, the flows, the reflection,
// the label sum of the new u in label order) is that of the in-place
// launches, so both variants give the same bits.
#pragma once
#include "mf_kernels.h"

namespace mf {

// Reciprocals 1 / (nb + m) of the Gauss-Seidel denominators, nb = 0 .. 6
// neighbours, rounded once on the host and shared by every rPDRQ kernel.
struct Rden {
  float r[7];
};

inline void set_rden(Rden& d, float m) {
  for (int i = 0; i < 7; i++) d.r[i] = 1.f / ((float)i + m);
}

// d.r[nb] by selects (a dynamic index would copy the table to scratch
// memory); a compile-time nb folds to one entry.
__device__ __forceinline__ float rden_at(const Rden d, int nb) {
  float v = d.r[0];
#pragma unroll
  for (int i = 1; i < 7; i++) v = nb == i ? d.r[i] : v;
  return v;
}

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
  float sigma, tau, rho, inv_st, alpha;
  Rden rden;            // 1 / (|N(x)| + m) for |N(x)| = 0 .. 6, rounded once on the host
  int iso, keep_z;
  int strip;          // tiles per column strip (see strip_tile)
  int nt;             // non-temporal stores of the new iterate
  const int* done;
  CapGen cg;            // cg.img: `cap` is one image plane
};

// Staged rectangle of a pass with NS symmetric sweeps (2 NS + 1 half-sweeps):
// rows -OY .. TY+OY, cols -OX .. 63+OX (whole 4-element groups).
template <int NS>
struct DrHalo {
  static constexpr int OY = 2 * NS + 1;
  static constexpr int OX = (2 * NS + 1 + 3) / 4 * 4;
  static constexpr int GPR = (64 + 2 * OX) / 4;   // 4-element groups per staged row
};

template <int TY, bool TWO, int NS = 1>
struct SmemDR {
  static constexpr int SW = 64 + 2 * DrHalo<NS>::OX;       // cols -OX .. 63+OX
  static constexpr int SH = TY + 2 * DrHalo<NS>::OY + 1;   // rows -OY .. TY+OY
  __align__(16) float su[SH][SW];
  __align__(16) float sqx[SH][SW];
  __align__(16) float sqy[SH][SW];
  __align__(16) float sps[SH][SW];
  __align__(16) float spt[SH][SW];    // p-bar of the label (p-bar_t for two labels)
  __align__(16) float sb[SH][SW];       // Potts: holds the label sum of u^k until the first b
};

// A tile whose staged rectangle (rows -OY .. TY+OY, cols -OX .. 63+OX) lies
// inside the grid, so that its b and half-sweep cells (rows -2 NS ..
// TY-1+2 NS, cols -2 NS .. 63+2 NS) all have their four neighbours inside.
template <int TY, int NS>
__device__ __forceinline__ bool dr_interior(int x0, int y0, int W, int H) {
  return x0 > 0 && y0 > 0 && x0 + 64 + DrHalo<NS>::OX <= W && y0 + TY + DrHalo<NS>::OY < H;
}

// EDGE false: an interior tile (dr_interior), whose every boundary test is
// true and folds away; the arithmetic is unchanged.  NS: symmetric sweeps
// per iteration (the preconditioner M_NS), 2 NS + 1 half-sweeps on regions
// shrinking by one cell per side.
template <typename TS, int TY, int NL, bool TWO, bool EDGE = true, int NS = 1, int NT = 256>
__device__ __forceinline__ void tile_dr2d(const KDF<TS>& A, int x0, int y0, SmemDR<TY, TWO, NS>& S) {
  constexpr int TX = 64, V = 4, TPR = TX / V, RSTEP = NT / TPR, RPT = TY / RSTEP;
  constexpr int OX = DrHalo<NS>::OX, OY = DrHalo<NS>::OY;
  constexpr int GPR = DrHalo<NS>::GPR;
  constexpr int NG = SmemDR<TY, TWO, NS>::SH * GPR;
  constexpr int KG = (NG + NT - 1) / NT;
  static_assert(RPT >= 1, "tile height must be a multiple of 16");
  static_assert(!TWO || NL == 1, "the two-label model carries one label");
  static_assert(NS >= 1 && NS <= 4 && 2 * NS < TY, "1 to 4 sweeps; the halo stays inside one tile row");
  auto& su = S.su;
  auto& sqx = S.sqx;
  auto& sqy = S.sqy;
  auto& sps = S.sps;
  auto& spt = S.spt;
  auto& sb = S.sb;
  const int tid = threadIdx.x;
  const int W = A.W, H = A.H, pitch = A.pitch;
  const long long P = A.P;
  // neighbour-inside-the-grid tests (zero flux outside)
  auto xp = [&](int x) { return !EDGE || x + 1 < W; };
  auto xm = [&](int x) { return !EDGE || x > 0; };
  auto yp = [&](int y) { return !EDGE || y + 1 < H; };
  auto ym = [&](int y) { return !EDGE || y > 0; };

  // this thread's staged groups (rows -OY .. TY+OY, cols -OX .. 63+OX)
  long long gi[KG];
  int gnv[KG];
#pragma unroll
  for (int m = 0; m < KG; m++) {
    const int h = tid + NT * m;
    const int r = h / GPR - OY, c = (h % GPR) * 4 - OX;
    const int gy = y0 + r, gx = x0 + c;
    const int nv = (h < NG && gy >= 0 && gy < H && gx >= 0) ? (W - gx >= V ? V : (W - gx > 0 ? W - gx : 0)) : 0;
    gnv[m] = nv;
    gi[m] = nv > 0 ? (long long)gy * pitch + gx : 0;
  }
  // write staged groups into an LDS array (entries outside the grid: 0; an
  // interior tile's staged rectangle lies inside the grid)
  auto put = [&](float (*dst)[SmemDR<TY, TWO, NS>::SW], int m, const float (&v)[V]) {
    const int h = tid + NT * m;
    if (h < NG) {
      const int r = h / GPR, c = (h % GPR) * 4;
#pragma unroll
      for (int e = 0; e < V; e++) dst[r][c + e] = (!EDGE || e < gnv[m]) ? v[e] : 0.f;
    }
  };
  // owned groups
  const int c0 = (tid % TPR) * V;
  const int rr0 = tid / TPR;
  const int gx0 = x0 + c0;
  const int nvx = W - gx0 < 0 ? 0 : (W - gx0 > V ? V : W - gx0);
  int nvj[RPT];
  long long oj[RPT];
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    const int gy = y0 + rr0 + RSTEP * j;
    nvj[j] = gy < H ? nvx : 0;
    oj[j] = (long long)gy * pitch + gx0;
  }
  // capacities of the owned groups: plane `pl` (raw), or the image plane
  const bool img = A.cg.img != 0;
  auto load_cap = [&](int pl, float (&o)[RPT][V]) {
#pragma unroll
    for (int j = 0; j < RPT; j++) ldv<V>(A.cap + (img ? 0 : (long long)pl * P), nvj[j] > 0 ? oj[j] : 0, o[j]);
  };
  auto cap_val = [&](float raw, int lv) { return img ? cap_from(raw, A.cg.lv[lv], A.cg.pw) : raw; };
  // u, q-bar, p-bar of one label on the staged groups and its capacities on
  // the owned groups, fetched into registers one label ahead of their use.
  // Potts loads p-bar when the label is staged instead, except BF16 with
  // n >= 4: a label ahead it spills registers under the four-waves-per-SIMD
  // limit and runs slower (FP32 n = 4 1024^2 38.2 -> 40.0 us, BF16 n = 2
  // 21.7 -> 24.3 us), but BF16 n = 4 and 8 gain (37.2 -> 36.2, 69.8 ->
  // 68.0 us).
  constexpr bool PF_PB = TWO || (sizeof(TS) == 2 && NL >= 4);
  float nu[KG][V], nqx[KG][V], nqy[KG][V], npt[KG][V], ncl[RPT][V];
  auto fetch = [&](int l) {
    const float* u_in = A.u_in + (long long)l * P;
    const TS* qx_in = A.qb_in + (long long)(2 * l) * P;
    const TS* pb_in = A.pb_in + (long long)l * P;
#pragma unroll
    for (int m = 0; m < KG; m++) {
      ldv<V>(u_in, gi[m], nu[m]);
      ldv<V>(qx_in, gi[m], nqx[m]);
      ldv<V>(qx_in + P, gi[m], nqy[m]);
      if (PF_PB) ldv<V>(pb_in, gi[m], npt[m]);
    }
    load_cap(TWO ? 1 : l, ncl);
  };
  fetch(0);

  // ---- label-independent staging: p-bar_s and (Potts) the label sum of u^k
  {
    float lps[KG][V];
#pragma unroll
    for (int m = 0; m < KG; m++) ldv<V>(A.psb_in, gi[m], lps[m]);
    if constexpr (!TWO) {
      float acc[KG][V];
#pragma unroll
      for (int m = 0; m < KG; m++)
#pragma unroll
        for (int e = 0; e < V; e++) acc[m][e] = 0.f;
#pragma unroll
      for (int l = 0; l < NL; l++) {
        float lu[KG][V];
#pragma unroll
        for (int m = 0; m < KG; m++) ldv<V>(A.u_in + (long long)l * P, gi[m], lu[m]);
#pragma unroll
        for (int m = 0; m < KG; m++)
#pragma unroll
          for (int e = 0; e < V; e++) acc[m][e] += lu[m][e];
      }
#pragma unroll
      for (int m = 0; m < KG; m++) put(sb, m, acc[m]);
    }
#pragma unroll
    for (int m = 0; m < KG; m++) put(sps, m, lps[m]);
  }
  float ocs[RPT][V];   // two labels: C_s
  if (TWO) load_cap(0, ocs);
  float usn[RPT][V];   // sum over labels of the new u (label order)
#pragma unroll
  for (int j = 0; j < RPT; j++)
#pragma unroll
    for (int e = 0; e < V; e++) usn[j][e] = 0.f;
  const float tau = A.tau, rho = A.rho;
  // b region T+[-2NS,+2NS+1]: thread tid takes cells tid + NT k, the same
  // cells for every label, so the Potts label sum of u^k at those cells,
  // staged in sb, moves to registers before the first b overwrites it (a
  // seventh LDS array would leave room for only three workgroups per CU)
  constexpr int BW = TX + 4 * NS + 1;
  constexpr int BN = (TY + 4 * NS + 1) * BW;
  constexpr int NB = (BN + NT - 1) / NT;
  float rsus[TWO ? 1 : NB];

  // Gauss-Seidel value of cell (r, c) from its neighbours in su and its b
  auto gs_b = [&](int r, int c, float bv) {
    const int hx = x0 + c, hy = y0 + r;
    const int R = r + OY, C = c + OX;
    float s = 0.f;
    int nb = 0;
    if (xm(hx)) { s += su[R][C - 1]; nb++; }
    if (xp(hx)) { s += su[R][C + 1]; nb++; }
    if (ym(hy)) { s += su[R - 1][C]; nb++; }
    if (yp(hy)) { s += su[R + 1][C]; nb++; }
    return (bv * A.inv_st + s) * rden_at(A.rden, nb);
  };
  auto gs = [&](int r, int c) { return gs_b(r, c, sb[r + OY][c + OX]); };
  // Half-sweep over the cells of one colour (0 red, 1 black: parity of
  // x + y; x0 and y0 are even) of rows rlo .. rlo+nr-1, cols clo .. clo+nc-1:
  // threads map onto that colour's cells only, lane pairs onto the j-th
  // such cell of two consecutive rows (the two rows' cells alternate in
  // column parity, so a wave's LDS accesses fall in distinct banks).
  auto half_sweep = [&](int rlo, int nr, int clo, int nc, int colour) {
    const int nch = (nc + 1) / 2;
    const int npr = (nr + 1) / 2;
    for (int h = tid; h < 2 * npr * nch; h += NT) {
      const int pr = h >> 1;
      const int r = rlo + 2 * (pr / nch) + (h & 1);
      const int c = clo + 2 * (pr % nch) + ((colour - r - clo) & 1);
      if (r < rlo + nr && c < clo + nc) su[r + OY][c + OX] = gs(r, c);
    }
  };

#pragma unroll 1
  for (int l = 0; l < NL; l++) {
    // ---- stage u, q-bar, p-bar of label l on the staged rectangle, then
    // start the loads of label l+1
    // (Potts other than BF16 n >= 4: p-bar of the label is loaded here, not
    // a label ahead, which keeps the registers within four waves per SIMD)
    if constexpr (!PF_PB) {
#pragma unroll
      for (int m = 0; m < KG; m++) ldv<V>(A.pb_in + (long long)l * P, gi[m], npt[m]);
    }
#pragma unroll
    for (int m = 0; m < KG; m++) {
      put(su, m, nu[m]);
      put(sqx, m, nqx[m]);
      put(sqy, m, nqy[m]);
      put(spt, m, npt[m]);
    }
    float ocl[RPT][V];   // C_t (two labels) or C_l, raw
#pragma unroll
    for (int j = 0; j < RPT; j++)
#pragma unroll
      for (int e = 0; e < V; e++) ocl[j][e] = ncl[j][e];
    if (l + 1 < NL) fetch(l + 1);
    lds_barrier();
    // ---- b on T+[-2NS,+2NS+1]: -sigma (div q-bar + p-bar - p-bar_s) (+ st (n u - sum u) for Potts),
    // and the first (red) half-sweep on the same region: a red cell's value
    // needs its own b and the old u of its black neighbours, which no red
    // update changes, so both run in one pass (b of a black cell reads only
    // its own old u)
#pragma unroll
    for (int k = 0; k < NB; k++) {
      const int h = tid + NT * k;
      if (k == NB - 1 && h >= BN) continue;
      const int r = h / BW - 2 * NS, c = h % BW - 2 * NS;
      const int hx = x0 + c, hy = y0 + r;
      const int R = r + OY, C = c + OX;
      const float d = ((xp(hx) ? sqx[R][C] : 0.f) - (xm(hx) ? sqx[R][C - 1] : 0.f)) +
                      ((yp(hy) ? sqy[R][C] : 0.f) - (ym(hy) ? sqy[R - 1][C] : 0.f));
      float bl = -A.sigma * ((d + spt[R][C]) - sps[R][C]);
      if constexpr (!TWO) {
        if (l == 0) rsus[k] = sb[R][C];
        bl += (A.sigma * A.tau) * ((float)NL * su[R][C] - rsus[k]);
      }
      sb[R][C] = bl;
      if (((r + c) & 1) == 0) su[R][C] = gs_b(r, c, bl);
    }
    lds_barrier();
    // ---- half-sweep j (red for even j) on T+[-(2NS-j), +(2NS+1-j)]: for one
    // sweep red on T+[-2,+3] (above), black on T+[-1,+2], red on T+[0,+1]
#pragma unroll
    for (int j = 1; j <= 2 * NS; j++) {
      half_sweep(j - 2 * NS, TY + 4 * NS + 1 - 2 * j, j - 2 * NS, TX + 4 * NS + 1 - 2 * j, j & 1);
      lds_barrier();
    }
    // ---- flows y = y-bar + tau K u and the relaxed reflection on the owned groups
    TS* qx_out = A.qb_out + (long long)(2 * l) * P;
    TS* pb_out = A.pb_out + (long long)l * P;
    float* u_out = A.u_out + (long long)l * P;
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      const int r = rr0 + RSTEP * j;
      const int gy = y0 + r;
      float un[V], qxo[V], qyo[V], zqx[V], zqy[V], pto[V], zpt[V];
      // the group's row of u (and its right neighbour), the row below, and
      // q-bar, p-bar: 16-byte LDS reads, one group per lane
      float lu[V + 1], lud[V], lqx[V], lqy[V], lpt[V];
      {
        const int R = r + OY, C = c0 + OX;
        const f32x4_t a = *reinterpret_cast<const f32x4_t*>(&su[R][C]);
        const f32x4_t b = *reinterpret_cast<const f32x4_t*>(&su[R + 1][C]);
        const f32x4_t x = *reinterpret_cast<const f32x4_t*>(&sqx[R][C]);
        const f32x4_t y = *reinterpret_cast<const f32x4_t*>(&sqy[R][C]);
        const f32x4_t t = *reinterpret_cast<const f32x4_t*>(&spt[R][C]);
#pragma unroll
        for (int e = 0; e < V; e++) {
          lu[e] = a[e];
          lud[e] = b[e];
          lqx[e] = x[e];
          lqy[e] = y[e];
          lpt[e] = t[e];
        }
        lu[V] = su[R][C + V];
      }
#pragma unroll
      for (int e = 0; e < V; e++) {
        const int gx = gx0 + e;
        const float u0 = lu[e];
        un[e] = u0;
        usn[j][e] += u0;
        float g0 = 0.f, g1 = 0.f;
        if (xp(gx)) g0 = lu[e + 1] - u0;
        if (yp(gy)) g1 = lud[e] - u0;
        // q = q-bar - tau grad u;  z_q = P_alpha(2q - q-bar);  q-bar += rho (z_q - q)
        const float qb0 = lqx[e], qb1 = lqy[e];
        const float q0 = qb0 - tau * g0, q1 = qb1 - tau * g1;
        float z0 = 2.f * q0 - qb0, z1 = 2.f * q1 - qb1;
        if (A.iso) proj2<true>(z0, z1, A.alpha);
        else proj2<false>(z0, z1, A.alpha);
        qxo[e] = qb0 + rho * (z0 - q0);
        qyo[e] = qb1 + rho * (z1 - q1);
        zqx[e] = z0;
        zqy[e] = z1;
        // p = p-bar + tau u;  z = min(C, 2p - p-bar);  p-bar += rho (z - p)
        const float pbv = lpt[e];
        const float pv = pbv + tau * u0;
        const float zpv = fminf(cap_val(ocl[j][e], TWO ? 1 : l), 2.f * pv - pbv);
        pto[e] = pbv + rho * (zpv - pv);
        zpt[e] = zpv;
      }
      const int nv = nvj[j];
      const long long idx = oj[j];
      stg<V>(u_out, idx, nv, true, un, A.nt != 0);
      stg<V>(qx_out, idx, nv, true, qxo, A.nt != 0);
      stg<V>(qx_out + P, idx, nv, true, qyo, A.nt != 0);
      stg<V>(pb_out, idx, nv, true, pto, A.nt != 0);
      if (A.keep_z) {
        stg<V>(A.zq + (long long)(2 * l) * P, idx, nv, true, zqx, A.nt != 0);
        stg<V>(A.zq + (long long)(2 * l + 1) * P, idx, nv, true, zqy, A.nt != 0);
        stg<V>(A.zp + (long long)l * P, idx, nv, true, zpt, A.nt != 0);
      }
    }
    if (NL > 1) lds_barrier();   // the next label's staging overwrites the arrays
  }
  // ---- p_s = p-bar_s - tau sum_i u_i;  z_s = (min(C_s,) 2 p_s - p-bar_s + tau)
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    const int r = rr0 + RSTEP * j;
    float pso[V], zps[V];
#pragma unroll
    for (int e = 0; e < V; e++) {
      const float psbv = sps[r + OY][c0 + e + OX];
      const float psv = psbv - tau * usn[j][e];
      float zsv = (2.f * psv - psbv) + tau;
      if (TWO) zsv = fminf(cap_val(ocs[j][e], 0), zsv);
      pso[e] = psbv + rho * (zsv - psv);
      zps[e] = zsv;
    }
    const int nv = nvj[j];
    const long long idx = oj[j];
    stg<V>(A.psb_out, idx, nv, true, pso, A.nt != 0);
    if (A.keep_z) stg<V>(A.zs, idx, nv, true, zps, A.nt != 0);
  }
}

}  // namespace mf
