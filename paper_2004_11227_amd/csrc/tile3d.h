// 3-D fused rpADMM tile (two-label model), z-marching; shared by the
// single-solve kernel and the persistent pool kernel.
//
// A block owns a 64 x 8 tile of the xy plane and a slab [z0, z1) of planes.
// It marches s = z0-2 .. z1, and at step s
//   1. stages q^k(s) (x, y, z components) and v(s) = (p_t - p_s) - u/c on
//      the tile plus its xy halo, into ring slot s & 1;
//   2. forms w(s) = div q^k(s) + v(s) (needs q_z^k(s-1), still in the other
//      slot) and, on the same cells in the same LDS phase, q^{k+1}(s-1) =
//      P_alpha(q^k(s-1) + grad w / a) in place (needs w(s-1) of the cell
//      and its +x, +y neighbours, formed a step earlier, and the cell's own
//      w(s) for the z difference);
//   3. for the owned pixels of plane s-1: d = div q^{k+1}(s-1) (the q_z of
//      plane s-2 is kept in registers), the pointwise p and u updates, and
//      the stores.
// Every plane is read from memory once per slab (plus the warm-up planes
// z0-1, z1 and the q_z component of z0-2), so z-neighbours cost no extra
// traffic; xy halos are shared through L2.
// The arithmetic is the same device-function sequence as the unfused 3-D
// baseline, so the two agree bit for bit.
#pragma once
#include "mf_kernels.h"

namespace mf {

template <typename TS>
__device__ __forceinline__ float quant3(float v);
template <>
__device__ __forceinline__ float quant3<float>(float v) { return v; }
template <>
__device__ __forceinline__ float quant3<bf16_t>(float v) {
  return __uint_as_float(((uint32_t)f2bf(v)) << 16);
}

template <typename TS>
struct K3 {
  int W, H, D;
  int pitch;           // row stride in elements (>= W)
  long long P, SZ;     // plane stride (fields), z stride (pitch*H)
  int tiles_x, tiles_y, tz;
  const TS* cap;
  const float* u_in;
  float* u_out;
  const TS* q_in;
  TS* q_out;
  const TS* ps_in;
  TS* ps_out;
  const TS* p_in;
  TS* p_out;
  Coef k;
  CapGen cg;           // with IMG: `cap` is one image plane
  double* acc;
  const int* done;
  int write;
  int iso;
  int strip;          // 2-D tile order: tiles per column strip (see strip_tile)
  int nt;             // non-temporal stores of the new iterate
};

__device__ __forceinline__ void proj3r(float& x, float& y, float& z, float alpha, int iso) {
  if (iso) proj3<true>(x, y, z, alpha);
  else proj3<false>(x, y, z, alpha);
}

// proj3r with selects in place of the isotropic case's branch: the same
// operations on the same values (the scale is formed for every cell and
// applied where |q| > alpha), so a loop over several cells stays one basic
// block and its LDS reads can all be in flight together.
__device__ __forceinline__ void proj3s(float& x, float& y, float& z, float alpha, int iso) {
  if (iso) {
    const float n2 = (x * x + y * y) + z * z;
    const bool out = n2 > alpha * alpha;
    const float sc = alpha * rsq(n2);
    x = out ? x * sc : x;
    y = out ? y * sc : y;
    z = out ? z * sc : z;
  } else {
    proj3<false>(x, y, z, alpha);
  }
}

template <bool SU, int TY = 8>
struct Smem3 {
  static constexpr int SW = 64 + 8;   // cols -4 .. 67
  static constexpr int SH = TY + 3;   // rows -2 .. TY
  __align__(16) float sqx[2][SH][SW];
  __align__(16) float sqy[2][SH][SW];
  __align__(16) float sqz[2][SH][SW];
  __align__(16) float sw[2][SH][SW];
  __align__(16) float su[SU ? 2 : 1][SU ? SH : 1][SU ? SW : 1];
  double sred[4 * 5];
};

// Registers holding one plane's loads ahead of their use: the owned pixels
// (q, u, p_t, p_s), at most one xy-halo entry of q and one of (u, p_t, p_s)
// per thread, and the capacities of the owned pixels.
template <int V>
struct Plane3 {
  float qx[V], qy[V], qz[V], u[V], p[V], ps[V];
  float hqx, hqy, hqz, hu, hp, hps;
};

// One 64 x TY tile (TY = 8 or 16; V = TY / 4 columns per thread) of the xy
// plane over the slab [z0, z1).  The global loads of plane s+1 (and the
// capacities of plane s) are issued at the start of step s, so their latency
// overlaps the LDS phases of step s.  IMG: the capacities are computed from
// one image plane (A.cg), read once per pixel instead of the two planes.
template <typename TS, bool CHECK, bool VEC, bool SU, int TY = 8, bool IMG = false>
__device__ __forceinline__ void tile3d(const K3<TS>& A, int x0, int y0, int z0, int z1, Smem3<SU, TY>& S,
                                       double (&g)[5]) {
  static_assert(!CHECK || SU, "the gap needs the u staging array");
  static_assert(TY == 8 || TY == 16, "3-D tiles are 64 x 8 or 64 x 16");
  constexpr int TX = 64, V = TY / 4, TPR = TX / V, OX = 4;
  constexpr int NHQ = 3 * (TX + 3) + 3 * TY;   // q halo: rows -2, -1, TY; cols -2, -1, TX
  constexpr int NHW = 2 * (TX + 2) + 2 * TY;   // w halo: rows -1, TY; cols -1, TX
  static_assert(NHQ <= 256 && NHW <= 256, "one halo entry per thread");
  auto& sqx = S.sqx;
  auto& sqy = S.sqy;
  auto& sqz = S.sqz;
  auto& sw = S.sw;
  auto& su = S.su;
  const int tid = threadIdx.x;
  const int W = A.W, H = A.H, D = A.D, pitch = A.pitch;
  const long long P = A.P, SZ = A.SZ;
  const int c0 = (tid % TPR) * V;
  const int r0 = tid / TPR;      // owned row of the tile (0..7)
  const int gx0 = x0 + c0, gy = y0 + r0;
  const int nvxy = (gy < H) ? (W - gx0 < 0 ? 0 : (W - gx0 > V ? V : W - gx0)) : 0;
  constexpr bool vec = VEC;
  const Coef k = A.k;
  const TS* qx_in = A.q_in;
  const TS* qy_in = A.q_in + P;
  const TS* qz_in = A.q_in + 2 * P;

  // this thread's halo entries (tile coordinates), fixed over the march
  int hq_r = 0, hq_c = 0, hw_r = 0, hw_c = 0;
  if (tid < NHQ) {
    if (tid < 3 * (TX + 3)) {
      const int rr = tid / (TX + 3);
      hq_r = rr == 0 ? -2 : (rr == 1 ? -1 : TY);
      hq_c = tid % (TX + 3) - 2;
    } else {
      const int hh = tid - 3 * (TX + 3);
      hq_r = hh / 3;
      const int cc = hh % 3;
      hq_c = cc == 0 ? -2 : (cc == 1 ? -1 : TX);
    }
  }
  if (tid < NHW) {
    if (tid < 2 * (TX + 2)) {
      hw_r = tid < TX + 2 ? -1 : TY;
      hw_c = tid % (TX + 2) - 1;
    } else {
      const int hh = tid - 2 * (TX + 2);
      hw_r = hh >> 1;
      hw_c = (hh & 1) ? TX : -1;
    }
  }
  const bool hq_xy = tid < NHQ && x0 + hq_c >= 0 && x0 + hq_c < W && y0 + hq_r >= 0 && y0 + hq_r < H;
  const bool hw_xy = tid < NHW && x0 + hw_c >= 0 && x0 + hw_c < W && y0 + hw_r >= 0 && y0 + hw_r < H;
  const long long hq_off = (long long)(y0 + hq_r) * pitch + (x0 + hq_c);
  const long long hw_off = (long long)(y0 + hw_r) * pitch + (x0 + hw_c);
  const long long own_off = (long long)gy * pitch + gx0;

  // Raw loads of plane s into F (no masking: entries outside the grid or
  // the slab load element 0 of the plane, one line for the whole wave); the
  // zeros are applied when the plane is staged, a step later, so the loads
  // stay in flight across the LDS phases.
  // The first warm-up plane z0-2 only supplies q_z^k (for div q^k at z0-1):
  // its other fields load element 0 (one cached line) instead of the plane;
  // their staged values feed only w(z0-2), which no output uses.
  auto fetch = [&](int s, Plane3<V>& F) {
    const bool zin = s >= 0 && s < D && s <= z1;
    const bool all = s > z0 - 2;
    const long long zoff = (long long)s * SZ;
    if (vec) {
      const long long i = (zin && nvxy > 0) ? zoff + own_off : 0;
      const long long ia = all ? i : 0;
      ldv<V>(qx_in, ia, F.qx);
      ldv<V>(qy_in, ia, F.qy);
      ldv<V>(qz_in, i, F.qz);
      ldv<V>(A.u_in, ia, F.u);
      ldv<V>(A.p_in, ia, F.p);
      ldv<V>(A.ps_in, ia, F.ps);
    } else {
#pragma unroll
      for (int e = 0; e < V; e++) {
        const long long i = (zin && e < nvxy) ? zoff + own_off + e : 0;
        const long long ia = all ? i : 0;
        F.qx[e] = ld(qx_in, ia);
        F.qy[e] = ld(qy_in, ia);
        F.qz[e] = ld(qz_in, i);
        F.u[e] = ld(A.u_in, ia);
        F.p[e] = ld(A.p_in, ia);
        F.ps[e] = ld(A.ps_in, ia);
      }
    }
    const long long iq = (zin && hq_xy) ? zoff + hq_off : 0;
    const long long iw = (zin && hw_xy && all) ? zoff + hw_off : 0;
    const long long iqa = all ? iq : 0;
    F.hqx = ld(qx_in, iqa);
    F.hqy = ld(qy_in, iqa);
    F.hqz = ld(qz_in, iq);
    F.hu = ld(A.u_in, iw);
    F.hp = ld(A.p_in, iw);
    F.hps = ld(A.ps_in, iw);
  };
  // Zero the entries of plane s that lie outside the grid.
  auto mask = [&](int s, Plane3<V>& F) {
    const bool zin = s >= 0 && s < D;
#pragma unroll
    for (int e = 0; e < V; e++) {
      const bool ok = zin && e < nvxy;
      F.qx[e] = ok ? F.qx[e] : 0.f;
      F.qy[e] = ok ? F.qy[e] : 0.f;
      F.qz[e] = ok ? F.qz[e] : 0.f;
      F.u[e] = ok ? F.u[e] : 0.f;
      F.p[e] = ok ? F.p[e] : 0.f;
      F.ps[e] = ok ? F.ps[e] : 0.f;
    }
    const bool iq = zin && hq_xy, iw = zin && hw_xy;
    F.hqx = iq ? F.hqx : 0.f;
    F.hqy = iq ? F.hqy : 0.f;
    F.hqz = iq ? F.hqz : 0.f;
    F.hu = iw ? F.hu : 0.f;
    F.hp = iw ? F.hp : 0.f;
    F.hps = iw ? F.hps : 0.f;
  };
  // Capacities of the owned pixels of plane z (raw: only pixels inside the
  // grid and the slab are used; with IMG the image values, in cs).
  auto fetch_caps = [&](int z, float (&cs)[V], float (&ct)[V]) {
    const bool ok = z >= z0 && z < z1;
    if (vec) {
      const long long i = (ok && nvxy > 0) ? (long long)z * SZ + own_off : 0;
      ldv<V>(A.cap, i, cs);
      if (!IMG) ldv<V>(A.cap + P, i, ct);
    } else {
#pragma unroll
      for (int e = 0; e < V; e++) {
        const long long i = (ok && e < nvxy) ? (long long)z * SZ + own_off + e : 0;
        cs[e] = ld(A.cap, i);
        if (!IMG) ct[e] = ld(A.cap + P, i);
      }
    }
  };

  // owner registers: values of plane s-1 (rotated each step)
  float u_m[V], p_m[V], s_m[V];   // u, p_t, p_s at plane s-1
  float q1z_mm[V];                // q_z^{k+1} at plane s-2
  double dk_m[V];                 // div q^k at plane s-1 (gap, FP64)
#pragma unroll
  for (int e = 0; e < V; e++) {
    u_m[e] = p_m[e] = s_m[e] = q1z_mm[e] = 0.f;
    dk_m[e] = 0.0;
  }
  Plane3<V> F;
  fetch(z0 - 2, F);
  float cs_n[V], ct_n[V];         // capacities of plane s-1 (loaded a step ahead)
#pragma unroll
  for (int e = 0; e < V; e++) cs_n[e] = ct_n[e] = 0.f;

#pragma unroll 1
  for (int s = z0 - 2; s <= z1; s++) {
    const int sl = s & 1, pl = sl ^ 1;   // slot of plane s, slot of plane s-1
    // ---- 1. stage plane s from the prefetch registers
    mask(s, F);
    float u_c[V], p_c[V], s_c[V];
#pragma unroll
    for (int e = 0; e < V; e++) {
      const int c = c0 + OX + e;
      u_c[e] = F.u[e];
      p_c[e] = F.p[e];
      s_c[e] = F.ps[e];
      sqx[sl][r0 + 2][c] = F.qx[e];
      sqy[sl][r0 + 2][c] = F.qy[e];
      sqz[sl][r0 + 2][c] = F.qz[e];
      sw[sl][r0 + 2][c] = vterm(p_c[e], s_c[e], u_c[e], k.inv_c);
      if (CHECK) su[sl][r0 + 2][c] = u_c[e];
    }
    if (tid < NHQ) {
      sqx[sl][hq_r + 2][hq_c + OX] = F.hqx;
      sqy[sl][hq_r + 2][hq_c + OX] = F.hqy;
      sqz[sl][hq_r + 2][hq_c + OX] = F.hqz;
    }
    if (tid < NHW) {
      sw[sl][hw_r + 2][hw_c + OX] = vterm(F.hp, F.hps, F.hu, k.inv_c);
      if (CHECK) su[sl][hw_r + 2][hw_c + OX] = F.hu;
    }
    float cs[V], ct[V];
#pragma unroll
    for (int e = 0; e < V; e++) {
      cs[e] = IMG ? cap_from(cs_n[e], A.cg.lv[0], A.cg.pw) : cs_n[e];
      ct[e] = IMG ? cap_from(cs_n[e], A.cg.lv[1], A.cg.pw) : ct_n[e];
    }
    // ---- issue the loads of plane s+1 and the capacities of plane s
    fetch(s + 1, F);
    fetch_caps(s, cs_n, ct_n);
    lds_barrier();
    // ---- gap of plane s-1 of the input iterate (owned pixels)
    if (CHECK && s - 1 >= z0 && s - 1 < z1) {
      const int zz = s - 1;
      const int nv = nvxy;
#pragma unroll
      for (int e = 0; e < V; e++) {
        if (e < nv) {
          const int gx = gx0 + e, c = c0 + OX + e;
          const double u0 = fmin(1.0, fmax(0.0, (double)su[pl][r0 + 2][c]));
          const double gxx = gx + 1 < W ? fmin(1.0, fmax(0.0, (double)su[pl][r0 + 2][c + 1])) - u0 : 0.0;
          const double gyy = gy + 1 < H ? fmin(1.0, fmax(0.0, (double)su[pl][r0 + 3][c])) - u0 : 0.0;
          const double gzz = zz + 1 < D ? fmin(1.0, fmax(0.0, (double)su[sl][r0 + 2][c])) - u0 : 0.0;
          const double dq = dk_m[e];
          g[0] += (1.0 - u0) * (double)cs[e] + u0 * (double)ct[e];
          g[1] += A.iso ? sqrt((gxx * gxx + gyy * gyy) + gzz * gzz) : (fabs(gxx) + fabs(gyy)) + fabs(gzz);
          g[2] += fmin((double)cs[e], (double)ct[e] + dq);
          const double r = ((double)p_m[e] - (double)s_m[e]) + dq;
          g[3] += r * r;
          g[4] += (double)s_m[e];
        }
      }
    }
    // FP64 div q^k at the owned pixels of plane s, for the next step's gap
    // (step 2 overwrites q_z^k(s-1) in place: the gap variant waits until
    // every thread has read it)
    if (CHECK) {
#pragma unroll
      for (int e = 0; e < V; e++) {
        const int gx = gx0 + e, c = c0 + OX + e;
        dk_m[e] = (((gx + 1 < W) ? (double)sqx[sl][r0 + 2][c] : 0.0) - ((gx > 0) ? (double)sqx[sl][r0 + 2][c - 1] : 0.0)) +
                  (((gy + 1 < H) ? (double)sqy[sl][r0 + 2][c] : 0.0) - ((gy > 0) ? (double)sqy[sl][r0 + 1][c] : 0.0)) +
                  (((s + 1 < D) ? (double)sqz[sl][r0 + 2][c] : 0.0) - ((s > 0) ? (double)sqz[pl][r0 + 2][c] : 0.0));
      }
      lds_barrier();
    }
    // ---- 2. w(s) = div q^k(s) + v(s) on rows -1..TY, cols -1..TX, and, on
    // the same cells where they lie in rows -1..TY-1, cols -1..TX-1,
    // q^{k+1}(s-1) = P_alpha(q^k(s-1) + grad w / a) in place.  A cell's q
    // step needs w(s-1) of its +x and +y neighbours (the previous step's,
    // complete) and its own w(s), which the same thread has just formed, so
    // the two need no barrier between them.  Each thread takes cells
    // tid + 256 k; all its reads come before its writes (a cell reads no
    // other cell's w(s) or q^k(s-1)), so the LDS reads of all its cells are
    // in flight together; the last, partial round recomputes a valid cell in
    // its idle threads and stores nothing.
    {
      constexpr int NC = (TY + 2) * (TX + 2), KC = (NC + 255) / 256;
      const bool qon = s - 1 >= z0 - 1;
      float wv[KC], qxv[KC], qyv[KC], qzv[KC];
#pragma unroll
      for (int kk = 0; kk < KC; kk++) {
        int h = tid + 256 * kk;
        if (kk == KC - 1) h = h < NC ? h : NC - 1;
        const int r = h / (TX + 2) - 1, c = h % (TX + 2) - 1;
        const int hx = x0 + c, hy = y0 + r;
        const float d = div3(sqx[sl][r + 2][c + OX], sqx[sl][r + 2][c + OX - 1], sqy[sl][r + 2][c + OX],
                             sqy[sl][r + 1][c + OX], sqz[sl][r + 2][c + OX], sqz[pl][r + 2][c + OX],
                             hx + 1 < W, hx > 0, hy + 1 < H, hy > 0, s + 1 < D, s > 0);
        const float wn = wterm(d, sw[sl][r + 2][c + OX]);
        wv[kk] = wn;
        // cells in row TY or column TX have no q step: they form a copy at
        // an in-range cell, which is not stored
        const int rq = r < TY ? r : TY - 1, cq = c < TX ? c : TX - 1;
        const float w0 = sw[pl][rq + 2][cq + OX];
        float qx = qstep(sqx[pl][rq + 2][cq + OX], sw[pl][rq + 2][cq + OX + 1], w0, x0 + cq + 1 < W, k.inv_a);
        float qy = qstep(sqy[pl][rq + 2][cq + OX], sw[pl][rq + 3][cq + OX], w0, y0 + rq + 1 < H, k.inv_a);
        float qz = qstep(sqz[pl][rq + 2][cq + OX], wn, w0, s < D, k.inv_a);
        proj3s(qx, qy, qz, k.alpha, A.iso);
        qxv[kk] = quant3<TS>(qx);
        qyv[kk] = quant3<TS>(qy);
        qzv[kk] = quant3<TS>(qz);
      }
#pragma unroll
      for (int kk = 0; kk < KC; kk++) {
        const int h = tid + 256 * kk;
        if (kk < KC - 1 || h < NC) {
          const int r = h / (TX + 2) - 1, c = h % (TX + 2) - 1;
          sw[sl][r + 2][c + OX] = wv[kk];
          if (qon && r < TY && c < TX) {
            sqx[pl][r + 2][c + OX] = qxv[kk];
            sqy[pl][r + 2][c + OX] = qyv[kk];
            sqz[pl][r + 2][c + OX] = qzv[kk];
          }
        }
      }
    }
    lds_barrier();
    // ---- 3. owned pixels of plane s-1: divergence, updates, stores
    if (s - 1 >= z0 && s - 1 < z1) {
      const int zz = s - 1;
      const int nv = nvxy;
      const long long idx = (long long)zz * SZ + own_off;
      float qxv[V], qyv[V], qzv[V], pn[V], psn[V], un[V];
#pragma unroll
      for (int e = 0; e < V; e++) {
        const int gx = gx0 + e, c = c0 + OX + e;
        qxv[e] = sqx[pl][r0 + 2][c];
        qyv[e] = sqy[pl][r0 + 2][c];
        qzv[e] = sqz[pl][r0 + 2][c];
        const float d = div3(qxv[e], sqx[pl][r0 + 2][c - 1], qyv[e], sqy[pl][r0 + 1][c], qzv[e], q1z_mm[e],
                             gx + 1 < W, gx > 0, gy + 1 < H, gy > 0, zz + 1 < D, zz > 0);
        float t, sd = 0.f, sr = 0.f;
        label_update(k, u_m[e], p_m[e], s_m[e], d, ct[e], pn[e], t, sd, sr);
        psn[e] = finish_ps(k, s_m[e], sd, sr, true, cs[e]);
        un[e] = finish_u(k, t, psn[e]);
      }
      if (A.write) {
        stg<V>(A.q_out, idx, nv, vec, qxv, A.nt != 0);
        stg<V>(A.q_out + P, idx, nv, vec, qyv, A.nt != 0);
        stg<V>(A.q_out + 2 * P, idx, nv, vec, qzv, A.nt != 0);
        stg<V>(A.p_out, idx, nv, vec, pn, A.nt != 0);
        stg<V>(A.ps_out, idx, nv, vec, psn, A.nt != 0);
        stg<V>(A.u_out, idx, nv, vec, un, A.nt != 0);
      }
    }
    // ---- rotate owner registers
#pragma unroll
    for (int e = 0; e < V; e++) {
      q1z_mm[e] = sqz[pl][r0 + 2][c0 + OX + e];
      u_m[e] = u_c[e];
      p_m[e] = p_c[e];
      s_m[e] = s_c[e];
    }
    lds_barrier();
  }
}

}  // namespace mf
