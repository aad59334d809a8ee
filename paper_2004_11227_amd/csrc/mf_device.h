// Device-side building blocks of the max-flow sweeps (gfx950).
//
// Every kernel variant (fused tile, unfused baseline, batched) evaluates the
// method through these inline functions, in the same operation order, and
// the library is compiled with -ffp-contract=off: variants that compute the
// same iterate therefore agree bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

// ---------------------------------------------------------------- storage
// bfloat16 is kept as raw 16-bit words.  Widening is exact (shift into the
// high half of an FP32 word); narrowing is gfx950's conversion instruction
// (v_cvt_pk_bf16_f32: round to nearest, ties to even; NaNs stay NaN).
typedef uint16_t bf16_t;
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float ld(const float* p, long long i) { return p[i]; }
__device__ __forceinline__ float ld(const bf16_t* p, long long i) {
  return __uint_as_float(((uint32_t)p[i]) << 16);
}
__device__ __forceinline__ bf16_t f2bf(float f) { return __builtin_bit_cast(bf16_t, (__bf16)f); }
__device__ __forceinline__ void st(float* p, long long i, float v) { p[i] = v; }
__device__ __forceinline__ void st(bf16_t* p, long long i, float v) { p[i] = f2bf(v); }
__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ uint32_t bf_pack(float a, float b) {
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));   // element 0 in the low half
}

// V consecutive elements starting at p[i] (i a multiple of V, 4*V-byte
// aligned): one vector memory instruction per lane.
template <int V>
__device__ __forceinline__ void ldv(const float* p, long long i, float (&o)[V]) {
  if constexpr (V == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p + i);
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
  } else if constexpr (V == 2) {
    const float2 t = *reinterpret_cast<const float2*>(p + i);
    o[0] = t.x; o[1] = t.y;
  } else {
    o[0] = p[i];
  }
}
template <int V>
__device__ __forceinline__ void ldv(const bf16_t* p, long long i, float (&o)[V]) {
  if constexpr (V == 4) {
    const uint2 t = *reinterpret_cast<const uint2*>(p + i);
    o[0] = bf_lo(t.x); o[1] = bf_hi(t.x); o[2] = bf_lo(t.y); o[3] = bf_hi(t.y);
  } else if constexpr (V == 2) {
    const uint32_t t = *reinterpret_cast<const uint32_t*>(p + i);
    o[0] = bf_lo(t); o[1] = bf_hi(t);
  } else {
    o[0] = ld(p, i);
  }
}
// Vector stores of the sweeps' outputs.  With `nt` the stores carry the
// non-temporal hint: the new iterate is not read again by this sweep, so on
// a working set larger than the last-level cache it should not take L2
// capacity from the halo rows that neighbouring tiles still have to read.
// (On a working set that fits the 256 MB last-level cache the hint costs
// more than it saves: the next sweep then reads the iterate from HBM.)
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v, bool nt) {
  if (nt) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <int V>
__device__ __forceinline__ void stv(float* p, long long i, const float (&v)[V], bool nt = false) {
  if constexpr (V == 4) {
    st_stream(reinterpret_cast<f32x4_t*>(p + i), f32x4_t{v[0], v[1], v[2], v[3]}, nt);
  } else if constexpr (V == 2) {
    st_stream(reinterpret_cast<f32x2_t*>(p + i), f32x2_t{v[0], v[1]}, nt);
  } else {
    st_stream(p + i, v[0], nt);
  }
}
template <int V>
__device__ __forceinline__ void stv(bf16_t* p, long long i, const float (&v)[V], bool nt = false) {
  if constexpr (V == 4) {
    st_stream(reinterpret_cast<u32x2_t*>(p + i), u32x2_t{bf_pack(v[0], v[1]), bf_pack(v[2], v[3])}, nt);
  } else if constexpr (V == 2) {
    st_stream(reinterpret_cast<uint32_t*>(p + i), bf_pack(v[0], v[1]), nt);
  } else {
    st_stream(p + i, f2bf(v[0]), nt);
  }
}
// Workgroup barrier for communication through LDS only: waits for this
// wave's LDS operations and meets the other waves, but leaves its global
// loads in flight.  __syncthreads() also drains outstanding global loads (its
// release fence covers global memory), which would stall loads that were
// issued ahead of their use.  No kernel here communicates through global
// memory inside a workgroup.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Guarded scalar load without a branch: the load always issues (from
// element 0 when `ok` is false, which every plane has) and the value is
// selected afterwards.  A load inside a branch makes the compiler wait for it
// at the end of the branch, which serialises the loads of a tile; branchless
// loads can all be in flight before the first use.
template <typename T>
__device__ __forceinline__ float ldz(const T* p, long long i, bool ok) {
  const float v = ld(p, ok ? i : 0);
  return ok ? v : 0.f;
}

// Group of V elements of one row, `nv` of them inside the grid (0..V).
// With `vec` the row pitch is a multiple of V, so a group that starts inside
// the row lies wholly inside the row's storage (the tail of a padded row
// included): one vector access, elements past the grid edge read as 0 and
// are written with don't-care values.  Without `vec`, element accesses.
// Loads are branchless (see ldz).
template <int V, typename T>
__device__ __forceinline__ void ldg(const T* p, long long i, int nv, bool vec, float (&o)[V]) {
  if (vec) {
    ldv<V>(p, nv > 0 ? i : 0, o);
#pragma unroll
    for (int e = 0; e < V; e++) o[e] = e < nv ? o[e] : 0.f;
  } else {
#pragma unroll
    for (int e = 0; e < V; e++) o[e] = ldz(p, i + e, e < nv);
  }
}
template <int V, typename T>
__device__ __forceinline__ void stg(T* p, long long i, int nv, bool vec, const float (&v)[V], bool nt = false) {
  if (vec) {
    if (nv > 0) stv<V>(p, i, v, nt);
  } else {
#pragma unroll
    for (int e = 0; e < V; e++)
      if (e < nv) st(p, i + e, v[e]);
  }
}

// ---------------------------------------------------------------- capacities
// Capacities generated from one image plane I instead of stored planes: the
// data cost of label l at x as a function of the image value and a per-label
// level, C_l(x) = |I(x) - lv[l]|^pw with pw 1 or 2, evaluated in FP32 where
// it is used (two-label: C_s from lv[0], C_t from lv[1]).
struct CapGen {
  int img = 0;        // 0: capacity planes; 1: one image plane
  int pw = 2;         // 1 or 2
  float lv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
};
__device__ __forceinline__ float cap_from(float I, float lv, int pw) {
  const float d = I - lv;
  return pw == 1 ? fabsf(d) : d * d;
}
// Capacity l at storage index i: plane l of `cap`, or computed from the
// image plane `cap` (element-wise kernels; l is a compile-time index there).
template <typename T>
__device__ __forceinline__ float cap_ld(const T* cap, long long P, int l, long long i, const CapGen& cg) {
  return cg.img ? cap_from(ld(cap, i), cg.lv[l], cg.pw) : ld(cap + (long long)l * P, i);
}

// ---------------------------------------------------------------- scalars
struct Coef {
  float alpha;      // TV weight
  float inv_c;      // 1/c
  float c;          // c
  float ku;         // multiplier-step factor: r c (FG) or c (EB)
  float rho;        // EB relaxation rho (1 for FG)
  float omr;        // 1 - rho
  float inv_a;      // 1/a   (q preconditioner N = a c I)
  float inv_a1;     // 1/a1  (two-label: 1/a~)
  float inv_a2;     // 1/a2  (two-label: 1/a~)
};

// 1/sqrt(v) by the hardware reciprocal square root (v_rsq_f32, about 1 ulp),
// its argument kept at least the smallest normal so that a zero or subnormal
// squared norm (possible only with alpha = 0) still gives a finite factor.
__device__ __forceinline__ float rsq(float v) { return __builtin_amdgcn_rsqf(fmaxf(v, 1.17549435e-38f)); }

// P_alpha: isotropic (pointwise Euclidean ball, eq. projections) or
// anisotropic (per-component clamp).  A vector inside the ball is returned
// unchanged; outside it is scaled by alpha/|q|, formed as alpha times the
// reciprocal square root of |q|^2 (the result's norm is alpha to a few ulp).
template <bool ISO>
__device__ __forceinline__ void proj2(float& x, float& y, float alpha) {
  if (ISO) {
    const float n2 = x * x + y * y;
    if (n2 > alpha * alpha) {
      const float s = alpha * rsq(n2);
      x = x * s;
      y = y * s;
    }
  } else {
    x = fminf(alpha, fmaxf(-alpha, x));
    y = fminf(alpha, fmaxf(-alpha, y));
  }
}
template <bool ISO>
__device__ __forceinline__ void proj3(float& x, float& y, float& z, float alpha) {
  if (ISO) {
    const float n2 = (x * x + y * y) + z * z;
    if (n2 > alpha * alpha) {
      const float s = alpha * rsq(n2);
      x = x * s;
      y = y * s;
      z = z * s;
    }
  } else {
    x = fminf(alpha, fmaxf(-alpha, x));
    y = fminf(alpha, fmaxf(-alpha, y));
    z = fminf(alpha, fmaxf(-alpha, z));
  }
}

// Divergence at a pixel from its own flux and the flux of its backward
// neighbours; `hi_k` says the forward neighbour along axis k exists, `lo_k`
// that the backward one does (zero flux through the boundary).
__device__ __forceinline__ float div2(float qx, float qx_w, float qy, float qy_n,
                                      bool hix, bool lox, bool hiy, bool loy) {
  return ((hix ? qx : 0.f) - (lox ? qx_w : 0.f)) + ((hiy ? qy : 0.f) - (loy ? qy_n : 0.f));
}
__device__ __forceinline__ float div3(float qx, float qx_w, float qy, float qy_n, float qz,
                                      float qz_b, bool hix, bool lox, bool hiy, bool loy,
                                      bool hiz, bool loz) {
  return (((hix ? qx : 0.f) - (lox ? qx_w : 0.f)) + ((hiy ? qy : 0.f) - (loy ? qy_n : 0.f))) +
         ((hiz ? qz : 0.f) - (loz ? qz_b : 0.f));
}

// v = (p_i - p_s) - u_i / c; the q-step argument is w = div q^k + v, and
// q^{k+1} = P_alpha(q^k + grad(w) / a)  (the (I - div^*div / a) q^k +
// grad(p - p_s - u/c) / a form of the q-updates of Section 3).
__device__ __forceinline__ float vterm(float p, float ps, float u, float inv_c) {
  return (p - ps) - u * inv_c;
}
__device__ __forceinline__ float wterm(float dq, float v) { return dq + v; }
__device__ __forceinline__ float qstep(float q, float wn, float w, bool inside, float inv_a) {
  return q + inv_a * (inside ? (wn - w) : 0.f);
}

// Per-label part of the p and u updates (rpADMMI / rpADMMII, two-label and
// Potts; the two-label model is the one-label case with p = p_t, a1 = a2 = a~
// and an extra clip of p_s at C_s):
//   r_i   = rho (p_i - p_s) - u_i / c
//   p_i'  = min(C_i, p_i - (r_i + rho d_i) / a1)
//   t_i   = u_i - ku ((rho d_i + p_i') - (1 - rho)(p_i - p_s))
// and the sums sum_d += rho d_i, sum_r += r_i.  The p_s and final u steps are
// finish_ps / finish_u (u_i' = t_i + ku p_s').  EB (rpADMMII) uses rho and
// ku = c; FG (rpADMMI) is the same expression with rho = 1, 1 - rho = 0 and
// ku = r c (the relaxation acts on the multiplier step only).
__device__ __forceinline__ void label_update(const Coef& k, float u, float p, float ps, float d,
                                             float C, float& pn, float& t, float& sum_d,
                                             float& sum_r) {
  const float dpp = p - ps;
  const float r = k.rho * dpp - u * k.inv_c;
  const float rd = k.rho * d;
  pn = fminf(C, p - (r + rd) * k.inv_a1);
  t = u - k.ku * ((rd + pn) - k.omr * dpp);
  sum_d += rd;
  sum_r += r;
}
__device__ __forceinline__ float finish_ps(const Coef& k, float ps, float sum_d, float sum_r,
                                           bool two, float Cs) {
  const float v = ps + ((sum_d + sum_r) + k.inv_c) * k.inv_a2;
  return two ? fminf(Cs, v) : v;
}
__device__ __forceinline__ float finish_u(const Coef& k, float t, float psn) {
  return t + k.ku * psn;
}

// ---------------------------------------------------------------- reductions
// One step of a wavefront sum: v plus v moved across lanes by the DPP control
// CTRL; rows outside ROWS add 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_add(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xf, false);
  return v + __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wavefront whose lanes are all active, by DPP
// lane moves instead of LDS permutes: pairs and quads (quad permutations),
// then 8 and 16 lanes (half-row and row mirrors) give every lane its row's
// sum; row broadcasts of lanes 15 and 31 then accumulate the rows into lane
// 63, whose value is returned to all lanes.
__device__ __forceinline__ double wave_total(double v) {
  v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Block-wide sum of NQ doubles, then one hardware FP64 atomic per quantity per
// block into slot (block id mod 64) of `dst` (rows of 8 doubles), so that
// thousands of blocks do not serialise on one address; the slots are summed
// in a fixed order by the bookkeeping kernel.
template <int NQ, int NWAVES>
__device__ __forceinline__ void block_accumulate(double (&v)[NQ], double* dst, double* sred) {
  const int lane = threadIdx.x & 63;
  const int wave = (threadIdx.x + threadIdx.y * blockDim.x) >> 6;
#pragma unroll
  for (int j = 0; j < NQ; j++) v[j] = wave_total(v[j]);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NQ; j++) sred[wave * NQ + j] = v[j];
  }
  __syncthreads();
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  if (tid < NQ) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVES; w++) s += sred[w * NQ + tid];
    unsafeAtomicAdd(dst + (blockIdx.x & 63) * 8 + tid, s);
  }
}

// Euclidean projection of (v_0..v_{n-1}) onto the probability simplex: the
// threshold is theta = max_j (S_j - 1) / k_j, where S_j and k_j are the sum
// and count of the entries ranked at or above v_j (ties broken by index);
// the projection is max(v - theta, 0).  Rank form without a sort, so the
// arrays stay in registers.
template <int N>
__device__ __forceinline__ double simplex_theta(const double (&v)[N]) {
  double theta = -1e300;
#pragma unroll
  for (int j = 0; j < N; j++) {
    double s = 0.0;
    double k = 0.0;
#pragma unroll
    for (int i = 0; i < N; i++) {
      const bool above = (v[i] > v[j]) || (v[i] == v[j] && i <= j);
      s += above ? v[i] : 0.0;
      k += above ? 1.0 : 0.0;
    }
    const double t = (s - 1.0) / k;
    theta = t > theta ? t : theta;
  }
  return theta;
}
// One component of the projection, max(v - theta, 0).
__device__ __forceinline__ double simplex_part(double v, double theta) { return v - theta > 0.0 ? v - theta : 0.0; }
template <int N>
__device__ __forceinline__ void simplex_proj(const double (&v)[N], double (&w)[N]) {
  const double theta = simplex_theta<N>(v);
#pragma unroll
  for (int i = 0; i < N; i++) w[i] = simplex_part(v[i], theta);
}

// XCD-aware tile order: consecutive workgroup ids are dispatched round-robin
// over the 8 XCDs, so map the workgroups that land on one XCD to one
// contiguous run of tiles; neighbouring tiles then share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  if (nb < 8) return b;
  const int x = b & 7, slot = b >> 3;
  const int base = nb >> 3, rem = nb & 7;
  return x * base + (x < rem ? x : rem) + slot;
}

// Order of the 2-D tiles within one XCD's contiguous run: column strips of
// `sw` tiles (64 * sw pixels), each walked row by row.  A tile's upper
// neighbour was then loaded at most a strip's width of tiles earlier on the
// same XCD, so its halo rows are still in that XCD's L2; a row-major walk of
// a wide grid puts a whole row of tiles (2.4 MB of state at 4096 columns,
// more than the 4 MB L2 holds with the writes and the workgroups in flight)
// between the two.  Any order gives the same iterate.  (The host takes
// strips only for working sets beyond the last-level cache: within it the
// row-major walk measured faster.)
constexpr int kStripTiles = 16;
__device__ __forceinline__ void strip_tile(int tile, int tiles_x, int tiles_y, int sw, int& tx, int& ty) {
  const int nfull = tiles_x / sw;
  const int full = nfull * sw * tiles_y;
  if (tile < full) {
    const int s = tile / (sw * tiles_y);
    const int r = tile - s * sw * tiles_y;
    ty = r / sw;
    tx = s * sw + (r - ty * sw);
  } else {
    const int rem = tiles_x - nfull * sw;
    const int r = tile - full;
    ty = r / rem;
    tx = nfull * sw + (r - ty * rem);
  }
}

}  // namespace mf
