/*
 * FP64 CPU oracle (TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke
 * check and the benchmark's CPU-baseline leg; never by the solver).
 *
 * Each function follows the paper's equations in the paper's order and
 * notation, with whole-array passes and plain loops.  Citations name the
 * paper's equation labels and sections.  Full-array loops are split over
 * rows with OpenMP; reductions are summed per row and then in row order, so
 * results do not depend on the thread count.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static size_t npix(const or_grid* g) { return (size_t)g->nx * g->ny * g->nz; }
static long nrows(const or_grid* g) { return g->ny * g->nz; }
static double* dalloc(size_t n) {
  double* p = (double*)calloc(n ? n : 1, sizeof(double));
  if (!p) abort();
  return p;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the later parallel loops (reductions stay in row order, so the
 * results do not depend on it). */
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Forward differences with Neumann boundary (the discretisation the paper
 * takes from Chambolle-Pock for its bound ||div^* div|| <= 8, Theorem 1):
 * (grad f)_k(x) = f(x + e_k) - f(x) if x + e_k lies in the grid, else 0. */
void or_grad(const or_grid* g, const double* f, double* out) {
  const size_t N = npix(g);
  const long nx = g->nx, ny = g->ny, nz = g->nz;
#pragma omp parallel for schedule(static)
  for (long r = 0; r < nrows(g); r++) {
    const long z = r / ny, y = r % ny;
    for (long x = 0; x < nx; x++) {
      const size_t i = (size_t)r * nx + x;
      out[i] = (x + 1 < nx) ? f[i + 1] - f[i] : 0.0;
      out[N + i] = (y + 1 < ny) ? f[i + nx] - f[i] : 0.0;
      if (g->ndim == 3) out[2 * N + i] = (z + 1 < nz) ? f[i + (size_t)nx * ny] - f[i] : 0.0;
    }
  }
}

/* div = -grad^*  (the adjoint relation used throughout Section 3):
 * div q(x) = sum_k [ q_k(x) 1{x+e_k inside} - q_k(x-e_k) 1{x-e_k inside} ]. */
void or_div(const or_grid* g, const double* q, double* out) {
  const size_t N = npix(g);
  const long nx = g->nx, ny = g->ny, nz = g->nz;
  const size_t sz = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
  for (long r = 0; r < nrows(g); r++) {
    const long z = r / ny, y = r % ny;
    for (long x = 0; x < nx; x++) {
      const size_t i = (size_t)r * nx + x;
      double s = 0.0;
      const double* qx = q;
      const double* qy = q + N;
      s += (x + 1 < nx ? qx[i] : 0.0) - (x > 0 ? qx[i - 1] : 0.0);
      s += (y + 1 < ny ? qy[i] : 0.0) - (y > 0 ? qy[i - nx] : 0.0);
      if (g->ndim == 3) {
        const double* qz = q + 2 * N;
        s += (z + 1 < nz ? qz[i] : 0.0) - (z > 0 ? qz[i - sz] : 0.0);
      }
      out[i] = s;
    }
  }
}

/* P_alpha of eq. (projections): q / max(1, |q|/alpha) with the pointwise
 * Euclidean norm (isotropic TV).  The anisotropic variant (l1 TV, used by
 * the exactness tests) clamps every component to [-alpha, alpha]. */
void or_project_alpha(const or_grid* g, int tv, double alpha, double* q) {
  const size_t N = npix(g);
  const int d = g->ndim;
#pragma omp parallel for schedule(static)
  for (long r = 0; r < nrows(g); r++) {
    for (long x = 0; x < g->nx; x++) {
      const size_t i = (size_t)r * g->nx + x;
      if (tv == OR_ANISO) {
        for (int k = 0; k < d; k++) {
          double v = q[k * N + i];
          q[k * N + i] = v > alpha ? alpha : (v < -alpha ? -alpha : v);
        }
      } else {
        double n2 = 0.0;
        for (int k = 0; k < d; k++) n2 += q[k * N + i] * q[k * N + i];
        const double nrm = sqrt(n2);
        if (alpha <= 0.0) {
          for (int k = 0; k < d; k++) q[k * N + i] = 0.0;
        } else {
          const double m = nrm / alpha > 1.0 ? nrm / alpha : 1.0;
          for (int k = 0; k < d; k++) q[k * N + i] = q[k * N + i] / m;
        }
      }
    }
  }
}

/* Euclidean projection onto the probability simplex (the pointwise constraint
 * set of the relaxed Potts model, eq. pw-simplex), by the sort-and-threshold
 * method of Held, Wolfe and Crowder (1974). */
void or_simplex_project(int n, const double* v, double* out) {
  double s[64];
  for (int i = 0; i < n; i++) s[i] = v[i];
  for (int i = 1; i < n; i++) { /* insertion sort, descending */
    double t = s[i];
    int j = i - 1;
    while (j >= 0 && s[j] < t) { s[j + 1] = s[j]; j--; }
    s[j + 1] = t;
  }
  double cum = 0.0, theta = 0.0;
  for (int j = 0; j < n; j++) {
    cum += s[j];
    const double t = (cum - 1.0) / (double)(j + 1);
    if (s[j] - t > 0.0) theta = t;
  }
  for (int i = 0; i < n; i++) out[i] = v[i] - theta > 0.0 ? v[i] - theta : 0.0;
}

static int nbr_count(const or_grid* g, long x, long y, long z) {
  int c = (x > 0) + (x + 1 < g->nx) + (y > 0) + (y + 1 < g->ny);
  if (g->ndim == 3) c += (z > 0) + (z + 1 < g->nz);
  return c;
}

/* One symmetric red-black Gauss-Seidel sweep (red, black, red) for
 * st * (-Delta + m I) u = b with Neumann boundary, i.e. the sRBGS
 * preconditioned step u <- u + M^{-1}(b - st(-Delta + m I) u) used by rPDRQ
 * (eq. iteration:quadratic:seg and the Potts form with T_0 of Lemma 1).
 * Red = (x + y + z) even.  Within a colour every update reads only the other
 * colour, so the in-place order inside a colour does not matter. */
void or_rbgs_sweep(const or_grid* g, double m, double st, const double* b, double* u) {
  const long nx = g->nx, ny = g->ny, nz = g->nz;
  const size_t sz = (size_t)nx * ny;
  const int colours[3] = {0, 1, 0};
  for (int pass = 0; pass < 3; pass++) {
    const int col = colours[pass];
#pragma omp parallel for schedule(static)
    for (long r = 0; r < nrows(g); r++) {
      const long z = r / ny, y = r % ny;
      for (long x = 0; x < nx; x++) {
        if (((x + y + z) & 1) != col) continue;
        const size_t i = (size_t)r * nx + x;
        double s = b[i] / st;
        if (x > 0) s += u[i - 1];
        if (x + 1 < nx) s += u[i + 1];
        if (y > 0) s += u[i - nx];
        if (y + 1 < ny) s += u[i + nx];
        if (g->ndim == 3) {
          if (z > 0) s += u[i - sz];
          if (z + 1 < nz) s += u[i + sz];
        }
        u[i] = s / ((double)nbr_count(g, x, y, z) + m);
      }
    }
  }
}

static int nl_of(const or_params* p) { return p->model == OR_TWO ? 1 : p->nlabels; }

/* Initial point (the paper states none): q = 0, u = 0 and the source/sink
 * flows at the pointwise minimum capacity, a feasible point with zero
 * conservation residual. */
void or_init(const or_grid* g, const or_params* p, const double* caps,
             double* u, double* q, double* ps, double* pp) {
  const size_t N = npix(g);
  const int L = nl_of(p), d = g->ndim;
  const int ncap = p->model == OR_TWO ? 2 : p->nlabels;
  memset(u, 0, sizeof(double) * L * N);
  memset(q, 0, sizeof(double) * (size_t)L * d * N);
  for (size_t i = 0; i < N; i++) {
    double m = caps[i];
    for (int k = 1; k < ncap; k++) m = caps[k * N + i] < m ? caps[k * N + i] : m;
    ps[i] = m;
    for (int l = 0; l < L; l++) pp[l * N + i] = m;
  }
}

/* q-step shared by every ADMM variant of Section 3 (rpADMMII, rpADMMI and the
 * multi-label forms): q <- P_alpha((I - (1/a) div^* div) q + (1/a) grad(f))
 * with f = p_t - p_s - u/c (two-label) or p_i - p_s - u_i/c (label i).
 * Since div^* = -grad, (I - (1/a) div^* div) q = q + (1/a) grad(div q). */
static void admm_q_step(const or_grid* g, const or_params* p, double* q, const double* f) {
  const size_t N = npix(g);
  const int d = g->ndim;
  double* dq = dalloc(N);
  double* gdq = dalloc((size_t)d * N);
  double* gf = dalloc((size_t)d * N);
  or_div(g, q, dq);
  or_grad(g, dq, gdq);
  or_grad(g, f, gf);
  for (size_t j = 0; j < (size_t)d * N; j++)
    q[j] = (q[j] + gdq[j] / p->a) + gf[j] / p->a;
  or_project_alpha(g, p->tv, p->alpha, q);
  free(dq); free(gdq); free(gf);
}

/* Two-label rpADMMII (Eckstein-Bertsekas type, eq. rpADMMII) and rpADMMI
 * (Fortin-Glowinski type, eq. rpADMMI); FG is the EB p-step with rho = 1
 * and a relaxed multiplier step u <- u - r c (A p + B q). */
static void admm_two(const or_grid* g, const or_params* p, const double* caps,
                     double* u, double* q, double* ps, double* pt) {
  const size_t N = npix(g);
  const double* Cs = caps;
  const double* Ct = caps + N;
  const double c = p->c, at = p->a_tilde;
  const int eb = p->method == OR_EB;
  const double rho = eb ? p->relax : 1.0;
  double* f = dalloc(N);
  double* dq = dalloc(N);
  for (size_t i = 0; i < N; i++) f[i] = pt[i] - ps[i] - u[i] / c;
  admm_q_step(g, p, q, f);
  or_div(g, q, dq); /* div q^{k+1} */
  for (size_t i = 0; i < N; i++) {
    const double ptn = fmin(Ct[i], pt[i] - rho / at * (pt[i] - ps[i]) + 1.0 / at * (-rho * dq[i] + u[i] / c));
    const double psn = fmin(Cs[i], ps[i] - rho / at * (ps[i] - pt[i]) + 1.0 / at * (rho * dq[i] - u[i] / c + 1.0 / c));
    double un;
    if (eb)
      un = u[i] - c * ((ptn - psn) - (1.0 - rho) * (pt[i] - ps[i]) + rho * dq[i]);
    else
      un = u[i] - p->relax * c * ((ptn - psn) + dq[i]);
    pt[i] = ptn; ps[i] = psn; u[i] = un;
  }
  free(f); free(dq);
}

/* Multi-label (Potts) rpADMMII (component-wise EB scheme of the multi-phase
 * section, with coefficient 1 on (p_i^{k+1} - p_s^{k+1}) in the u-step as in
 * the general EB update) and rpADMMI (eq. multi:fg:4), both with the block
 * preconditioner diag(a1 I, ..., a1 I, a2 I) of eq. multilabel:pre:p. */
static void admm_potts(const or_grid* g, const or_params* p, const double* caps,
                       double* u, double* q, double* ps, double* pp) {
  const size_t N = npix(g);
  const int n = p->nlabels, d = g->ndim;
  const double c = p->c, a1 = p->a1, a2 = p->a2;
  const int eb = p->method == OR_EB;
  const double rho = eb ? p->relax : 1.0;
  double* f = dalloc(N);
  double* dqa = dalloc((size_t)n * N);
  for (int l = 0; l < n; l++) {
    for (size_t i = 0; i < N; i++) f[i] = pp[l * N + i] - ps[i] - u[l * N + i] / c;
    admm_q_step(g, p, q + (size_t)l * d * N, f);
    or_div(g, q + (size_t)l * d * N, dqa + (size_t)l * N);
  }
  for (size_t i = 0; i < N; i++) {
    double sum_d = 0.0, sum_r = 0.0;
    double pn[64];
    for (int l = 0; l < n; l++) {
      const double pi = pp[l * N + i], ui = u[l * N + i], di = dqa[l * N + i];
      pn[l] = fmin(caps[l * N + i], pi - 1.0 / a1 * (rho * (pi - ps[i]) - ui / c + rho * di));
      sum_d += di;
      sum_r += rho * (pi - ps[i]) - ui / c;
    }
    const double psn = ps[i] + 1.0 / a2 * (rho * sum_d + sum_r + 1.0 / c);
    for (int l = 0; l < n; l++) {
      const double pi = pp[l * N + i], ui = u[l * N + i], di = dqa[l * N + i];
      double un;
      if (eb)
        un = ui - c * (rho * di + (pn[l] - psn) - (1.0 - rho) * (pi - ps[i]));
      else
        un = ui - p->relax * c * (di + pn[l] - psn);
      u[l * N + i] = un;
      pp[l * N + i] = pn[l];
    }
    ps[i] = psn;
  }
  free(f); free(dqa);
}

void or_admm_iter(const or_grid* g, const or_params* p, const double* caps,
                  double* u, double* q, double* ps, double* pp) {
  if (p->model == OR_TWO) admm_two(g, p, caps, u, q, ps, pp);
  else admm_potts(g, p, caps, u, q, ps, pp);
}

/* rPDRQ (relaxed, preconditioned Douglas-Rachford with the sRBGS
 * preconditioner): two-label eq. iteration:quadratic:seg with
 * K = (-grad; I; -I), T_Q = st(-Delta + 2I); multi-label eq. pdrq:4labels
 * for general n with T_0 = diag(-Delta + (n+1) I) of Lemma 1.  The resolvent
 * of tau dG for G = -<1, p_s> + indicators is min(C_s, . + tau) on p_s,
 * (. + tau) for the unconstrained Potts p_s, P_alpha on q, min(C, .) on the
 * other flows. */
void or_pdrq_iter(const or_grid* g, const or_params* p, const double* caps,
                  double* u, double* qb, double* psb, double* pb,
                  double* zq, double* zs, double* zp) {
  const size_t N = npix(g);
  const int d = g->ndim;
  const double sg = p->sigma, tau = p->tau, rho = p->relax, st = sg * tau;
  const int two = p->model == OR_TWO;
  const int L = two ? 1 : p->nlabels;
  double* b = dalloc((size_t)L * N);
  double* dq = dalloc(N);
  double* gu = dalloc((size_t)d * N);
  double* qn = dalloc((size_t)d * N);
  /* b^k */
  for (int l = 0; l < L; l++) {
    or_div(g, qb + (size_t)l * d * N, dq);
    for (size_t i = 0; i < N; i++) {
      double bi = -sg * (dq[i] + pb[l * N + i] - psb[i]);
      if (!two) {
        double others = 0.0;
        for (int j = 0; j < L; j++) if (j != l) others += u[j * N + i];
        bi += st * ((double)(L - 1) * u[l * N + i] - others);
      }
      b[l * N + i] = bi;
    }
  }
  /* u^{k+1}: gs_sweeps symmetric red-black GS sweeps per label (one sweep is
   * the sRBGS preconditioner; n sweeps are the preconditioner M_n, n steps of
   * the preconditioned iteration for T u = b from u^k) */
  const double m = two ? 2.0 : (double)(L + 1);
  const int nsw = p->gs_sweeps > 1 ? p->gs_sweeps : 1;
  for (int l = 0; l < L; l++)
    for (int sw = 0; sw < nsw; sw++) or_rbgs_sweep(g, m, st, b + (size_t)l * N, u + (size_t)l * N);
  /* y^{k+1} = y-bar + tau K u^{k+1}, then the relaxed reflection */
  for (int l = 0; l < L; l++) {
    double* qbl = qb + (size_t)l * d * N;
    double* zql = zq + (size_t)l * d * N;
    or_grad(g, u + (size_t)l * N, gu);
    for (size_t j = 0; j < (size_t)d * N; j++) {
      qn[j] = qbl[j] - tau * gu[j];
      zql[j] = 2.0 * qn[j] - qbl[j];
    }
    or_project_alpha(g, p->tv, p->alpha, zql);
    for (size_t j = 0; j < (size_t)d * N; j++) qbl[j] = qbl[j] + rho * (zql[j] - qn[j]);
  }
  for (size_t i = 0; i < N; i++) {
    double usum = 0.0;
    for (int l = 0; l < L; l++) usum += u[l * N + i];
    const double psn = psb[i] - tau * usum;
    for (int l = 0; l < L; l++) {
      const double pn = pb[l * N + i] + tau * u[l * N + i];
      const double z = fmin(caps[(two ? 1 : l) * N + i], 2.0 * pn - pb[l * N + i]);
      zp[l * N + i] = z;
      pb[l * N + i] = pb[l * N + i] + rho * (z - pn);
    }
    double z = 2.0 * psn - psb[i] + tau;
    if (two) z = fmin(caps[i], z);
    zs[i] = z;
    psb[i] = psb[i] + rho * (z - psn);
  }
  free(b); free(dq); free(gu); free(qn);
}

/* pADMM-TY, the classical ADMM the paper compares against: the same q-step
 * as above, then the flows block by block.
 * Two labels (eq. ADMM:Tai_yuan): p_s, then p_t with the new p_s, then u:
 *   p_s' = min(C_s, p_t + div q' - u/c + 1/c),
 *   p_t' = min(C_t, p_s' - div q' + u/c),
 *   u'   = u - c (p_t' - p_s' + div q').
 * n labels (eq. mADMM:Tai_yuan), blocks in the order q, p_i, p_s, u:
 *   p_i' = min(C_i, p_s - div q_i' + u_i/c),
 *   p_s' = (sum_i (p_i' + div q_i' - u_i/c) + 1/c) / n   (the new p_i', as a
 *          sequential block update takes them; with the old p_i, as the
 *          printed superscript reads, the scheme diverges on every
 *          synthetic input tried),
 *   u_i' = u_i - c (p_i' - p_s' + div q_i').
 * The printed "u^k = u^k - ..." is the multiplier update u^{k+1}. */
void or_ty_iter(const or_grid* g, const or_params* p, const double* caps,
                double* u, double* q, double* ps, double* pp) {
  const size_t N = npix(g);
  const int d = g->ndim;
  const double c = p->c;
  double* f = dalloc(N);
  if (p->model == OR_TWO) {
    const double* Cs = caps;
    const double* Ct = caps + N;
    double* dq = dalloc(N);
    for (size_t i = 0; i < N; i++) f[i] = pp[i] - ps[i] - u[i] / c;
    admm_q_step(g, p, q, f);
    or_div(g, q, dq);
    for (size_t i = 0; i < N; i++) {
      const double psn = fmin(Cs[i], pp[i] + dq[i] - u[i] / c + 1.0 / c);
      const double ptn = fmin(Ct[i], psn - dq[i] + u[i] / c);
      u[i] = u[i] - c * (ptn - psn + dq[i]);
      ps[i] = psn;
      pp[i] = ptn;
    }
    free(dq);
  } else {
    const int n = p->nlabels;
    double* dqa = dalloc((size_t)n * N);
    for (int l = 0; l < n; l++) {
      for (size_t i = 0; i < N; i++) f[i] = pp[l * N + i] - ps[i] - u[l * N + i] / c;
      admm_q_step(g, p, q + (size_t)l * d * N, f);
      or_div(g, q + (size_t)l * d * N, dqa + (size_t)l * N);
    }
    for (size_t i = 0; i < N; i++) {
      double pn[64], s = 0.0;
      for (int l = 0; l < n; l++) {
        const double di = dqa[l * N + i], ui = u[l * N + i];
        pn[l] = fmin(caps[l * N + i], ps[i] - di + ui / c);
        s += pn[l] + di - ui / c;
      }
      const double psn = s / n + 1.0 / (n * c);
      for (int l = 0; l < n; l++) {
        u[l * N + i] = u[l * N + i] - c * (pn[l] - psn + dqa[l * N + i]);
        pp[l * N + i] = pn[l];
      }
      ps[i] = psn;
    }
    free(dqa);
  }
  free(f);
}

/* ALG1: the Chambolle-Pock primal-dual algorithm applied to the primal-dual
 * forms of the appendix (eqs. iteration:pd:seg and alg1:4labels), dual step
 * first with the extrapolated u-bar, then the primal step, then the
 * extrapolation u-bar' = 2 u' - u.
 * Two labels: q' = P_alpha(q - sigma grad u-bar), p_t' = min(C_t, p_t +
 *   sigma u-bar), p_s' = min(C_s, p_s - sigma u-bar + sigma) (the +sigma of
 *   the source term, as in the n-label p_s step; the printed p-bar on p_t is
 *   p_t), u' = u - tau (div q' + p_t' - p_s').
 * n labels: q_i' = P_alpha(q_i - sigma grad u-bar_i) (u-bar as in the
 *   general dual step), p_i' = min(C_i, p_i + sigma u-bar_i), p_s' = p_s -
 *   sigma sum_i u-bar_i + sigma, u_i' = u_i - tau (div q_i' + p_i' - p_s'). */
void or_cp_iter(const or_grid* g, const or_params* p, const double* caps,
                double* u, double* ub, double* q, double* ps, double* pp) {
  const size_t N = npix(g);
  const int d = g->ndim;
  const int two = p->model == OR_TWO;
  const int L = two ? 1 : p->nlabels;
  const double sg = p->sigma, tau = p->tau;
  double* gu = dalloc((size_t)d * N);
  double* dq = dalloc((size_t)L * N);
  for (int l = 0; l < L; l++) {
    double* ql = q + (size_t)l * d * N;
    or_grad(g, ub + (size_t)l * N, gu);
    for (size_t j = 0; j < (size_t)d * N; j++) ql[j] = ql[j] - sg * gu[j];
    or_project_alpha(g, p->tv, p->alpha, ql);
    or_div(g, ql, dq + (size_t)l * N);
  }
  for (size_t i = 0; i < N; i++) {
    double sum_ub = 0.0;
    for (int l = 0; l < L; l++) {
      pp[l * N + i] = fmin(caps[(two ? 1 : l) * N + i], pp[l * N + i] + sg * ub[l * N + i]);
      sum_ub += ub[l * N + i];
    }
    double psn = ps[i] - sg * sum_ub + sg;
    if (two) psn = fmin(caps[i], psn);
    ps[i] = psn;
    for (int l = 0; l < L; l++) {
      const double un = u[l * N + i] - tau * (dq[l * N + i] + pp[l * N + i] - psn);
      ub[l * N + i] = 2.0 * un - u[l * N + i];
      u[l * N + i] = un;
    }
  }
  free(gu); free(dq);
}

/* rho_k of rpADMMII at iteration k (the step from iterate k to k+1): the
 * relaxation may be any non-decreasing sequence in (0, 2); here either the
 * constant relax, or a linear rise from relax0 at k = 0 to relax at
 * k = relax_ramp, constant afterwards. */
double or_rho_at(const or_params* p, long k) {
  if (!(p->relax0 > 0.0) || p->relax_ramp <= 0 || k >= p->relax_ramp) return p->relax;
  return p->relax0 + (p->relax - p->relax0) * ((double)k / (double)p->relax_ramp);
}

/* Iterations k0 .. k0+iters-1 (k0 = index of the incoming iterate, which
 * only the rpADMMII relaxation schedule depends on). */
void or_run(const or_grid* g, const or_params* p, const double* caps, long k0, long iters,
            double* u, double* q, double* ps, double* pp,
            double* zq, double* zs, double* zp, double* ub) {
  or_params pk = *p;
  for (long k = 0; k < iters; k++) {
    if (p->method == OR_DR) or_pdrq_iter(g, p, caps, u, q, ps, pp, zq, zs, zp);
    else if (p->method == OR_TY) or_ty_iter(g, p, caps, u, q, ps, pp);
    else if (p->method == OR_CP) or_cp_iter(g, p, caps, u, ub, q, ps, pp);
    else {
      if (p->method == OR_EB) pk.relax = or_rho_at(p, k0 + k);
      or_admm_iter(g, &pk, caps, u, q, ps, pp);
    }
  }
}

/* Energies.  Primal: relaxed min-cut (eq. seg:chanvese) at clip(u, 0, 1), or
 * relaxed Potts (eq. relaxed-potts) at the pointwise simplex projection of u.
 * Dual: the max-flow objective sum p_s maximised over p for fixed q subject
 * to conservation and capacities: sum min(C_s, C_t + div q) (two-label,
 * eq. two-label-mf) or sum min_i (C_i + div q_i) (Potts, eq. potts-mf).
 * out = [data, tv, dual, residual^2, flow]; primal = data + alpha * tv. */
void or_energy(const or_grid* g, const or_params* p, const double* caps,
               const double* u, const double* q, const double* ps, const double* pp,
               double out[5]) {
  const size_t N = npix(g);
  const int d = g->ndim;
  const int two = p->model == OR_TWO;
  const int L = two ? 1 : p->nlabels;
  const long R = nrows(g);
  double* ub = dalloc((size_t)L * N);
  double* gu = dalloc((size_t)d * N);
  double* dq = dalloc((size_t)L * N);
  double* rowacc = dalloc((size_t)R * 5);
  if (two) {
    for (size_t i = 0; i < N; i++) ub[i] = u[i] < 0.0 ? 0.0 : (u[i] > 1.0 ? 1.0 : u[i]);
  } else {
    double v[64], w[64];
    for (size_t i = 0; i < N; i++) {
      for (int l = 0; l < L; l++) v[l] = u[l * N + i];
      or_simplex_project(L, v, w);
      for (int l = 0; l < L; l++) ub[l * N + i] = w[l];
    }
  }
  for (int l = 0; l < L; l++) or_div(g, q + (size_t)l * d * N, dq + (size_t)l * N);
  for (int l = 0; l < L; l++) {
    or_grad(g, ub + (size_t)l * N, gu);
#pragma omp parallel for schedule(static)
    for (long r = 0; r < R; r++) {
      double tv = 0.0;
      for (long x = 0; x < g->nx; x++) {
        const size_t i = (size_t)r * g->nx + x;
        if (p->tv == OR_ANISO) {
          for (int k = 0; k < d; k++) tv += fabs(gu[k * N + i]);
        } else {
          double s = 0.0;
          for (int k = 0; k < d; k++) s += gu[k * N + i] * gu[k * N + i];
          tv += sqrt(s);
        }
      }
      rowacc[r * 5 + 1] += tv;
    }
  }
#pragma omp parallel for schedule(static)
  for (long r = 0; r < R; r++) {
    double data = 0.0, dual = 0.0, r2 = 0.0, flow = 0.0;
    for (long x = 0; x < g->nx; x++) {
      const size_t i = (size_t)r * g->nx + x;
      if (two) {
        const double Cs = caps[i], Ct = caps[N + i];
        data += (1.0 - ub[i]) * Cs + ub[i] * Ct;
        dual += fmin(Cs, Ct + dq[i]);
        const double res = pp[i] - ps[i] + dq[i];
        r2 += res * res;
      } else {
        double mn = INFINITY;
        for (int l = 0; l < L; l++) {
          data += ub[l * N + i] * caps[l * N + i];
          const double t = caps[l * N + i] + dq[l * N + i];
          mn = t < mn ? t : mn;
          const double res = dq[l * N + i] + pp[l * N + i] - ps[i];
          r2 += res * res;
        }
        dual += mn;
      }
      flow += ps[i];
    }
    rowacc[r * 5 + 0] = data;
    rowacc[r * 5 + 2] = dual;
    rowacc[r * 5 + 3] = r2;
    rowacc[r * 5 + 4] = flow;
  }
  for (int k = 0; k < 5; k++) out[k] = 0.0;
  for (long r = 0; r < R; r++)
    for (int k = 0; k < 5; k++) out[k] += rowacc[r * 5 + k];
  free(ub); free(gu); free(dq); free(rowacc);
}

/* Labels: two-label threshold u > 1/2 (any threshold in (0,1) is exact for a
 * binary minimiser, remark after eq. seg:chanvese); Potts argmax, lowest
 * index on ties. */
void or_labels(const or_grid* g, const or_params* p, const double* u, int* lab) {
  const size_t N = npix(g);
  if (p->model == OR_TWO) {
    for (size_t i = 0; i < N; i++) lab[i] = u[i] > 0.5;
    return;
  }
  for (size_t i = 0; i < N; i++) {
    int best = 0;
    for (int l = 1; l < p->nlabels; l++)
      if (u[l * N + i] > u[best * N + i]) best = l;
    lab[i] = best;
  }
}
