/*
 * FP64 CPU oracle for the continuous max-flow / min-cut methods of
 * Sun, Tai and Yuan, "Efficient ADMM and Splitting Methods for Continuous
 * Min-cut and Max-flow Problems" (arXiv 2004.11227).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU solver; it is plain loops in double
 * precision, written to be checked against the paper by eye.
 *
 * Grid: nx (fastest) x ny x nz, spacing 1; a 2-D grid has nz = 1, ndim = 2.
 * Planar layout, one contiguous plane of N = nx*ny*nz doubles per scalar:
 *   u  [L][N]          labelling function(s) (multiplier of the conservation law)
 *   q  [L][ndim][N]    spatial flows; component k is the k-th fastest axis
 *   ps [N]             source flow
 *   p  [L][N]          two-label: p_t (L = 1); Potts: p_1..p_n (L = n)
 *   caps               two-label: [C_s, C_t]; Potts: [C_1..C_n]
 * For rPDRQ, (q, ps, p) hold the reflected variables (q-bar, p-bar) and the
 * resolvent outputs of the last iteration are written to (zq, zs, zp).
 * The comparison methods of the experiments section are here too: the
 * classical sequential ADMM (pADMM-TY) and the Chambolle-Pock primal-dual
 * algorithm (ALG1, which also keeps the extrapolated u-bar [L][N]).
 */
#ifndef MAXFLOW_ORACLE_H
#define MAXFLOW_ORACLE_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { int ndim; long nx, ny, nz; } or_grid;

enum { OR_TWO = 0, OR_POTTS = 1 };
enum { OR_FG = 0, OR_EB = 1, OR_DR = 2, OR_TY = 3, OR_CP = 4 };
enum { OR_ISO = 0, OR_ANISO = 1 };

typedef struct {
  int model, method, tv, nlabels;
  double alpha;          /* TV weight                                        */
  double c;              /* ADMM step                                        */
  double relax;          /* FG: r; EB: rho (constant, or the schedule's end); DR: rho */
  double sigma, tau;     /* rPDRQ / ALG1 step sizes                          */
  double a;              /* q preconditioner N = a c I                       */
  double a_tilde;        /* two-label p preconditioner M = a~ c I_2          */
  double a1, a2;         /* Potts block preconditioner diag(a1 I.., a2 I)    */
  int gs_sweeps;         /* DR: symmetric red-black GS sweeps per iteration
                            (the preconditioner M_n; 0 or 1 -> one sweep)   */
  double relax0;         /* EB: rho_0 of a non-decreasing schedule; 0 -> the
                            constant rho = relax                             */
  long relax_ramp;       /* EB: rho_k rises linearly from relax0 to relax over
                            relax_ramp iterations, then stays at relax      */
} or_params;

void or_grad(const or_grid* g, const double* f, double* out);
void or_div(const or_grid* g, const double* q, double* out);
void or_project_alpha(const or_grid* g, int tv, double alpha, double* q);
void or_simplex_project(int n, const double* v, double* out);
void or_rbgs_sweep(const or_grid* g, double m, double st, const double* b, double* u);

void or_init(const or_grid* g, const or_params* p, const double* caps,
             double* u, double* q, double* ps, double* pp);
void or_admm_iter(const or_grid* g, const or_params* p, const double* caps,
                  double* u, double* q, double* ps, double* pp);
void or_pdrq_iter(const or_grid* g, const or_params* p, const double* caps,
                  double* u, double* qb, double* psb, double* pb,
                  double* zq, double* zs, double* zp);
void or_ty_iter(const or_grid* g, const or_params* p, const double* caps,
                double* u, double* q, double* ps, double* pp);
void or_cp_iter(const or_grid* g, const or_params* p, const double* caps,
                double* u, double* ub, double* q, double* ps, double* pp);
double or_rho_at(const or_params* p, long k);
void or_run(const or_grid* g, const or_params* p, const double* caps, long k0, long iters,
            double* u, double* q, double* ps, double* pp,
            double* zq, double* zs, double* zp, double* ub);
void or_energy(const or_grid* g, const or_params* p, const double* caps,
               const double* u, const double* q, const double* ps, const double* pp,
               double out[5]);
void or_labels(const or_grid* g, const or_params* p, const double* u, int* lab);
int  or_num_threads(void);
void or_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
