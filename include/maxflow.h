/*
 * maxflow.h -- C ABI of the MI355X (gfx950) continuous max-flow / min-cut
 * solver for the methods of Sun, Tai and Yuan, "Efficient ADMM and Splitting
 * Methods for Continuous Min-cut and Max-flow Problems" (arXiv 2004.11227).
 *
 * Models (Section 2.1):
 *   MF_TWO_LABEL  relaxed min-cut, eq. seg:chanvese, and its dual max-flow,
 *                 eq. two-label-mf:  max sum p_s  s.t. |q| <= alpha,
 *                 p_s <= C_s, p_t <= C_t, p_t - p_s + div q = 0
 *                 (the sign convention of the augmented Lagrangian
 *                 eq. augfunc:twolabel).
 *   MF_POTTS      relaxed Potts model, eq. relaxed-potts, and its dual,
 *                 eq. potts-mf:  max sum p_s  s.t. |q_i| <= alpha,
 *                 p_i <= C_i, div q_i - p_s + p_i = 0.
 * Methods (Section 3):
 *   MF_RPADMM_FG  rpADMMI, relaxed preconditioned ADMM of Fortin-Glowinski
 *                 type (eq. rpADMMI; multi-label eq. multi:fg:4).
 *   MF_RPADMM_EB  rpADMMII, relaxed preconditioned ADMM of Eckstein-Bertsekas
 *                 type (eq. rpADMMII; multi-label component-wise scheme of the
 *                 multi-phase EB subsection, with coefficient 1 on
 *                 (p_i^{k+1} - p_s^{k+1}) in the multiplier step as in the
 *                 general EB update eq. update:two:sun:lag).
 *   MF_RPDRQ      rPDRQ, relaxed Douglas-Rachford with a symmetric red-black
 *                 Gauss-Seidel preconditioner (eq. iteration:quadratic:seg;
 *                 multi-label eq. pdrq:4labels for general n, T_0 of Lemma 1).
 * The comparison methods of the experiments section (element-wise kernels;
 * the unfused variant is implied):
 *   MF_PADMM_TY   pADMM-TY, the classical sequential ADMM (eq. ADMM:Tai_yuan;
 *                 multi-label eq. mADMM:Tai_yuan, blocks q, p_i, p_s, u in
 *                 sequence, so the p_s step takes the new p_i).  Uses c and
 *                 a; no convergence guarantee.
 *   MF_CP_ALG1    ALG1, the Chambolle-Pock primal-dual algorithm of the
 *                 appendix (eqs. iteration:pd:seg, alg1:4labels; the
 *                 two-label p_s step with +sigma as in the n-label one).
 *                 sigma 0 -> 0.4, tau 0 -> 1 / (L^2 sigma) with L^2 = 4 ndim
 *                 + 2 (two labels) or 4 ndim + n + 1 (n labels); sigma tau
 *                 L^2 > 1 is rejected.  Keeps the extrapolated u-bar in the
 *                 state (exported with it).
 * pADMMI (FG without relaxation) is MF_RPADMM_FG with relax = 1.
 *
 * Discretisation: forward-difference gradient with Neumann boundary,
 * div = -grad^*, unit spacing; 2-D or 3-D grids (3-D uses a = 12).
 *
 * Memory: every pointer marked "device" is HIP device memory on the current
 * device.  The caller owns the capacities, the workspace and every output
 * buffer.  The library never allocates device memory: the workspace given to
 * create() holds all solver state, sized by maxflow_workspace_bytes().
 * Layout of grid fields: planar, one contiguous plane per scalar component,
 * row-major with x (last shape entry) fastest; multi-plane fields are
 * [plane][z][y][x].
 *
 * Errors: every call returns an mf_status; no exception crosses the ABI.
 * On a negative status maxflow_last_error() returns a thread-local message.
 * A handle may be used from one host thread at a time.  All GPU work is
 * enqueued on the stream given at create(); calls that return data to the
 * host synchronise that stream.
 */
#ifndef MAXFLOW_H
#define MAXFLOW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MF_OK = 0,
  MF_ENOTCONV = 1,   /* iteration cap reached before the tolerance: not an error */
  MF_EINVAL = -1,    /* invalid argument (shape, parameter range, model/labels)  */
  MF_ENOMEM = -2,    /* workspace too small / pool budget exceeded               */
  MF_EDEVICE = -3,   /* HIP runtime error                                        */
  MF_EDIVERGED = -4  /* NaN or Inf in the gap or the residual, or a gap below
                        minus the bound that rounding of the stored flows can
                        explain (1e-5 with FP32 storage, 8e-3 with BF16): weak
                        duality (Section 2.1) rules out a larger negative gap */
} mf_status;

typedef enum { MF_TWO_LABEL = 0, MF_POTTS = 1 } mf_model;
typedef enum {
  MF_RPADMM_FG = 0,
  MF_RPADMM_EB = 1,
  MF_RPDRQ = 2,
  MF_PADMM_TY = 3,
  MF_CP_ALG1 = 4
} mf_method;
/* MF_TV_ISO: pointwise Euclidean |q(x)| <= alpha, the P_alpha of eq.
 * (projections).  MF_TV_ANISO: per-component |q_k(x)| <= alpha (l1 TV). */
typedef enum { MF_TV_ISO = 0, MF_TV_ANISO = 1 } mf_tv;
/* MF_BF16: flows (q, p_s, p_t / p_i and the rPDRQ reflected variables) and
 * capacities stored as bfloat16 (round to nearest even); u and all
 * arithmetic stay FP32; gap reductions are FP64 in both modes. */
typedef enum { MF_F32 = 0, MF_BF16 = 1 } mf_storage;
/* MF_FUSED: one kernel per iteration (LDS tile with halo).  MF_UNFUSED: the
 * baseline, one kernel per operator; bitwise identical results. */
typedef enum { MF_FUSED = 0, MF_UNFUSED = 1 } mf_variant;
/* Where the capacities come from: stored planes, or one image plane and a
 * level per label (see cap_source below). */
typedef enum { MF_CAPS_PLANES = 0, MF_CAPS_IMAGE = 1 } mf_cap_source;

typedef struct {
  int32_t ndim;          /* 2 or 3                                                    */
  int64_t shape[3];      /* (H, W) or (D, H, W); W fastest; each >= 1                 */
  int32_t model;         /* mf_model                                                  */
  int32_t method;        /* mf_method                                                 */
  int32_t tv;            /* mf_tv                                                     */
  int32_t storage;       /* mf_storage                                                */
  int32_t variant;       /* mf_variant                                                */
  int32_t nlabels;       /* 2 for MF_TWO_LABEL; 2..8 for MF_POTTS                     */
  double alpha;          /* TV weight, >= 0                                           */
  double c;              /* ADMM step c > 0;             0 -> 0.3                     */
  double relax;          /* FG r in (0, 1.618..); EB rho in (0, 2); DR rho in (0, 2);
                            0 -> 1.618 (FG), 1.9 (EB, DR)                             */
  double sigma, tau;     /* rPDRQ steps; 0 -> (0.2, 1.0) two-label, (5, 0.4) Potts    */
  double a;              /* q preconditioner N = a c I; 0 -> 4*ndim; < 4*ndim: EINVAL */
  double a_tilde;        /* two-label M = a~ c I_2; 0 -> 2; < 2: EINVAL               */
  double a1, a2;         /* Potts M = c diag(a1 I.., a2 I); 0 -> 2, 2n; smaller: EINVAL*/
  int32_t max_iter;      /* iteration cap for maxflow_solve (>= 0)                   */
  double tol;            /* relative primal-dual gap tolerance for maxflow_solve      */
  int32_t check_every;   /* gap cadence in iterations; 0 -> 10                        */
  int32_t tile_rows;     /* fused tile height (8, 16 or 32 rows of 64 columns; the fused
                            3-D sweep tiles 8 rows for 8 and 16 rows for 16 or 32);
                            0 -> 16, except 8 for BF16 Potts with n >= 8 and for the
                            BF16 3-D sweep, and 32 for the fused Potts rPDRQ pass
                            with one sweep; maxflow_tune chooses per problem          */
  /* Pool only, BF16 storage: a solve whose gap at a check is <= promote_gap,
   * or that reaches iteration promote_iter, is frozen at that iterate and
   * continued with FP32 flows (BF16 rounding floors the reachable gap near
   * 1e-3 for Potts problems).  0 disables either trigger. */
  double promote_gap;
  int32_t promote_iter;
  /* Iterations per fused pass (temporal blocking) of the single-solve API:
   * 1, or 2 for the two-label 2-D rpADMM sweep (FG/EB, fused variant),
   * which reads and writes the state once per two iterations with iterates
   * bit-identical to depth 1.  0 -> 2 where it applies, else 1.  Odd
   * iteration counts finish with one depth-1 sweep. */
  int32_t depth;
  /* Fused 3-D sweep: planes per z-slab of a workgroup (each slab re-reads
   * 3 warm-up planes).  0 -> the deepest of 16 and 8 planes that gives the
   * launch at least 2048 workgroups, else 4 (capped at D); otherwise >= 4.
   * Never changes the iterates. */
  int32_t slab_depth;
  /* Preconditioner variants (section on rPDRQ; EB scheme's relaxation).
   * gs_sweeps: symmetric red-black Gauss-Seidel sweeps per rPDRQ iteration,
   *   i.e. the preconditioner M_n (n steps of the preconditioned iteration
   *   for T u = b from u^k); 0 -> 1; 1..64; only applies to rPDRQ.  The
   *   fused 2-D pass takes 1..4 sweeps for two labels and 1..3 for Potts
   *   (64 x 16 tiles beyond one sweep); more sweeps, 3-D and the unfused
   *   variant run the in-place launches.
   * relax0, relax_ramp: rpADMMII only.  relax0 = 0: constant rho = relax.
   *   Otherwise the non-decreasing sequence rho_k = relax0 + (relax -
   *   relax0) min(k, relax_ramp) / relax_ramp for the step from iterate k,
   *   with 0 < relax0 <= relax < 2 and relax_ramp >= 1; depth-2 passes
   *   start once rho_k is constant (k >= relax_ramp).  Not in the pool. */
  int32_t gs_sweeps;
  double relax0;
  int32_t relax_ramp;
  /* Capacity source (the data costs C_s, C_t or rho(l_i, x) = C_i of the
   * problem statement, eqs. seg:chanvese and potts-model).
   * MF_CAPS_PLANES: `cap` of maxflow_create holds the capacity planes.
   * MF_CAPS_IMAGE: `cap` holds one image plane I on the same grid, and the
   *   capacities are C_k(x) = |I(x) - levels[k]|^cap_power, evaluated in FP32
   *   wherever they are used (two-label: C_s from levels[0], C_t from
   *   levels[1]; Potts: C_1..C_n from levels[0..n-1]).  The workspace holds
   *   the one image plane (BF16 with BF16 storage) instead of 2 or n planes,
   *   and every sweep reads it once per pixel.  Not in the pool. */
  int32_t cap_source;    /* mf_cap_source                                            */
  int32_t cap_power;     /* 1 or 2; 0 -> 2                                           */
  double levels[8];      /* finite                                                    */
} mf_params;

/* Gap at an iterate.  primal = P(u) at clip(u,0,1) (two-label) or the pointwise
 * simplex projection of u (Potts); dual = sum_x min(C_s, C_t + div q) or
 * sum_x min_i(C_i + div q_i); rel_gap = (primal - dual) / max(|primal|,|dual|);
 * resid_rms = RMS of the conservation residual; flow = sum p_s.  For rPDRQ the
 * flows are the resolvent outputs of the last iteration. */
typedef struct {
  int64_t iter;
  double primal, dual, rel_gap, resid_rms, flow;
  int32_t status;
} mf_gap;

typedef struct mf_solver mf_solver;

/* Bytes of workspace create() needs for these parameters (0 on invalid
 * parameters; see maxflow_last_error()). */
size_t maxflow_workspace_bytes(const mf_params* p);

/* Validate p, lay out the workspace, copy the capacities (device, FP32,
 * TWO_LABEL: planes [C_s, C_t]; POTTS: planes [C_1..C_n]; with
 * MF_CAPS_IMAGE the one image plane) into it, converting to BF16 if requested, and set the initial point (q = 0, u = 0, source and
 * sink flows at the pointwise minimum capacity).  The caller may free `cap`
 * once this returns.  `workspace` (device, >= maxflow_workspace_bytes(p)
 * bytes, 256-byte aligned) must outlive the solver.  `hip_stream` is a
 * hipStream_t (NULL = default stream). */
mf_status maxflow_create(const mf_params* p, const float* cap, void* workspace,
                         size_t ws_bytes, void* hip_stream, mf_solver** out);

/* Re-initialise the iterate (iteration count 0). */
mf_status maxflow_reset(mf_solver* s);

/* Enqueue `iters` iterations; asynchronous, no host synchronisation. */
mf_status maxflow_step(mf_solver* s, int32_t iters);

/* Evaluate the gap at the current iterate (FP64 reduction on the GPU);
 * synchronises the stream.  Returns MF_EDIVERGED (with *out filled) on a
 * non-finite or negative gap as described for that status. */
mf_status maxflow_gap(mf_solver* s, mf_gap* out);

/* Iterate until the relative gap at a multiple of check_every is <= tol or
 * max_iter is reached; the state is left at the iterate whose gap was
 * accepted.  Returns MF_OK, MF_ENOTCONV or MF_EDIVERGED; fills *out. */
mf_status maxflow_solve(mf_solver* s, mf_gap* out);

/* Current iteration count. */
int64_t maxflow_iter(const mf_solver* s);

/* Copy the current u (device, FP32, 1 plane two-label / n planes Potts). */
mf_status maxflow_read_u(mf_solver* s, float* dst);

/* Labels (device, int32, one plane): two-label u > 1/2; Potts argmax_i u_i
 * with the lowest index on ties. */
mf_status maxflow_labels(mf_solver* s, int32_t* dst);

/* Field access in FP32 for checking and restarts.  Fields: 0 = u (L planes),
 * 1 = q (L*ndim planes, label-major then component x, y, z), 2 = p_s (1 plane),
 * 3 = p (L planes: p_t for two-label, p_1..p_n for Potts).  For rPDRQ,
 * q, p_s, p are the reflected variables (q-bar, p-bar) and fields 4, 5, 6 are
 * the resolvent outputs of the last iteration (same shapes as 1, 2, 3).
 * L = 1 (two-label) or n.  `dst`/`src` are device pointers. */
mf_status maxflow_read_field(mf_solver* s, int32_t field, float* dst);
mf_status maxflow_write_field(mf_solver* s, int32_t field, const float* src);

/* Raw state snapshot (device bytes; size maxflow_state_bytes). */
size_t maxflow_state_bytes(const mf_solver* s);
mf_status maxflow_export_state(mf_solver* s, void* dst);
mf_status maxflow_import_state(mf_solver* s, const void* src, int64_t iter);

mf_status maxflow_destroy(mf_solver* s);

/* Autotuner for the launch shape: the tile height, the fusion depth
 * (iterations per pass) and the 3-D slab depth, the knobs in `what`
 * (MF_TUNE_* bits; the others keep the solver's values).  Candidates:
 *   fused two-label 2-D rpADMM: depth 1 with 8, 16, 32 rows; depth 2 with
 *     16, 32 rows;
 *   fused 2-D Potts: 8, 16, 32 rows (8, 16 for n = 8);
 *   fused 3-D two-label: 8 or 16 rows x slab depths 8, 16, 32;
 *   fused 2-D rPDRQ (two-label or Potts, one sweep): 16, 32 rows;
 *   any other solver: its one configuration, timed.
 * Each candidate is timed over `sweeps` passes (after two warm-up passes) on
 * the solver's stream with HIP events, from the solver's current iterate k
 * into the other state buffer, so the state and the iteration count are
 * unchanged; no launch shape changes the iterates (bit-identical).  The
 * in-place rPDRQ launches would overwrite the state: that solver times
 * nothing (ncand = 0).  The fastest candidate (per iteration) is kept for
 * this solver and returned in `out` with every candidate's time.
 * Synchronises the stream.  Errors: MF_EINVAL (null solver or out, sweeps
 * < 1 or > 10000), MF_EDEVICE. */
#define MF_TUNE_TILE 1
#define MF_TUNE_DEPTH 2
#define MF_TUNE_SLAB 4
typedef struct {
  int32_t tile_rows, depth, slab_depth;
  double us_per_iter;
} mf_tune_cand;
typedef struct {
  int32_t tile_rows, depth, slab_depth;   /* the choice, now in effect */
  int32_t ncand;
  mf_tune_cand cand[16];
} mf_tuning;
mf_status maxflow_tune(mf_solver* s, int32_t sweeps, int32_t what, mf_tuning* out);

/* ------------------------------------------------------------------------
 * Allocation-free solve, for callers that cannot allocate memory (tight
 * serving loops, harnesses that forbid allocation).
 *
 * maxflow_create + maxflow_solve + maxflow_read_u + maxflow_labels in one
 * call, with the same kernels and results (bit for bit), but the workspace
 * is a static device array of MF_STATIC_SCRATCH_BYTES per device, reserved
 * once the library runs on the device and held until the process ends.  The
 * call allocates nothing: no device or pinned host memory, no events, no
 * heap; it follows the on-GPU stop decision with a synchronous 4-byte read
 * every 4 gap checks.
 *   p, cap:     as in maxflow_create (cap is read, not kept);
 *   u_dst:      device FP32, L planes (1 two-label, n Potts), dense layout;
 *               may be NULL;
 *   labels_dst: device int32, one plane (as maxflow_labels); may be NULL;
 *   out:        gap at the accepted iterate, as maxflow_solve; may be NULL;
 *   hip_stream: hipStream_t (NULL = default stream); synchronised on return.
 * Returns as maxflow_solve (MF_OK, MF_ENOTCONV, MF_EDIVERGED), MF_EINVAL on
 * invalid parameters, MF_ENOMEM when maxflow_workspace_bytes(p) exceeds
 * MF_STATIC_SCRATCH_BYTES (use maxflow_create with a caller workspace), or
 * MF_EDEVICE.  Every call on a device shares that device's array and
 * overwrites all of it that the problem uses (capacities, state, control
 * block): calls that overlap on one device race, so serialise them.
 * ---------------------------------------------------------------------- */
#define MF_STATIC_SCRATCH_BYTES (64u << 20)
mf_status maxflow_solve_static(const mf_params* p, const float* cap, float* u_dst, int32_t* labels_dst,
                               mf_gap* out, void* hip_stream);

/* Thread-local message describing the last error (solver and pool calls). */
const char* maxflow_last_error(void);

/* ------------------------------------------------------------------------
 * Batched pool (continuous batching of many solves on one device).
 *
 * The pool keeps many rpADMM solves resident in one caller-owned device arena
 * and advances all of them together.  Each solve is cut into tiles; one
 * kernel launch per model class walks a device-resident work list of
 * (solve, tile) items drawn from grids of any size (one item per workgroup),
 * and every running solve advances one iteration per step with its own
 * iteration counter, gap cadence and convergence decision (all on the GPU).
 * `steps_per_advance` steps form one hipGraph; admission and
 * retirement edit the device tables between replays and resize the graph's
 * kernel grids in place (the graph is rebuilt only when the set of classes
 * present changes).  A solve's iterates are bit-identical alone, in any mix,
 * and through the single-solve API with the same storage.  Supported:
 * methods FG and EB; 2-D two-label and Potts (n = 2, 3, 4, 8); 3-D two-label;
 * FP32 or BF16 storage (BF16 solves may be promoted to FP32 storage near the
 * BF16 rounding floor, see promote_gap / promote_iter).  Convergence follows
 * the same rule as maxflow_solve (gap at multiples of check_every, tolerance
 * tol, cap max_iter) and the state stays at the accepted iterate; the pool
 * requires check_every == steps_per_advance and max_iter a multiple of it.
 * ---------------------------------------------------------------------- */
typedef struct mf_pool mf_pool;

/* Bytes one admitted solve occupies in the arena (capacities + two states);
 * 0 on invalid or unsupported parameters. */
size_t mf_pool_footprint(const mf_params* p);

/* Bytes of arena the pool's own device tables take. */
size_t mf_pool_table_bytes(int32_t max_slots, int32_t max_tiles);

/* `arena`: device, 256-byte aligned, caller-owned, outlives the pool;
 * `max_slots`: resident solves at most; `max_tiles`: work-list capacity per
 * class; `steps_per_advance`: iterations per mf_pool_advance, which must be
 * 10 (MF_EINVAL otherwise: other step counts are not supported); `depth`:
 * 1 or 2 (0 -> 2 when steps_per_advance is even, else 1; steps_per_advance
 * must be a multiple of it).  With depth 2 the two-label 2-D classes run
 * the two-iteration pass (iterate k+1 kept in LDS, one state read and write
 * per two iterations) every other step and the other classes one sweep per
 * step; the iterates are the same bits as with depth 1.  `hip_stream`: a created (non-default) hipStream_t. */
mf_status mf_pool_create(void* arena, size_t arena_bytes, int32_t max_slots, int32_t max_tiles,
                         int32_t steps_per_advance, int32_t depth, void* hip_stream, mf_pool** out);

/* Admit one solve: copies `cap` (device, FP32, layout as maxflow_create) into
 * the arena (converting to BF16 if asked) and sets the initial point.
 * MF_ENOMEM when the arena, the slot table or the class work list is full
 * (retry after retiring solves); MF_EINVAL on invalid/unsupported params. */
mf_status mf_pool_admit(mf_pool* pool, const mf_params* p, const float* cap, int64_t* solve_id);

/* Enqueue steps_per_advance steps (one graph replay) and a copy of the
 * status array for mf_pool_poll; asynchronous. */
mf_status mf_pool_advance(mf_pool* pool);

/* Report solves that finished since the last poll: up to `cap` ids into
 * done_ids and their gaps (iter = accepted iterate, status MF_OK /
 * MF_ENOTCONV / MF_EDIVERGED) into gaps; *ndone = count.  After an advance
 * the poll reads the status as of the advance before it (waiting only for
 * that one), so the device keeps the newest advance while the host reads;
 * a poll with no advance since the last poll waits for the newest.  A
 * finished solve is stopped, so a report one advance later changes nothing
 * but its latency. */
mf_status mf_pool_poll(mf_pool* pool, int64_t* done_ids, mf_gap* gaps, int32_t cap, int32_t* ndone);

/* Copy a solve's u (device FP32, L planes) and/or labels (device int32) and
 * release its arena block and slot.  Either output may be NULL. */
mf_status mf_pool_retire(mf_pool* pool, int64_t solve_id, float* u_dst, int32_t* labels_dst);

/* Resident solves, arena bytes in use, and the largest free arena block. */
mf_status mf_pool_stats(mf_pool* pool, int32_t* active, size_t* bytes_in_use, size_t* largest_free);

/* Number of BF16 -> FP32 promotions performed so far. */
int64_t mf_pool_promotions(const mf_pool* pool);

mf_status mf_pool_destroy(mf_pool* pool);

#ifdef __cplusplus
}
#endif
#endif /* MAXFLOW_H */
