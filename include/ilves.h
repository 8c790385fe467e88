/*
 * ilves.h -- C ABI of the MI355X (gfx950) constraint solver.
 *
 * The library solves the per-timestep constraint equations of constrained
 * molecular dynamics (Supplement section 2.3 of the ILVES paper):
 *
 *   given old positions r, unconstrained positions r_u, masses m and
 *   distance constraints k = (a_k, b_k, d_k), find lambda with
 *
 *     r'(lambda) = r_u - M^{-1} G(r)^T lambda                  (Eq. 6)
 *     g_k(r')   = 1/2 (|r'_a - r'_b|^2 - d_k^2) = 0             (Eq. ecconstr)
 *
 *   by Newton's method on A(x, y) = G(x) M^{-1} G(y)^T           (Eq. defA)
 *     A(r'_l, r) z_l = g(r'_l),  lambda_{l+1} = lambda_l + z_l    (Eq. newton-constraint-equation)
 *   or by the chord method with the constant A(r, r)             (Supplement section 3, ILVES-F)
 *   until max_k |g_k| / d_k^2 <= tol                              (Supplement section 4).
 *
 * Sign convention: g has the opposite sign of the paper's Eq. ecconstr and
 * lambda carries no time step, lambda_here = -h^2 lambda_paper.
 *
 * Every linear system is solved by a sparse LU (Newton) factorisation
 * without pivoting on a fill-reducing ordering and symbolic factorisation
 * that ilves_plan_create computes once from the bond graph (Supplement
 * section 3: line graph L(G) and ordering).
 *
 * Conventions for every entry point:
 *   - positions are structure-of-arrays: x[0..s), y[0..s), z[0..s) back to
 *     back, 3*s doubles, in nm; masses in amu (> 0);
 *   - "device" pointers are HIP device (or managed) memory of the current
 *     device; "host" pointers are ordinary host memory;
 *   - the caller owns every array it passes; the plan owns its own device
 *     buffers and workspace;
 *   - functions return ILVES_OK or an error code and never throw; a message
 *     for the last error of the calling thread is in ilves_last_error().
 */
#ifndef ILVES_H
#define ILVES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ilves_plan* ilves_plan_t;

typedef enum {
  ILVES_OK = 0,
  ILVES_ERR_ARG = 1,            /* bad argument (null pointer, negative size, ...)          */
  ILVES_ERR_TOPOLOGY = 2,       /* self pair, duplicate pair, atom index out of range, d<=0 */
  ILVES_ERR_HIP = 3,            /* a HIP runtime call failed                                */
  ILVES_ERR_NOMEM = 4,          /* host or device allocation failed                         */
  ILVES_ERR_SINGULAR = 5,       /* per molecule: a pivot vanished (redundant constraints)   */
  ILVES_ERR_NOT_CONVERGED = 6,  /* per molecule: iteration cap reached before tol           */
  ILVES_ERR_NONFINITE = 7,      /* per molecule: NaN or Inf met in the residual             */
  ILVES_ERR_UNSUPPORTED = 8,    /* option combination not built into this library           */
  ILVES_ERR_TIMEOUT = 9         /* per molecule: the workgroups of a split molecule did not
                                   meet at a barrier within its wait limit; later solves of
                                   the plan report it too until ilves_plan_reset_barriers  */
} ilves_status_t;

enum { ILVES_PREC_FP64 = 0, ILVES_PREC_MIXED = 1 };
enum { ILVES_VARIANT_NEWTON = 0, ILVES_VARIANT_CHORD = 1 };
enum { ILVES_WARM_ZERO = 0, ILVES_WARM_MLP = 1, ILVES_WARM_CALLER = 2, ILVES_WARM_DECOUPLED = 3 };

typedef struct {
  int32_t precision;     /* ILVES_PREC_FP64: factor and solves in FP64;
                            ILVES_PREC_MIXED: matrix, factor and triangular solves
                            in FP32, residual, lambda and positions in FP64      */
  int32_t variant;       /* ILVES_VARIANT_NEWTON (refactor A(r', r) every
                            iteration) or ILVES_VARIANT_CHORD (factor A(r, r)
                            once per solve)                                      */
  int32_t max_iter;      /* iteration cap; <= 0 selects 20 (Newton FP64) or 40   */
  int32_t warm_start;    /* ILVES_WARM_ZERO: lambda_0 = 0; ILVES_WARM_CALLER:
                            lambda_0 read from the lambda argument;
                            ILVES_WARM_MLP: lambda_0 from the loaded network
                            (see ilves_solve_learned);
                            ILVES_WARM_DECOUPLED: lambda_0 of each constraint
                            from its own quadratic |u_k - lambda C_kk e_k|^2 =
                            d_k^2 (the constraint taken alone, root nearest 0;
                            the Newton step from 0 when there is none),
                            computed in the solve; a molecule restarts from 0
                            when that start is not better than 0 (as for MLP) */
  int32_t block_threads; /* cap on the threads per workgroup of molecules kept in
                            LDS (64..1024); 0 = automatic; molecules that do not
                            fit in LDS always use 512 or 1024                   */
  int32_t lds_limit;     /* bytes of LDS a molecule may use; 0 = auto            */
  int32_t ordering;      /* 0 auto, 1 minimum degree, 2 nested dissection        */
  int32_t split_rows;    /* molecules with more constraints than this are split
                            across several workgroups (block-bordered LU with a
                            Schur complement on the constraints that join the
                            parts); 0 = automatic (4096), < 0 = never          */
  int32_t split_part_rows; /* constraints per part of a split molecule;
                            0 = automatic (about twelve parts of 384 to 1,024
                            constraints, larger while the split exceeds its
                            limits)                                             */
} ilves_options_t;

/* Fills *opt with defaults (FP64 Newton, lambda_0 = 0, automatic schedule).
 * Defined by: Supplement section 2.3 (Newton from lambda_0 = 0). */
void ilves_default_options(ilves_options_t* opt);

/*
 * Builds a plan for a topology: validates it, splits it into molecules
 * (connected components of the constraint graph), builds each molecule's
 * line graph, orders it, computes the symbolic LU factorisation and the
 * level schedule, and uploads everything to the current device.
 *   n_atoms        number of atoms s (> 0)
 *   n_constraints  number of constraints n (>= 0)
 *   pairs          host int32 [n][2], atom indices, a != b, no duplicates
 *   d              host double [n], target distances (nm, > 0)
 *   opt            host options (NULL = defaults)
 *   out            receives the plan handle
 * The topology is copied; the caller may free it afterwards.
 * Defined by: Supplement section 2.2 (constraints g_k, Eq. ecconstr) and
 * section 3 (the graph G of constrained bonds, its line graph L(G) whose
 * adjacency is the pattern of A, the fill-reducing ordering and the
 * initialisation done once before the Newton iterations).
 * Errors: ILVES_ERR_ARG, ILVES_ERR_TOPOLOGY, ILVES_ERR_NOMEM, ILVES_ERR_HIP.
 */
ilves_status_t ilves_plan_create(int32_t n_atoms, int32_t n_constraints, const int32_t* pairs,
                                 const double* d, const ilves_options_t* opt, ilves_plan_t* out);

/* Releases the plan and its device memory.  NULL is accepted.  Errors: none
 * (ILVES_OK).  No defining passage (resource management). */
ilves_status_t ilves_plan_destroy(ilves_plan_t plan);

/* Number of molecules: connected components of G with at least one
 * constraint (Supplement section 3, G is usually disconnected); -1 for a
 * NULL plan. */
int32_t ilves_plan_num_molecules(ilves_plan_t plan);

/*
 * Bound on the polls of a split molecule's barrier wait (the workgroups of
 * a split molecule meet twice per Newton iteration; every wait polls a
 * counter in device memory with a short sleep).  Default 2^22 polls
 * (seconds).  A workgroup whose wait runs out marks the molecule poisoned,
 * which releases every other waiter; the molecule reports ILVES_ERR_TIMEOUT
 * in this and every later solve of the plan.  A small limit forces that
 * path (used to test it).  Takes effect at the next solve enqueued.
 * Defined by: Supplement section 3 (shared and private partitions of L(G),
 * the shared part's Schur complement solved between the partitions' own
 * eliminations); the barrier itself is this library's design.
 * Errors: ILVES_ERR_ARG (NULL plan, polls < 0).
 */
ilves_status_t ilves_plan_set_wait_limit(ilves_plan_t plan, int32_t polls);

/*
 * Clears the barrier state of every split molecule of the plan (arrival
 * count, generation and poisoned flag), so that molecules that reported
 * ILVES_ERR_TIMEOUT solve again.  Synchronises the device first (no solve of
 * any plan may be left in flight; the call waits for all of them) and
 * again after clearing.  The current device must be the plan's.  Host call,
 * not graph-capturable.  Defined by: as ilves_plan_set_wait_limit.
 * Errors: ILVES_ERR_ARG (NULL plan, other device), ILVES_ERR_HIP.
 */
ilves_status_t ilves_plan_reset_barriers(ilves_plan_t plan);

/*
 * Plan statistics, host int64 array of ILVES_STAT_COUNT entries:
 *   [0] molecules, [1] constraints, [2] atoms in constraints,
 *   [3] stored factor entries, [4] fill entries, [5] factor updates,
 *   [6] largest level count, [7] sum of level counts, [8] molecules whose factor fits in
 *   LDS (mixed precision), [9] the others, [10] workspace bytes,
 *   [11] plan bytes on the device, [12] molecules split across workgroups,
 *   [13] workgroups (parts) of the split molecules, [14] largest separator
 *   (constraints joining the parts of one molecule), [15] split molecules
 *   whose parts keep only their factor values in LDS (FP64), [16] split
 *   molecules whose parts keep their factor values and per-row structure in
 *   LDS and read pair tasks and update lists from global memory (mixed
 *   precision), [17] elimination levels of the split molecules' parts whose
 *   items are shared over several lanes (in the factorisation or the
 *   backward substitution: levels with long chains of entries).
 * Defined by: Supplement section 3 (L(G), ordering, fill of the factors).
 * Errors: ILVES_ERR_ARG (NULL plan or stats).
 */
#define ILVES_STAT_COUNT 18
ilves_status_t ilves_plan_stats(ilves_plan_t plan, int64_t* stats);

/*
 * Per-molecule description, host arrays of length num_molecules (any may be
 * NULL): constraint count, atom count, level count, and the first input
 * constraint index of each molecule in the plan's molecule order.
 * Defined by: Supplement section 3 (molecules, levels of the elimination).
 * Errors: ILVES_ERR_ARG (NULL plan).
 */
ilves_status_t ilves_plan_molecules(ilves_plan_t plan, int32_t* n_con, int32_t* n_atoms,
                                    int32_t* n_levels, int32_t* first_constraint);

/*
 * Perturbed inputs for repeated solves (for example a captured HIP graph
 * replayed over many steps): r_u = r + sigma * z, z standard normal, with
 * z drawn from the counter-based generator Philox4x32-10 (Salmon et al.,
 * SC 2011) and the Box-Muller transform.  For atom i and step s = *step:
 * words w = Philox4x32-10(counter {i, 0, s mod 2^32, s / 2^32}, key {seed mod
 * 2^32, seed / 2^32}); u1 = ((w1 2^32 + w0) >> 11 + 1/2) 2^-53, u2 likewise
 * from (w3, w2); z_x = sqrt(-2 ln u1) cos(2 pi u2), z_y = sqrt(-2 ln u1)
 * sin(2 pi u2); z_z is the first normal of the counter {i, 1, ...}.
 * r, r_u: device SoA [3][n_atoms] FP64 (may not alias); step: device
 * uint64, read when the kernel runs.  Asynchronous on hip_stream.
 * Defined by: no passage of the paper (input generation for benchmarks
 * and tests; the generator follows Salmon et al.).
 * Errors: ILVES_ERR_ARG (negative n_atoms or sigma, null pointers),
 * ILVES_ERR_HIP.
 */
ilves_status_t ilves_perturb_normal(const double* r, int32_t n_atoms, double sigma, uint64_t seed,
                                    const uint64_t* step, double* r_u, void* hip_stream);

/* *counter += delta on the device (advances the step of
 * ilves_perturb_normal inside a captured graph).  counter: device uint64.
 * Defined by: no passage (input generation).
 * Errors: ILVES_ERR_ARG (null), ILVES_ERR_HIP. */
ilves_status_t ilves_counter_add(uint64_t* counter, uint64_t delta, void* hip_stream);

/*
 * Leapfrog around the solve (constrained MD; main text, section on the
 * constrained equations of motion, with the constraints solved for the new
 * positions every step).  One step:
 *   ilves_md_kick_drift:  v += h M^-1 f;  r_u = r + h v
 *   ilves_solve(plan, r, r_u, mass, tol, r_new, ...)
 *   ilves_md_finish:      v = (r_new - r) / h;  r = r_new
 * All arrays are device SoA [3][n_atoms] FP64 (mass [n_atoms]); v holds the
 * half-step velocities.  r_u and r_new must not alias r.  Units: nm, ps,
 * amu, forces in amu nm ps^-2.  Asynchronous on hip_stream, graph-capturable.
 * Defined by: Supplement section 2.3, Eqs. nonlinear:1a-1c (the constrained
 * leapfrog whose position step is the constraint solve).
 * Errors: ILVES_ERR_ARG (n_atoms < 0, h not positive, null pointers),
 * ILVES_ERR_HIP.
 */
ilves_status_t ilves_md_kick_drift(const double* r, double* v, const double* f, const double* mass, double h,
                                   int32_t n_atoms, double* r_u, void* hip_stream);
ilves_status_t ilves_md_finish(double* r, const double* r_new, double h, int32_t n_atoms, double* v,
                               void* hip_stream);

/*
 * Launch tuning of a plan (a performance knob; results agree to rounding).
 * band_block[b] is the threads per workgroup of launch band b.  Molecules
 * held wholly in LDS fall in bands 0..3 by their LDS size (<= 8 KB, <= 24 KB,
 * <= 64 KB, larger); molecules with only part (or none) of their data in LDS
 * fall in band 3 up to 4096 constraints and in band 4 above.  The partly-LDS
 * kernels exist with 512 and 1024 threads only; smaller requests round up to
 * 512.  The launch group of the largest molecules held in LDS runs 1024
 * threads whatever its band's entry when its LDS allows one workgroup per
 * CU and no group running beside it fits in the LDS it leaves (unless the
 * plan's block_threads caps it lower).  lds_limit caps the LDS one molecule may use (0 = all of it); lowering
 * it moves molecules out of LDS.  Defined by: no passage (a launch knob of
 * this library; the ordering and factorisation it schedules are those of
 * Supplement section 3).
 */
typedef struct {
  int32_t band_block[5];   /* 64, 128, 256, 512 or 1024 */
  int32_t lds_limit;       /* bytes, 0 = maximum */
  int32_t reserved[2];
} ilves_tuning_t;

/* Current tuning of the plan.  Errors: ILVES_ERR_ARG (NULL plan or t). */
ilves_status_t ilves_plan_get_tuning(ilves_plan_t plan, ilves_tuning_t* t);

/* Re-derives the placement and launch groups of the plan from a tuning
 * (the ordering and symbolic factorisation are kept).  Synchronises the
 * device; no solve on this plan may be in flight, and HIP graphs that
 * captured solves of this plan before the call hold freed addresses and must
 * be captured again.  Errors: ILVES_ERR_ARG, ILVES_ERR_HIP, ILVES_ERR_NOMEM. */
ilves_status_t ilves_plan_tune(ilves_plan_t plan, const ilves_tuning_t* t);

/*
 * One constraint solve (the hot path), asynchronous on hip_stream.
 *   r, r_u     device double [3][n_atoms]  old and unconstrained positions (nm)
 *   mass       device double [n_atoms]     masses (amu, > 0)
 *   tol        bound on max |g_k| / d_k^2 (e.g. 1e-12)
 *   r_out      device double [3][n_atoms]  constrained positions; atoms in no
 *              constraint get r_u.  May alias neither r nor r_u.
 *   lambda     device double [n_constraints] multipliers in input order; read
 *              as lambda_0 when warm_start = ILVES_WARM_CALLER or MLP (not
 *              read for ILVES_WARM_ZERO or ILVES_WARM_DECOUPLED)
 *   iters      device int32 [num_molecules] linear solves per molecule
 *   status     device int32 [num_molecules] ILVES_OK, ILVES_ERR_SINGULAR,
 *              ILVES_ERR_NOT_CONVERGED or ILVES_ERR_NONFINITE per molecule
 *              (ILVES_ERR_TIMEOUT for a split molecule whose barrier wait
 *              hit the plan's wait limit)
 *   hip_stream hipStream_t (NULL = the null stream)
 * The call allocates nothing, never synchronises the host and may be
 * captured in a HIP graph.  One solve per plan may be in flight at a time.
 * The return code reports argument and launch errors only; convergence is
 * reported per molecule in status[] (read it after synchronising).
 * Defined by: Supplement section 2.3 (Eq. 6 position map, Eq. defA Newton
 * matrix, Eqs. newton-constraint-equation update from lambda_0 = 0) and
 * section 4 (stopping rule max_k |g_k| / d_k^2 <= Tol).
 * Errors: ILVES_ERR_ARG (NULL plan or array, tol not positive, other
 * device), ILVES_ERR_HIP (launch failure).
 */
ilves_status_t ilves_solve(ilves_plan_t plan, const double* r, const double* r_u, const double* mass,
                           double tol, double* r_out, double* lambda, int32_t* iters, int32_t* status,
                           void* hip_stream);

/*
 * Velocity constraints (the velocity half of RATTLE): projects velocities v
 * onto the tangent space of the constraints at positions r,
 *   v_out = v - M^{-1} G(r)^T mu   with   G(r) v_out = 0,
 * i.e. A(r, r) mu = G(r) v with A = G M^{-1} G^T -- the linearisation of the
 * position constraints (Eq. defA at r' = r) with the velocity differences of
 * each constraint's atoms in place of the unconstrained bond vectors.  It
 * runs the chord iteration of the solve (one step is exact in FP64; the FP32
 * factor of the mixed precision refines in a second step).
 *   r, v, v_out  device double [3][n_atoms]; atoms in no constraint keep v.
 *                v_out may alias neither r nor v.
 *   mass         device double [n_atoms]
 *   tol          bound on max |e_k . (v_a - v_b)| / (|e_k| |v_a - v_b|)
 *   precision    ILVES_PREC_FP64 or ILVES_PREC_MIXED
 *   mu           device double [n_constraints] multipliers (input order)
 *   iters, status  as for ilves_solve
 * Asynchronous on hip_stream, allocates nothing, graph-capturable; one solve
 * or projection per plan in flight.  Defined by: Supplement section 2 (the
 * velocity constraints G(r) v = 0 that follow from differentiating g along
 * the motion, with the multiplier term of the equations of motion) and
 * Eq. defA at r' = r.  Errors as ilves_solve.
 */
ilves_status_t ilves_project_velocities(ilves_plan_t plan, const double* r, const double* v, const double* mass,
                                        double tol, int32_t precision, double* v_out, double* mu, int32_t* iters,
                                        int32_t* status, void* hip_stream);

/* Same as ilves_solve with explicit precision / variant / warm start /
 * iteration cap, overriding the plan's options for this call, and an
 * optional convergence history:
 *   history      device double [num_molecules][history_len] or NULL; entry
 *                (m, l) receives molecule m's maximum relative violation
 *                max_k |g_k| / d_k^2 at iterate l (before its l-th linear
 *                solve; l = iters[m] is the final one).  Entries past the
 *                molecule's last iterate are left unchanged; after a learned
 *                or decoupled start falls back to lambda_0 = 0 the restart
 *                overwrites the start's entries.  history_len 0 = none.
 * Defined by: as ilves_solve; the chord variant by Supplement section 3
 * (ILVES-F, the constant matrix A(r, r) factored once per solve); the
 * history is the quantity of Supplement section 4's stopping rule, whose
 * decrease shows the convergence order (Supplement section 2.3).
 * Errors as ilves_solve, plus ILVES_ERR_ARG for an unknown precision,
 * variant or warm start, or history_len < 0 or > 0 with a NULL history;
 * ILVES_ERR_UNSUPPORTED for ILVES_WARM_MLP without a loaded network. */
ilves_status_t ilves_solve_ex(ilves_plan_t plan, const double* r, const double* r_u, const double* mass,
                              double tol, int32_t precision, int32_t variant, int32_t warm_start,
                              int32_t max_iter, double* r_out, double* lambda, int32_t* iters,
                              int32_t* status, double* history, int32_t history_len, void* hip_stream);

/*
 * Learned warm start.  A small network predicts lambda_0 for the Newton
 * iteration (whose own start is lambda_0 = 0, Supplement section 2.3) from
 * 16 per-constraint features of the local geometry (see
 * ilves_features).  With w_k = 1/m_a + 1/m_b and t0_k the decoupled
 * (diatomic) solution of constraint k,
 *   lambda_0,k = (t0_k + scale * MLP((f_k - mean) / std)) / w_k,
 * MLP = [16 -> 64 -> 64 -> 1], trained with the exact GELU x Phi(x) and
 * evaluated in BF16 on the matrix cores with FP32 accumulation and the tanh
 * form of GELU (within 4.8e-4 of the exact one).  Parameters are a flat float array
 * of ilves_mlp_param_count() values: W1 [16][64] row-major (input x hidden),
 * b1 [64], W2 [64][64], b2 [64], W3 [64], b3 [1]; the normalisation block
 * has ilves_mlp_norm_count() values: mean [16], std [16] (> 0), scale.
 */
int32_t ilves_mlp_param_count(void);
int32_t ilves_mlp_norm_count(void);

/* Copies network parameters and normalisation (host float arrays of
 * n_params = ilves_mlp_param_count() and n_norm = ilves_mlp_norm_count()
 * values) into the plan and reserves the plan's feature buffers (4 * 17
 * bytes per constraint).  Defined by: no passage (the learned start is not
 * in the paper; it replaces the lambda_0 = 0 of Supplement section 2.3).
 * Errors: ILVES_ERR_ARG (NULL pointer, a count that differs from the
 * library's, a non-finite value, a feature scale not > 0), ILVES_ERR_HIP. */
ilves_status_t ilves_mlp_load(ilves_plan_t plan, const float* params, int32_t n_params, const float* norm,
                              int32_t n_norm);

/* Features of every constraint, in plan row order (ilves_plan_row_constraints
 * maps rows to input constraints): feat device float [n_constraints][16],
 * w device float [n_constraints].  Asynchronous on hip_stream.  Defined by:
 * no passage (learned start); the coupling ratios are entries of Eq. defA.
 * Errors: ILVES_ERR_ARG (NULL argument), ILVES_ERR_HIP. */
ilves_status_t ilves_features(ilves_plan_t plan, const double* r, const double* r_u, const double* mass,
                              float* feat, float* w, void* hip_stream);

/* Host int32 [n_constraints]: input constraint index of each plan row
 * (rows are ordered by elimination level, Supplement section 3).
 * Errors: ILVES_ERR_ARG (NULL argument). */
ilves_status_t ilves_plan_row_constraints(ilves_plan_t plan, int32_t* cid);

/* The network's lambda_0 (device double [n_constraints], input order).
 * Defined by: no passage (learned start).  Errors: ILVES_ERR_ARG (NULL
 * argument), ILVES_ERR_UNSUPPORTED if no network was loaded, ILVES_ERR_HIP. */
ilves_status_t ilves_mlp_predict(ilves_plan_t plan, const double* r, const double* r_u, const double* mass,
                                 double* lambda, void* hip_stream);

/* Solve started from the network's lambda_0, with a per-molecule fallback to
 * lambda_0 = 0 when the prediction's maximum relative violation is not below
 * that of lambda = 0 (or not finite), or when the violation rises in two
 * consecutive iterations.  fallback: device int32 [num_molecules] set to 1
 * where the fallback was taken (may be NULL).  Other arguments as
 * ilves_solve_ex.  Defined by: as ilves_solve, with lambda_0 from the
 * network instead of 0.  Errors as ilves_solve_ex, plus
 * ILVES_ERR_UNSUPPORTED without a loaded network. */
ilves_status_t ilves_solve_learned(ilves_plan_t plan, const double* r, const double* r_u, const double* mass,
                                   double tol, int32_t precision, int32_t variant, int32_t max_iter,
                                   double* r_out, double* lambda, int32_t* iters, int32_t* status,
                                   int32_t* fallback, void* hip_stream);

/* Training kernels (FP32, device arrays, asynchronous on hip_stream;
 * defined by no passage of the paper: the network of the learned start).
 * Forward pass of normalised inputs x [n][16] -> out [n].
 * Errors: ILVES_ERR_ARG (NULL argument, n < 0), ILVES_ERR_HIP. */
ilves_status_t ilves_mlp_forward_f32(const float* params, const float* x, int32_t n, float* out,
                                     void* hip_stream);

/* Floats of workspace ilves_mlp_grad_f32 needs for n samples (0 for n <= 0). */
int64_t ilves_mlp_grad_workspace(int32_t n);

/* Gradient of L = 1/(2n) sum_s (out_s - y_s)^2 with respect to the
 * parameters: grad [param_count], loss [1], work [ilves_mlp_grad_workspace(n)].
 * Partial sums are combined in a fixed order (deterministic).
 * Errors: ILVES_ERR_ARG (NULL argument, n <= 0, work_floats too small),
 * ILVES_ERR_HIP. */
ilves_status_t ilves_mlp_grad_f32(const float* params, const float* x, const float* y, int32_t n, float* grad,
                                  float* loss, float* work, int64_t work_floats, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid allocation): the
 * gradient of ilves_mlp_grad_f32, same kernels and same result, with the
 * per-workgroup partial sums in a fixed device array of the library instead
 * of a caller workspace.  Allocates nothing.  At most
 * ILVES_MLP_GRAD_STATIC_MAX_SAMPLES samples per call (the array holds 192
 * workgroup records of 5,314 floats, 4.1 MB per GPU, kept until the process
 * ends).  Every call on a GPU shares that GPU's array: calls that overlap on
 * one GPU (several streams or host threads at once) race and must be
 * serialised by the caller.  params, x, y, grad, loss as ilves_mlp_grad_f32.
 * Errors: ILVES_ERR_ARG (NULL argument, n <= 0, n above the maximum),
 * ILVES_ERR_HIP.
 */
#define ILVES_MLP_GRAD_STATIC_MAX_SAMPLES 12288
ilves_status_t ilves_mlp_grad_f32_static(const float* params, const float* x, const float* y, int32_t n,
                                         float* grad, float* loss, void* hip_stream);

/* One Adam step (Kingma and Ba) on n parameters, step counting from 1.
 * Errors: ILVES_ERR_ARG (NULL argument, n <= 0, step < 1), ILVES_ERR_HIP. */
ilves_status_t ilves_mlp_adam_f32(float* params, const float* grad, float* m, float* v, int32_t n, float lr,
                                  float beta1, float beta2, float eps, int32_t step, void* hip_stream);

/*
 * Planner diagnostics (host only, no GPU needed; not a solve path -- the
 * solve entry points never call it).  Plans the topology like
 * ilves_plan_create and replays, on the host and in the same order of
 * operations, the level schedule that the device kernel executes, including
 * the block-bordered scheme of molecules split across workgroups (options
 * split_rows / split_part_rows).  Used to test the ordering, symbolic
 * factorisation, task lists and splits on machines without a GPU.
 *   mass [n_atoms], r, r_u, r_out [3][n_atoms], lambda [n_constraints]: host
 *   iters, status: host int32 arrays with room for n_constraints entries
 *   (at least the number of molecules); *n_molecules receives that number
 *   schedule_stats: host int64 [6] (molecules, factor entries, factor updates,
 *   largest level count, fill entries, split molecules) or NULL
 * Defined by: as ilves_plan_create and ilves_solve.
 * Errors: as ilves_plan_create (ILVES_ERR_ARG, ILVES_ERR_TOPOLOGY).
 */
ilves_status_t ilves_plan_replay_host(int32_t n_atoms, int32_t n_constraints, const int32_t* pairs,
                                      const double* d, const ilves_options_t* opt, const double* mass,
                                      const double* r, const double* r_u, double tol, int32_t precision,
                                      int32_t variant, int32_t max_iter, double* r_out, double* lambda,
                                      int32_t* iters, int32_t* status, int32_t* n_molecules,
                                      int64_t* schedule_stats);

/* Static, human readable name of a status code. */
const char* ilves_status_string(ilves_status_t s);

/* Message describing the last error returned on the calling thread. */
const char* ilves_last_error(void);

/* Library version string. */
const char* ilves_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ILVES_H */
