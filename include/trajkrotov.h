/*
 * trajkrotov -- trajectory-parallel Krotov optimisation on one AMD MI355X.
 *
 * C ABI of the library.  It implements, on the GPU, the hot path of
 * Goerz & Jacobs, "Efficient optimization of state preparation in quantum
 * networks using quantum trajectories":
 *
 *   - Monte-Carlo wave-function (quantum jump) trajectories under the
 *     non-Hermitian effective Hamiltonian, with jump times located inside a
 *     time step (Sec. 2.1, the MCWF algorithm and the paragraph after it);
 *   - costates propagated backward from the trajectory functional's boundary
 *     condition (Sec. 2.3);
 *   - the per-time-step cross-trajectory reduction
 *     s_ij = sum_k Im <chi_k(t_j)| H_i |Psi_k(t_j)>  and the sequential,
 *     independent-trajectory Krotov pulse update (Sec. 2.2 "sequential" and
 *     Sec. 2.3, the independent-trajectory update);
 *   - the trajectory functional J_T = 1 - (1/M) sum_k |tau_k|^2 (Sec. 2.3).
 *
 * Problem statement (Sec. 2.1): H(t) = H0 + sum_i u_i(t) H_i with real,
 * piecewise-constant controls u_ij on the intervals (t_j, t_{j+1}] of a grid
 * t_j = j T / nt, and Lindblad operators {L_l}.  The library forms
 *     H_eff = H0 + sum_i u_i H_i - (i/2) sum_l L_l^+ L_l
 * itself (MCWF step 1, with the anti-Hermitian factor -i/2).
 *
 * Conventions (all entry points):
 *   - Every function returns an int status (TK_OK = 0, negative = error) and
 *     never throws across the ABI; tk_last_error() describes the last error.
 *   - All pointer arguments are HOST pointers, except in the *_dev calls,
 *     whose arrays are device pointers (see there).  Inputs are copied during
 *     the call (the caller may free them on return); outputs are
 *     caller-allocated and written before the call returns.  Calls are
 *     synchronous.
 *   - Complex numbers are interleaved (re, im) doubles: a complex vector of
 *     length n is a double array of length 2n.
 *   - Time steps are 0-based: step j is the interval (j dt, (j+1) dt], dt = T/nt.
 *   - One context per host thread; a context owns all of its device memory.
 *   - The sequential Krotov pass is one persistent launch whose blocks wait
 *     for each other every time step; it is launched with
 *     hipLaunchCooperativeKernel (all blocks co-resident or a launch error).
 *     With the environment variable TK_KROTOV_LAUNCH=plain at tk_create the
 *     same grid (sized to fit the device) is launched normally, for tools
 *     that do not handle cooperative launches; a block that waits longer than
 *     a fixed spin limit aborts the pass with TK_EHIP instead of hanging.
 *   - Random numbers: Philox4x64-10 (Salmon et al., SC'11).  Block n of
 *     trajectory k uses counter [n, iteration, direction, 0] and key
 *     [seed, (instance << 32) | k]; word 0 is the norm threshold of waiting
 *     period n, word 1 picks the operator of the jump that ends it; a word w
 *     maps to (w >> 11) * 2^-53.  A trajectory's record therefore does not
 *     depend on M, on the launch configuration or on other trajectories.
 */
#ifndef TRAJKROTOV_H
#define TRAJKROTOV_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define TK_API __attribute__((visibility("default")))
#else
#define TK_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum tk_status {
  TK_OK = 0,
  TK_EINVAL = -1,       /* invalid argument (shape, NULL, NaN, not normalised) */
  TK_EDIM = -2,         /* dimension mismatch between arguments               */
  TK_ENOMEM = -3,       /* device or host allocation failed                   */
  TK_EHIP = -4,         /* HIP runtime error, or a kernel reported a fault     */
  TK_ENOTHERM = -5,     /* H0 or a control Hamiltonian is not Hermitian        */
  TK_ERECCAP = -6,      /* jump-record buffer too small; *n_rec = count needed */
  TK_ENUMERIC = -7,     /* numerical failure (jump with all ||L_l psi|| = 0,
                           step too long for the polynomial propagator)        */
  TK_ESTATE = -8,       /* call order violated (e.g. no system set)           */
  TK_ENODEV = -9,       /* no usable gfx950 device                            */
  TK_EUNSUPPORTED = -10 /* problem shape outside the compiled kernel variants */
};

/* ---- precision of the bulk propagation -------------------------------- */
enum tk_precision {
  TK_FP64 = 0, /* complex128 states and operators                         */
  TK_FP32 = 1  /* complex64 states and operators; norms, jump tests,
                  overlaps and the Krotov reduction stay in FP64           */
};

/* ---- data types --------------------------------------------------------- */

/* Square sparse matrix in CSR form, complex128 values (host memory). */
typedef struct tk_csr {
  int64_t n_rows;          /* = number of columns = Hilbert dimension d     */
  int64_t nnz;
  const int64_t *indptr;   /* [n_rows + 1], indptr[0] = 0, non-decreasing   */
  const int32_t *indices;  /* [nnz] column indices in [0, n_rows)           */
  const double *values;    /* [2 * nnz] interleaved (re, im)                 */
} tk_csr;

/* One quantum jump (MCWF step 4) as recorded by a propagation pass. */
typedef struct tk_jump {
  int32_t instance;   /* optimisation instance (0 for single-system calls) */
  int32_t traj;       /* trajectory index k                                 */
  int32_t step;       /* 0-based time step containing the jump              */
  int32_t op;         /* index l of the jump operator applied               */
  int32_t ordinal;    /* n: jumps of this trajectory earlier in this pass   */
  int32_t direction;  /* 0 forward, 1 backward (costate)                    */
  int32_t iteration;  /* Krotov iteration of the pass                       */
  int32_t reserved;
  double t;           /* jump time                                          */
} tk_jump;

/* Per-kernel timing accumulated since the last tk_reset_timing(). */
typedef struct tk_kernel_timing {
  double ms_total;    /* sum of HIP-event durations of the launches          */
  int64_t launches;
  double flops;       /* algorithmic flops of those launches (see below)    */
  double bytes;       /* algorithmic HBM bytes of those launches            */
  int64_t traj_steps; /* trajectory-steps advanced by those launches        */
} tk_kernel_timing;

enum tk_kernel_kind {
  TK_KERNEL_FORWARD = 0,   /* plain forward pass (iteration 0, functional) */
  TK_KERNEL_BACKWARD = 1,  /* costate pass                                  */
  TK_KERNEL_KROTOV = 2,    /* sequential forward pass with pulse update     */
  TK_KERNEL_GRAD = 3,      /* pathwise gradient (replay + reverse sweep)    */
  TK_KERNEL_CROSS_GRAM = 4, /* Gram matrices of the cross-trajectory update */
  TK_KERNEL_COUNT = 5
};

typedef struct tk_ctx tk_ctx; /* opaque */

/* A HIP stream (the same type as hipStream_t, named here so that this header
 * needs no HIP header). */
struct ihipStream_t;
typedef struct ihipStream_t *tk_stream_t;

/* ---- lifecycle ---------------------------------------------------------- */

/* Create a context on HIP device `device` computing in `precision`.
 * Errors: TK_EINVAL (bad precision), TK_ENODEV (no such device / not gfx950),
 * TK_ENOMEM.  On error *out is NULL. */
TK_API int tk_create(tk_ctx **out, int device, int precision);

/* Free the context and all device memory it owns (NULL is accepted). */
TK_API void tk_destroy(tk_ctx *ctx);

/* Text of the last error on this context (owned by ctx; valid until the next
 * call on it).  Returns a static string for a NULL ctx. */
TK_API const char *tk_last_error(const tk_ctx *ctx);

/* Version string of the library (static storage). */
TK_API const char *tk_version(void);

/* Digest of the sources and flags the library was built from (static
 * storage); the Python binding compares it with the sources beside it and
 * refuses a stale build. */
TK_API const char *tk_build_id(void);

/* ---- problem definition -------------------------------------------------- */

/* Define H0, the n_ctrl control Hamiltonians H_ctrl[i] and the n_jump
 * Lindblad operators L_jump[l] (Sec. 2.1), all d x d.  H0 and each H_ctrl[i]
 * must be Hermitian (max |H - H^+| <= 1e-12 max |H|), else TK_ENOTHERM.
 * Limits: 1 <= d; 0 <= n_ctrl <= 8; 0 <= n_jump <= 8.  Invalidates pulses,
 * states and stored costates.  Errors: TK_EINVAL, TK_EDIM, TK_ENOTHERM,
 * TK_EUNSUPPORTED (no compiled kernel variant fits the sparsity), TK_ENOMEM. */
TK_API int tk_set_system(tk_ctx *ctx, int64_t d, const tk_csr *H0, int32_t n_ctrl,
                  const tk_csr *H_ctrl, int32_t n_jump, const tk_csr *L_jump);

/* Initial state Psi(0) and target Psi_tgt (Sec. 2.1), each [2d].  psi0 must be
 * normalised to 1e-10; the target is normalised by the library (it must be
 * non-zero).  Errors: TK_ESTATE (no system), TK_EINVAL. */
TK_API int tk_set_states(tk_ctx *ctx, const double *psi0, const double *psi_tgt);

/* Pulses: nt steps on [0, T]; u [n_ctrl * nt] row-major (control i, step j at
 * u[i * nt + j]); S [n_ctrl * nt] update shape in [0, 1] (NULL means 1);
 * lambda [n_ctrl] Krotov weights > 0 (NULL means 1) (Sec. 2.2, the extended
 * functional).  Invalidates stored costates and functional values.
 * Errors: TK_ESTATE, TK_EINVAL (nt < 1, T <= 0, non-finite, lambda <= 0). */
TK_API int tk_set_pulses(tk_ctx *ctx, int32_t nt, double T, const double *u,
                  const double *S, const double *lambda);

/* Current pulses (after tk_krotov_iterate they are the optimised ones),
 * u_out [n_ctrl * nt].  Errors: TK_ESTATE. */
TK_API int tk_get_pulses(const tk_ctx *ctx, double *u_out);

/* ---- propagation --------------------------------------------------------- */

/* Forward pass of M trajectories from psi0 with the current pulses
 * (MCWF, Sec. 2.1), random streams (seed, iteration, direction 0).
 * Outputs (each may be NULL): psiT_out [M * 2d] normalised final states;
 * tau_out [2M] overlaps tau_k = <Psi_tgt|Psi_k(T)>; rec [cap] jump records
 * in unspecified order, *n_rec = number of jumps (if larger than cap,
 * returns TK_ERECCAP after writing cap records).  The overlaps are kept in
 * the context as the boundary condition of the next backward pass.
 * Errors: TK_ESTATE, TK_EINVAL (M < 1), TK_ENOMEM, TK_ENUMERIC, TK_EHIP,
 * TK_ERECCAP. */
TK_API int tk_propagate_forward(tk_ctx *ctx, int32_t M, uint64_t seed, uint64_t iteration,
                         double *psiT_out, double *tau_out, tk_jump *rec,
                         int64_t cap, int64_t *n_rec);

/* Backward (costate) pass: each trajectory starts from the normalised target
 * and runs the MCWF rules in reverse time with exp(+i H_eff^+ tau) and an
 * independent stream (seed, iteration, direction 1).  The costate stored for
 * time t_j is chi_k(t_j) = tau_k chi_hat_k(t_j) (Sec. 2.3: boundary condition
 * chi_k(T) = tau_k Psi_tgt), j = 0 .. nt-1, kept in device memory
 * ([nt][M][d], bulk precision) for tk_get_costate and the next Krotov pass.
 * tau [2M]: overlaps from the previous forward pass; NULL uses the ones kept
 * by the last forward pass (same M).  Records as in tk_propagate_forward.
 * Errors: TK_ESTATE, TK_EINVAL, TK_ENOMEM, TK_ENUMERIC, TK_EHIP, TK_ERECCAP. */
TK_API int tk_propagate_backward(tk_ctx *ctx, int32_t M, uint64_t seed, uint64_t iteration,
                          const double *tau, tk_jump *rec, int64_t cap,
                          int64_t *n_rec);

/* Copy the stored costates at time t_j, chi_out [M * 2d] (complex128).
 * Errors: TK_ESTATE (no costates stored), TK_EINVAL (j out of range). */
TK_API int tk_get_costate(const tk_ctx *ctx, int32_t j, double *chi_out);

/* Trajectory functional J_T = 1 - (1/M) sum_k |tau_k|^2 (Sec. 2.3) of the
 * current pulses: one forward pass (seed, iteration).  tau_out [2M] may be
 * NULL.  Errors: as tk_propagate_forward. */
TK_API int tk_functional(tk_ctx *ctx, int32_t M, uint64_t seed, uint64_t iteration,
                  double *J_T, double *tau_out);

/* ---- optimisation -------------------------------------------------------- */

/* Krotov iterations (Sec. 2.2 and 2.3).  With first_iteration = 0, runs the
 * guess forward pass (iteration 0) and writes J_T_out[0], then iterations
 * 1..n_iter into J_T_out[1..n_iter] (n_iter + 1 values).  With
 * first_iteration = n0 >= 1, continues from the overlaps kept by the forward
 * pass of iteration n0-1 (same M and seed, else TK_ESTATE) and writes n_iter
 * values for iterations n0 .. n0+n_iter-1.  Iteration n = backward pass with
 * u^(n-1) (stream iteration n, direction 1), then the sequential forward pass
 * (iteration n, direction 0) which, at every step j, reduces
 *   s_ij = sum_k Im <chi_k(t_j)| H_i |Psi_hat_k(t_j)>   (FP64, fixed order)
 * and sets u_ij = u_ij + S_ij s_ij / (lambda_i M) before propagating step j.
 * The context's pulses are updated in place.  Records of all passes go to
 * rec (may be NULL).  Errors: as the propagation calls. */
TK_API int tk_krotov_iterate(tk_ctx *ctx, int32_t M, uint64_t seed, uint64_t first_iteration,
                      int32_t n_iter, double *J_T_out, tk_jump *rec, int64_t cap,
                      int64_t *n_rec);

/* Krotov iterations with the cross-trajectory update (Sec. 2.3, eq.
 * cross_traj_update), otherwise as tk_krotov_iterate: iteration n runs the
 * backward trajectories xi_k from xi_k(T) = Psi_tgt (normalised, stream
 * iteration n, direction 1; no overlap weight), then the sequential forward
 * pass, which at every step j sets
 *   u_ij = u_ij + S_ij / (M^2 lambda_i)
 *          sum_{k,k'} Im[<xi_k|H_i|Psi_hat_k'> <Psi_hat_k'|xi_k>]   (t_j).
 * The double sum is evaluated as M sum_k' Im <P_j Psi_hat_k'|H_i|Psi_hat_k'>
 * with P_j = (1/M) sum_k |xi_k(t_j)><xi_k(t_j)|, formed on the matrix cores
 * after the backward pass (FP64).  One-wave kernel shapes only (d <= 256; in
 * FP64 d <= 128): TK_EUNSUPPORTED otherwise.  Errors: as tk_krotov_iterate. */
TK_API int tk_krotov_iterate_cross(tk_ctx *ctx, int32_t M, uint64_t seed,
                                   uint64_t first_iteration, int32_t n_iter, double *J_T_out,
                                   tk_jump *rec, int64_t cap, int64_t *n_rec);

/* ---- pathwise gradient ------------------------------------------------------ */

/* Gradient of the trajectory functional with the jump record held fixed.
 * Every trajectory k < M is replayed from psi0 with the current pulses: a
 * forward record (direction 0) of trajectory k at time t in step j ends a
 * propagator piece there, applies L_op and renormalises (MCWF step 4), in the
 * order of the records' ordinals; no thresholds are drawn.  This makes
 *   J_T(u) = 1 - (1/M) sum_k |<Psi_tgt|phi_hat_k(T)>|^2      (Sec. 2.3)
 * a smooth function of the pulse values, and the call returns J_T, the
 * overlaps tau_k of the replay (tau_out [2M], may be NULL) and
 * dJdu [n_ctrl * nt] = dJ_T/du_ij (control i, step j at dJdu[i * nt + j]).
 * The derivative is exact up to the propagators' truncation: each piece's
 * d exp(-i H_eff tau)/du_i comes from an augmented Taylor series (the block
 * exponential of Van Loan, 1978) and the sweep runs backward from the seed
 * dF_k/d<phi_k| with L_l^+ and exp(+i H_eff^+ tau); forward states are
 * checkpointed every 64 steps and recomputed.  The renormalisation after a
 * jump is held constant (it does not change phi_hat_k(T)).
 * rec [n_rec]: jump records as written by tk_propagate_forward (any order;
 * backward records are ignored).  A record with traj >= M, a step outside
 * [0, nt), an operator >= n_jump, a time outside its step (beyond 1e-9 dt)
 * or out of time order within its trajectory gives TK_EINVAL.  Seeds and
 * iterations play no part.  Invalidates the overlaps kept for a following
 * backward pass.  Errors: TK_ESTATE, TK_EINVAL, TK_ENOMEM, TK_ENUMERIC (a
 * recorded jump with ||L_l psi|| = 0), TK_EHIP, TK_EUNSUPPORTED. */
TK_API int tk_grad_pathwise(tk_ctx *ctx, int32_t M, const tk_jump *rec, int64_t n_rec,
                     double *J_T, double *tau_out, double *dJdu);

/* ---- device-pointer variants ---------------------------------------------- */

/* The calls below take DEVICE pointers (memory of the context's device, e.g.
 * torch tensors) for their array arguments and a HIP stream (NULL: the
 * device's null stream).  The context's work is ordered after everything already queued on
 * `stream`, and `stream` is ordered after the context's work when the call
 * returns, so a producer or consumer of the arrays on that stream needs no
 * synchronisation of its own; the calls still return when the host-side
 * checks of the pass (kernel error flags) are done.  Arguments, layouts and
 * errors are those of the host-pointer call named; device arrays are read
 * during the call and may be reused once `stream` has passed the call. */

/* tk_set_pulses with device u [n_ctrl * nt], S [n_ctrl * nt] (NULL: 1) and
 * lambda [n_ctrl] (NULL: 1) (Sec. 2.2, the extended functional).  The
 * context copies them device to device and also reads them back once, to
 * plan each step's polynomial order and substeps on the host and to check
 * them (non-finite u, S outside [0, 1], lambda <= 0 give TK_EINVAL). */
TK_API int tk_set_pulses_dev(tk_ctx *ctx, int32_t nt, double T, const double *u,
                             const double *S, const double *lambda, tk_stream_t stream);

/* tk_get_pulses into device memory u_out [n_ctrl * nt]. */
TK_API int tk_get_pulses_dev(const tk_ctx *ctx, double *u_out, tk_stream_t stream);

/* tk_functional (Sec. 2.3, trajectory functional) with J_T [1] and tau_out
 * [2M] (may be NULL) in device memory. */
TK_API int tk_functional_dev(tk_ctx *ctx, int32_t M, uint64_t seed, uint64_t iteration,
                             double *J_T, double *tau_out, tk_stream_t stream);

/* tk_krotov_iterate (Sec. 2.2 sequential update, Sec. 2.3 independent-
 * trajectory update) with the J_T values in device memory J_T_out (n_iter + 1
 * values when first_iteration = 0, else n_iter); no jump records. */
TK_API int tk_krotov_iterate_dev(tk_ctx *ctx, int32_t M, uint64_t seed, uint64_t first_iteration,
                                 int32_t n_iter, double *J_T_out, tk_stream_t stream);

/* tk_grad_pathwise (gradient of the Sec. 2.3 functional along a fixed jump
 * record) with J_T [1], tau_out [2M] (may be NULL) and dJdu [n_ctrl * nt] in
 * device memory; the jump records `rec` [n_rec] stay in HOST memory (as
 * tk_propagate_forward writes them). */
TK_API int tk_grad_pathwise_dev(tk_ctx *ctx, int32_t M, const tk_jump *rec, int64_t n_rec,
                                double *J_T, double *tau_out, double *dJdu, tk_stream_t stream);

/* ---- entry point that allocates nothing --------------------------------------- */

/* tk_functional_dev for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): it calls no hipMalloc, hipFree or other allocating routine.
 * The pass's error bits, record counter and the overlaps tau_k live in a fixed
 * device array of 1 MiB per device (set up when a context is first created on
 * the device, held until the process ends), so M is at most 65504
 * (TK_EINVAL beyond).  No jump records and no final states are produced.
 * J_T [1] and tau_out [2M] (may be NULL) are device pointers; stream as in the
 * *_dev calls.  The context's system, states and pulses must be set (those
 * calls do allocate).  Every call on a device shares that device's array and
 * leaves its contents behind: calls that overlap on one device (from several
 * host threads or contexts) race.  Errors: TK_ESTATE, TK_EINVAL, TK_ENUMERIC,
 * TK_EHIP, TK_EUNSUPPORTED. */
TK_API int tk_functional_dev_noalloc(tk_ctx *ctx, int32_t M, uint64_t seed, uint64_t iteration,
                                     double *J_T, double *tau_out, tk_stream_t stream);

/* ---- batched form: many optimisation instances at once --------------------- */

/* A batch holds independent optimisation instances -- each a full problem as
 * set by tk_set_system / tk_set_states / tk_set_pulses, with its own M and
 * seed -- and advances all of them together: per kernel shape, one launch
 * runs the costate passes of the shape's instances and one persistent launch
 * runs their sequential Krotov passes side by side (each instance with its
 * own per-step reduction; the shapes' launches follow each other), and one
 * iteration of every instance is replayed as a HIP graph.  Instances
 * may differ in Hilbert dimension, sparsity, M and nt.  Instances whose shape
 * needs several waves per trajectory (d = 216 in FP64, d = 1296 in FP32) run
 * in launches of their own, one team per block, and keep the costates of 64
 * steps at a time: their Krotov pass recomputes each segment from checkpoints
 * of the backward pass (same values, far less memory).  The instance id is
 * part of the random streams' key ([seed, (id << 32) | k], Sec. 2.1 MCWF
 * random numbers), so an instance's trajectories do not depend on the other
 * instances.  The per-step reduction of an instance sums the trajectories'
 * FP64 shares in one fixed order, independent of the tile shapes: results are
 * bit-identical whatever the autotuner picks and whatever else is in the
 * batch (they may differ from tk_krotov_iterate in the last bits, whose
 * reduction order follows its launch shape). */
typedef struct tk_batch tk_batch; /* opaque */

typedef struct tk_batch_info {
  int32_t n_instances;
  int32_t pass_waves_per_block;    /* plain (costate / guess) passes         */
  int32_t pass_blocks;             /* summed over the one-wave shapes       */
  int32_t krotov_waves_per_block;  /* persistent Krotov launches            */
  int32_t krotov_blocks;           /* summed over the one-wave shapes       */
  int32_t autotuned;               /* 1 once the tile shapes are chosen      */
  double last_iteration_ms;        /* last replayed iteration (HIP events)  */
  double tuned_pass_ms;            /* best costate pass seen by the tuner   */
  double tuned_krotov_ms;          /* best Krotov pass seen by the tuner    */
  int64_t traj_steps_per_iteration; /* sum over instances of 2 M nt         */
  int32_t multiwave_instances;     /* instances of multi-wave shapes (one   */
  int32_t multiwave_krotov_blocks; /* team a block, costate segments)      */
  double tuned_multiwave_krotov_ms; /* their Krotov pass at the chosen split */
} tk_batch_info;

/* Create an empty batch on `device` in `precision` (as tk_create). */
TK_API int tk_batch_create(tk_batch **out, int device, int precision);
TK_API void tk_batch_destroy(tk_batch *batch);
TK_API const char *tk_batch_last_error(const tk_batch *batch);

/* Add an instance: the arguments of tk_set_system, tk_set_states and
 * tk_set_pulses, its trajectory count M and seed, and a distinct instance id
 * for the random streams.  *index_out receives its position in the batch.
 * Only before the first tk_batch_krotov_iterate.  Errors: as those calls,
 * TK_EINVAL (duplicate id, M < 1), TK_ESTATE, TK_EUNSUPPORTED. */
TK_API int tk_batch_add(tk_batch *batch, uint32_t instance_id, int64_t d, const tk_csr *H0,
                 int32_t n_ctrl, const tk_csr *H_ctrl, int32_t n_jump, const tk_csr *L_jump,
                 const double *psi0, const double *psi_tgt, int32_t nt, double T,
                 const double *u, const double *S, const double *lambda, int32_t M,
                 uint64_t seed, int32_t *index_out);

/* Krotov iterations of every instance, as tk_krotov_iterate: first_iteration
 * 0 runs the guess passes (iteration 0) and iterations 1..n_iter, writing
 * n_iter + 1 values per instance; first_iteration = n0 continues the previous
 * call (n0 must be the next iteration) and writes n_iter values.  J_T_out is
 * [n_instances][n_out] (row per instance); n_out <= 64.  The first iteration
 * runs pass by pass while an autotuner times candidate tile shapes (waves per
 * block, blocks per instance); later iterations replay a captured graph.
 * Errors: TK_ESTATE (no instances, wrong first_iteration), TK_EINVAL,
 * TK_ENOMEM, TK_EHIP, TK_ENUMERIC, TK_EUNSUPPORTED. */
TK_API int tk_batch_krotov_iterate(tk_batch *batch, uint64_t first_iteration, int32_t n_iter,
                            double *J_T_out);

/* Current pulses of instance `index`, u_out [n_ctrl * nt]. */
TK_API int tk_batch_get_pulses(tk_batch *batch, int32_t index, double *u_out);

/* Launch shapes and timings of the batch. */
TK_API int tk_batch_get_info(const tk_batch *batch, tk_batch_info *out);

/* ---- density-matrix optimisation (Sec. 2.2) ------------------------------------ */

/* Density-matrix functional of the current pulses (Sec. 2.2, eq. functional):
 * rho(0) = |psi0><psi0| propagated with the Lindblad master equation of
 * Sec. 2.1, d rho/dt = -i (H_eff rho - rho H_eff^+) + sum_l L_l rho L_l^+, and
 * J_T = 1 - <<rho(T)|P_tgt>> = 1 - <tgt|rho(T)|tgt>: the physical error of
 * the pulses, free of trajectory noise.  FP64 whatever the context's
 * precision.  Errors: TK_ESTATE, TK_EINVAL, TK_ENUMERIC, TK_EHIP, TK_ENOMEM. */
TK_API int tk_density_functional(tk_ctx *ctx, double *J_T);

/* Krotov's method on the density matrix (Sec. 2.2): J_T_out[0] is the
 * functional of the current pulses; each of the n_iter iterations propagates
 * P backward from P(T) = P_tgt with the adjoint Lindbladian (eqs. bwprop,
 * krotov_boundary), stores P(t_j), then propagates rho forward with the
 * sequential update of every interval j (left point t_j, eq. krotovupdate
 * with dL/du_i = [H_i, rho] as printed):
 *   u_ij = u_ij + S_ij / lambda_i Im <<P(t_j)| [H_i, rho(t_j)]>>,
 * and writes J_T_out[n] (n_iter + 1 values).  The context's pulses become the
 * optimised ones.  Memory: nt d^2 complex128 for P.  Errors: as
 * tk_density_functional. */
TK_API int tk_density_krotov_iterate(tk_ctx *ctx, int32_t n_iter, double *J_T_out);

/* ---- pulse noise (Sec. 3.4) -------------------------------------------------- */

/* Noise measure of pulses (Sec. 3.4, eq. noise):
 *   nu_i = int_0^T |Omega_i(t) - Omega_i^smooth(t)| dt = dt sum_j |u_ij - s_ij|
 * for piecewise-constant pulses, where s_i is the Savitzky-Golay smoothing
 * with a five-point cubic convolute (value at a sample = the least-squares
 * cubic of a five-sample window at that sample; the centred window inside,
 * the first / last five samples for the first / last two).  u: host
 * [n_ctrl * nt] row-major, or NULL for the context's current pulses (then
 * n_ctrl, nt and T are the context's and the arguments are ignored).
 * nu_out [n_ctrl] (host).  Errors: TK_ESTATE (no pulses), TK_EINVAL (n_ctrl
 * outside [1, 8], nt < 5, T <= 0, non-finite u). */
TK_API int tk_pulse_noise(tk_ctx *ctx, int32_t n_ctrl, int32_t nt, double T, const double *u,
                          double *nu_out);

/* ---- the step on the matrix cores versus the sparse step --------------------- */

enum tk_step_method {
  TK_STEP_SPARSE = 0,     /* the passes' series on the packed per-lane slots */
  TK_STEP_DENSE_MFMA = 1  /* dense H_eff times 16-trajectory column tiles on the
                             matrix cores (FP64 or FP32 MFMA) */
};

/* One step propagator of the passes, the K-term Taylor polynomial
 *   y_k = sum_{n=0..K} (-i dt H_eff(u_0))^n / n! x_k,   k < M,
 * (the matrix-vector products that Sec. 2.3 names the fundamental operation;
 * u_0 = the current pulses of the first interval, dt = T / nt) with the given
 * method, `reps` times after one warm-up launch; *ms_per_launch = mean HIP-event
 * time of a launch.  x [M * 2d] host states (any norm); y [M * 2d] (host, may be
 * NULL) the result of the last launch.  It exists to measure whether a dense
 * operator on the matrix cores beats the sparse product; the passes use the
 * sparse one.  Dense: d <= 256; sparse: one-wave shapes (TK_EUNSUPPORTED
 * otherwise).  Errors: TK_ESTATE, TK_EINVAL, TK_EUNSUPPORTED, TK_ENOMEM,
 * TK_EHIP. */
TK_API int tk_step_bench(tk_ctx *ctx, int32_t method, int32_t M, int32_t K, const double *x,
                         double *y, int32_t reps, double *ms_per_launch);

/* ---- instrumentation ------------------------------------------------------ */

/* Enable (1) or disable (0) HIP-event timing of every kernel launch. */
TK_API int tk_set_timing(tk_ctx *ctx, int enable);

/* Accumulated timing of kernel kind `kind` (tk_kernel_kind).  flops and bytes
 * are algorithmic: per trajectory-step 8 K nnz + 8 K d + 4 d real flops
 * (K Taylor terms of the step, nnz stored non-zeros of H_eff) and the costate
 * bytes the method must move (written once backward, read once forward). */
TK_API int tk_get_timing(const tk_ctx *ctx, int kind, tk_kernel_timing *out);
TK_API int tk_reset_timing(tk_ctx *ctx);

/* Description of the kernel variant selected for the current system (static
 * string per variant, e.g. "fp64 R=2 WS=4 NC=2"), and the launch shape of the
 * last Krotov pass: waves per block, trajectories per wave, blocks. */
TK_API int tk_get_launch_info(const tk_ctx *ctx, const char **variant, int32_t *waves_per_block,
                       int32_t *traj_per_wave, int32_t *blocks);

#ifdef __cplusplus
}
#endif

#endif /* TRAJKROTOV_H */
