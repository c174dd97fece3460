/*
 * qpa.h -- C ABI of the replica-batched Parallel Annealing (PA) engine for AMD MI355X.
 *
 * The engine minimises a QUBO objective E(x) = x^T Q x + c^T x over x in {0,1}^n
 * (symmetric Q; Sec. II, eq. (1) in symmetric-matrix form) or an Ising objective
 * H(s) = sum_{i<j} J_ij s_i s_j + sum_i b_i s_i over s in {-1,+1}^n (Sec. II, eq. (2))
 * with the Parallel Annealing dynamics of App. B of arXiv 2501.19221, run on R
 * independent replicas:
 *
 *   s_t   = sign(x_t)                       (sign(0) = +1)
 *   g_t   = lambda_t x_t + (J s_t + b)      (target part on binarised spins)
 *   m_t+1 = alpha m_t - eta g_t             (momentum)
 *   x_t+1 = clip(x_t + m_t+1, -1, 1)        (clipping)
 *
 * every operation rounded to FP32 separately in the order written.  A QUBO is first
 * mapped to Ising form with x = (1+s)/2 (App. A): J = Q without its diagonal,
 * b = Q 1 + c, and 2 E(x) = H(s) + K with K = (1/2) 1^T Q 1 + (1/2) tr Q + 1^T c; the
 * dynamics run on that (J, b).  The initial state is x_0[r][i] = sigma0 * (2u - 1) with
 * u the top 24 bits of the (r*n + i + 1)-th output of SplitMix64(seed), scaled by 2^-24;
 * m_0 = 0.  The default schedule is lambda_t = lambda0 * (1 - t/T) (App. B asks for a
 * gradual decrease to zero).  After T steps every replica's final spins sign(x_T) are
 * scored exactly (int64 for integer couplings, FP64 for float couplings) and the lowest
 * replica index attaining the minimum is reported.
 *
 * Conventions for every entry point:
 *  - Buffers marked "device" are HIP device pointers on the context's device; buffers
 *    marked "host" are ordinary host memory read during the call only.  The caller owns
 *    every buffer (inputs, outputs, workspace).  The library never frees caller memory
 *    and keeps no pointer to it after the call returns.
 *  - Work is enqueued on `stream` (a hipStream_t, NULL = default stream).  An entry point
 *    synchronises that stream once, after validating its inputs on the device, so that
 *    it can report invalid input through its return value; the remaining work is
 *    asynchronous, and outputs are ready when the stream is.
 *  - Errors: every entry point returns a qpa_status; QPA_OK is 0.  A human-readable
 *    message for the last failure on a context is returned by qpa_last_error().  No C++
 *    exception crosses this interface.  A context is not thread-safe: use one per host
 *    thread.  Calls that share a workspace must not overlap.
 */
#ifndef QPA_H
#define QPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QPA_OK = 0,
    QPA_E_ARG = 1,          /* null pointer, negative size, unknown enum value        */
    QPA_E_SHAPE = 2,        /* inconsistent sizes (CSR row pointers, n, nnz)          */
    QPA_E_ASYM = 3,         /* couplings not symmetric, or Ising diagonal not zero    */
    QPA_E_RANGE = 4,        /* integer row sum max_i sum_j |J_ij| + |b_i| >= 2^24:    */
                            /* FP32 fields would no longer be exact                   */
    QPA_E_WORKSPACE = 5,    /* workspace smaller than qpa_workspace_size()            */
    QPA_E_DEVICE = 6,       /* a HIP call failed                                      */
    QPA_E_UNSUPPORTED = 7   /* valid request outside what this library implements     */
} qpa_status;

typedef enum { QPA_KIND_QUBO = 0, QPA_KIND_ISING = 1 } qpa_kind;
typedef enum { QPA_FMT_DENSE = 0, QPA_FMT_CSR = 1 } qpa_format;
typedef enum { QPA_I8 = 0, QPA_I16 = 1, QPA_I32 = 2, QPA_F32 = 3 } qpa_dtype;

/* Field arithmetic of the dense path.  QPA_PREC_FP32: couplings stored and multiplied
 * in FP32.  QPA_PREC_BF16: couplings stored as bf16(J / 2^e) (round to nearest even,
 * e the smallest integer with max|J| <= 2^e) on the matrix cores with FP32
 * accumulation, the sum scaled back by 2^e; spins are exact in BF16.  Integer
 * couplings with |J| <= 256 are exact in BF16, so both settings give identical
 * trajectories for them.  CSR problems always use exact FP32 (or integer) sums. */
typedef enum { QPA_PREC_FP32 = 0, QPA_PREC_BF16 = 1 } qpa_precision;

/* One problem instance.  All array pointers are device pointers.
 *  dense  : n*n couplings, row-major, symmetric, dtype `coupling_dtype`.
 *           QUBO: Q (any diagonal, folded into b).  Ising: J (diagonal must be 0).
 *  CSR    : row_ptr[n+1] (int32, row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz),
 *           col[nnz] (dtype `index_dtype`: QPA_I32 or QPA_I16, each in [0, n)),
 *           weights[nnz] (dtype `coupling_dtype`).  Both (i,j) and (j,i) are stored
 *           with equal weights.  QUBO: entries (i,i) allowed.  Ising: none allowed.
 *  linear : n entries of dtype `linear_dtype`; c (QUBO) or b (Ising); NULL = zeros. */
typedef struct {
    int64_t n;
    int32_t kind;               /* qpa_kind   */
    int32_t format;             /* qpa_format */
    int32_t coupling_dtype;     /* qpa_dtype  */
    int32_t index_dtype;        /* qpa_dtype, CSR only: QPA_I32 or QPA_I16 */
    int32_t linear_dtype;       /* qpa_dtype  */
    int32_t reserved0;
    const void *dense;
    int64_t nnz;
    const int32_t *row_ptr;
    const void *col;
    const void *weights;
    const void *linear;
} qpa_problem;

/* Dynamics parameters (App. B).  lambda_table (host, `steps` floats) overrides the
 * default linear schedule when not NULL. */
typedef struct {
    int32_t replicas;           /* R >= 1                                       */
    int32_t steps;              /* T >= 0                                       */
    float eta;                  /* gradient step ("time step")                  */
    float alpha;                /* momentum coefficient                         */
    float lambda0;              /* initial weight of the quadratic H_initial    */
    float sigma0;               /* amplitude of the initial analog spins        */
    const float *lambda_table;  /* host, optional                               */
    uint64_t seed;              /* SplitMix64 seed of the initial state          */
    int32_t precision;          /* qpa_precision (dense path)                   */
    int32_t flags;              /* single solves: 0, QPA_SOLVE_STREAMED or
                                   QPA_SOLVE_BINNED, and/or QPA_SOLVE_GRAPH;
                                   qpa_solve_batch: 0 or one qpa_batch_flags value */
} qpa_params;

/* qpa_solve / qpa_steps: run a sparse instance with the per-step streamed kernel even
 * when its state fits on chip (the default then keeps it resident for all steps).  Both
 * kernels give the same bits. */
#define QPA_SOLVE_STREAMED 4
/* qpa_solve / qpa_steps / qpa_sbm_solve / qpa_sbm_steps (may be or-ed with
 * QPA_SOLVE_STREAMED): launch a step loop that takes one kernel per step as a HIP graph.
 * The graph is captured on a private stream of the context the first time a call's
 * launch sequence is seen (same problem arrays, workspace, sizes and step range) and
 * replayed afterwards; a context keeps the 8 most recent graphs.  Results are identical
 * to the plain launches.  Paths that run all steps in one launch ignore the flag. */
#define QPA_SOLVE_GRAPH 8
/* qpa_solve / qpa_steps: run a sparse instance with the binned step (two streaming
 * passes per step over an entry order built at the start of the call: the spin bits of
 * every coupling's column gathered chunk by chunk from LDS, then the fields summed bin
 * by bin in LDS and the update fused).  Applies to CSR problems with int8 or int16
 * couplings, integer fields and at most 8 replicas; other problems fail with
 * QPA_E_UNSUPPORTED.  Without a flag such instances take it when their spin words
 * (n x replicas rounded up to a power of two, one bit each) exceed 4 MiB, where the
 * per-row gather of the streamed kernel misses the cache on nearly every coupling.  The
 * bits equal the streamed kernel's (integer sums are exact in any order).  Excludes
 * QPA_SOLVE_STREAMED. */
#define QPA_SOLVE_BINNED 16

/* Path choice of qpa_solve_batch (params.flags, optionally or-ed with QPA_SOLVE_GRAPH:
 * the per-step loop of the dense tiles is then captured once as a HIP graph and replayed,
 * as for qpa_solve; qpa_solve requires neither value).  By default
 * every instance whose couplings are exact in BF16 (integer weights with |w| <= 256,
 * or any weights when precision is QPA_PREC_BF16) runs as dense matrix-core tiles when
 * a cost model finds that cheaper than the sparse kernel; the others run sparse. */
typedef enum {
    QPA_BATCH_SPARSE = 1,       /* every instance on the sparse task kernel      */
    QPA_BATCH_DENSE = 2         /* every BF16-exact instance as dense tiles      */
} qpa_batch_flags;

/* Outputs of a solve.  Every pointer is a device pointer and may be NULL except
 * `energy` and `best`.
 *  spins      [R*n] int8, final sign(x_T) of each replica, row-major by replica.
 *  energy     [R] double: the instance's own objective of those spins (E(x) for a
 *             QUBO with x = (1+s)/2, H(s) for Ising), exact for integer couplings,
 *             FP64-accumulated for float couplings.
 *  energy_i64 [R] int64: the same energies as exact integers (integer couplings only;
 *             left untouched for float couplings).
 *  best       [1] int32: lowest replica index attaining the minimum energy.
 *  x, m       [R*n] float: final analog spins and momenta. */
typedef struct {
    int8_t *spins;
    double *energy;
    int64_t *energy_i64;
    int32_t *best;
    float *x;
    float *m;
} qpa_outputs;

typedef struct qpa_ctx qpa_ctx;

/* Create a context bound to HIP device `device` (0-based).  *out receives the handle. */
qpa_status qpa_create(qpa_ctx **out, int device);

/* Destroy a context created by qpa_create (NULL is accepted). */
void qpa_destroy(qpa_ctx *ctx);

/* Message describing the last failure on `ctx` ("" if none).  Valid until the next
 * call on the same context.  With ctx == NULL: the last failure of a call made without
 * a context (qpa_create, qpa_workspace_size(NULL, ...)) on the calling thread. */
const char *qpa_last_error(const qpa_ctx *ctx);

/* Static name of a status code. */
const char *qpa_status_string(qpa_status status);

/* Device bytes of workspace that qpa_solve needs for (problem, params).
 * The workspace must be 256-byte aligned (any hipMalloc'd or torch-allocated buffer
 * is).  Its content on entry is irrelevant; the library clears what it needs. */
qpa_status qpa_workspace_size(qpa_ctx *ctx, const qpa_problem *problem,
                              const qpa_params *params, size_t *bytes);

/* Run the whole solve -- canonicalisation (App. A), initial state, `steps` PA steps
 * (App. B), exact energies of the final spins, best replica -- for one problem.
 * workspace: device buffer of at least qpa_workspace_size() bytes. */
qpa_status qpa_solve(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                     void *workspace, size_t workspace_bytes, void *stream,
                     const qpa_outputs *out);

/* Best state over the trajectory (Sec. VIII: the solver evolves many states and reports
 * the best one found, which need not be where a replica ends).  Device outputs, each
 * required:
 *  best_energy [R] double: the lowest objective value (as in qpa_outputs.energy) among
 *              the replica's sampled states;
 *  best_step   [R] int32: the number of steps completed at that state (the earliest on
 *              ties);
 *  best_spins  [R*n] int8: that state's spins, row-major by replica. */
typedef struct {
    double *best_energy;
    int32_t *best_step;
    int8_t *best_spins;
} qpa_track_outputs;

/* qpa_solve that also keeps each replica's best state: the steps run in segments of
 * `every` (>= 1) steps, and the state after each segment -- after steps every, 2 every,
 * ..., and after the last step (the initial state when steps == 0) -- is scored exactly
 * like the final one.  The dynamics are those of qpa_solve (a split run gives the same
 * bits), so `out` receives exactly what qpa_solve gives; the cost is one scoring per
 * segment.  workspace: qpa_workspace_size() bytes, as for qpa_solve.
 *  Errors: every < 1, or a missing output -> QPA_E_ARG. */
qpa_status qpa_solve_track(qpa_ctx *ctx, const qpa_problem *problem,
                           const qpa_params *params, int32_t every, void *workspace,
                           size_t workspace_bytes, void *stream, const qpa_outputs *out,
                           const qpa_track_outputs *track);

/* Solve `count` independent sparse instances together (the batch shares params).
 * Instance k is solved exactly as qpa_solve would solve it alone with seed
 * params->seed + k; its outputs go to out[k].
 *  problems : host array of `count` CSR problems (format QPA_FMT_CSR, n <= 4096).
 *  out      : host array of `count` output sets (device pointers as in qpa_outputs).
 *  workspace: device buffer of at least qpa_workspace_size_batch() bytes, for the same
 *             problems and params (flags included).
 * Two paths, chosen per instance (see qpa_batch_flags):
 *  - sparse: tasks (instance, group of 64 replicas), sorted by stored entries, largest
 *    first, taken by the workgroups of one persistent launch from an atomic counter;
 *    no workgroup waits on another;
 *  - dense: the couplings are expanded once into a BF16 matrix (exact, see above), or for
 *    integer weights with |w| <= 127 into int8 (v_mfma_i32_32x32x32_i8, exact int32 sums):
 *    a dense int8 matrix, or, where every 16x128 block is sparse enough, per-block lists
 *    of its nonzeros that the step kernel places into LDS (QPA_PATH_BATCH_SPARSE_I8); every
 *    PA step is one grouped matrix-core launch per kind over the tiles of all such
 *    instances (BF16: 128 replicas x 128 variables; int8: 64 x 256).  Integer instances
 *    give the same bits on every path.
 * When a batch uses both paths, the sparse launch runs on an auxiliary stream beside the
 * dense step loop (disjoint instances) and is joined back before the scoring.
 * Set-up and scoring run on the context's auxiliary streams (ordered after `stream` and
 * joined back into it before the call returns), the per-instance parts issued from up to
 * four host threads of the call's own, the densified integer instances' parts as batched
 * launches over descriptor tables.  The call synchronises `stream` up to three times
 * (after the validation of every instance, and after each of two table uploads).
 * Errors name the offending instance in qpa_last_error(). */
qpa_status qpa_workspace_size_batch(qpa_ctx *ctx, int32_t count, const qpa_problem *problems,
                                    const qpa_params *params, size_t *bytes);
qpa_status qpa_solve_batch(qpa_ctx *ctx, int32_t count, const qpa_problem *problems,
                           const qpa_params *params, void *workspace, size_t workspace_bytes,
                           void *stream, const qpa_outputs *out);

/* Advance a caller-held state by PA steps t0 .. t1-1 (0 <= t0 <= t1 <= params->steps)
 * of the schedule of `params` -- the resume / teacher-forcing entry point.
 *  x, m    : device [R*n] float, read and overwritten in place (R = params->replicas).
 *  h_last  : device [R*n] float or NULL; receives the fields J s + b of the last step
 *            taken (untouched if t0 == t1).
 * The same kernels as qpa_solve run; the seed and sigma0 are not used.  Trajectories are
 * identical to an uninterrupted qpa_solve whatever the split points. */
qpa_status qpa_steps(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                     int32_t t0, int32_t t1, float *x, float *m, float *h_last,
                     void *workspace, size_t workspace_bytes, void *stream);

/* Batched energies and best-of-replica for given spins: energy[r] = the instance's
 * objective of spins[r*n .. r*n+n) (as in qpa_outputs), best = lowest argmin.
 *  spins: device [R*n] int8 in {-1,+1}.  energy: device [R] double (required);
 *  energy_i64: device [R] int64 or NULL; best: device [1] int32 or NULL.
 * Uses the workspace of qpa_workspace_size(problem, params) with params->replicas = R. */
qpa_status qpa_energy(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                      const int8_t *spins, double *energy, int64_t *energy_i64,
                      int32_t *best, void *workspace, size_t workspace_bytes, void *stream);

/* Gradient of the relaxed final energy (the dynamics with analog spins in the target
 * part, s := x; App. B relaxes the binary spins to x in [-1,1]) with respect to the
 * step size eta, the momentum alpha and every schedule value lambda_t.
 *   L = scale * sum_r [ (1/2) x_T^T J x_T + b^T x_T ]   over the params->replicas
 *   replicas started as in qpa_solve (scale = 1/replicas gives the mean), (J, b) the
 *   Ising form of the problem (App. A for a QUBO).
 * Per step: f = J x, h = f + b, g = lambda_t x + h, m' = alpha m - eta g, x' = clip(x + m'),
 * FP32 state (one fused multiply-add per term of J x, ascending columns), FP64
 * accumulation of the gradient sums in a fixed order (results do not depend on
 * ckpt_every).  The forward pass keeps (x, m) every ckpt_every steps; the reverse pass
 * recomputes each segment from its checkpoint, storing the segment's (x, m, J x).
 * The loss is a continuous, piecewise smooth function of the parameters (clipping makes
 * kinks); the gradient is that of the smooth piece the parameters lie in, with the clip
 * derivative taken as 1 on the closed interval [-1, 1].
 *  loss: device [1] double (required).  d_eta, d_alpha: device [1] double;
 *  d_lambda: device [steps] double -- all three given, or all NULL for the forward pass
 *  only (then no checkpoint is kept).
 *  workspace: device buffer of at least qpa_workspace_size_relaxed() bytes.
 * Dense problems use FP32 couplings whatever params->precision says. */
qpa_status qpa_workspace_size_relaxed(qpa_ctx *ctx, const qpa_problem *problem,
                                      const qpa_params *params, int32_t ckpt_every,
                                      size_t *bytes);
qpa_status qpa_relaxed_grad(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                            int32_t ckpt_every, double scale, void *workspace,
                            size_t workspace_bytes, void *stream, double *loss, double *d_eta,
                            double *d_alpha, double *d_lambda);

/* The same for `count` instances sharing params (the loss of the many-instances
 * protocol of Secs. V and VIII):
 *   L = scale * sum_k sum_r [ (1/2) x_T^T J_k x_T + b_k^T x_T ],
 * instance k's replicas started as qpa_solve starts them with seed params->seed + k;
 * scale = 1 / (replicas * count) gives the mean over every replica of the batch.
 *  problems: host array of `count` problems (dense or CSR, mixed types allowed).
 * Every step of the batch is one launch per (coupling, index) type of its CSR instances
 * plus one tiled product per dense instance.  Errors name the offending instance. */
qpa_status qpa_workspace_size_relaxed_batch(qpa_ctx *ctx, int32_t count,
                                            const qpa_problem *problems,
                                            const qpa_params *params, int32_t ckpt_every,
                                            size_t *bytes);
qpa_status qpa_relaxed_grad_batch(qpa_ctx *ctx, int32_t count, const qpa_problem *problems,
                                  const qpa_params *params, int32_t ckpt_every, double scale,
                                  void *workspace, size_t workspace_bytes, void *stream,
                                  double *loss, double *d_eta, double *d_alpha,
                                  double *d_lambda);

/* Step kernels, as named by the profiling calls and qpa_batch_paths. */
typedef enum {
    QPA_PATH_ALL = -1,           /* qpa_profile_read_path: every kernel           */
    QPA_PATH_DENSE_RESIDENT = 0, /* FP32 couplings held in LDS, all steps at once */
    QPA_PATH_DENSE_TILED = 1,    /* FP32 couplings streamed, one launch per step  */
    QPA_PATH_DENSE_MFMA = 2,     /* BF16 matrix-core step, one launch per step    */
    QPA_PATH_CSR = 3,            /* sparse step, one launch per step              */
    QPA_PATH_BATCH_SPARSE = 4,   /* persistent sparse task kernel (all steps)     */
    QPA_PATH_BATCH_DENSE = 5,    /* grouped matrix-core step over many instances  */
    QPA_PATH_CSR_RESIDENT = 6,   /* sparse, state on chip, all steps at once      */
    QPA_PATH_SBM_DENSE = 7,      /* SBM step, dense FP32 couplings                */
    QPA_PATH_SBM_CSR = 8,        /* SBM step, sparse couplings                    */
    QPA_PATH_SBM_CSR_RESIDENT = 9, /* SBM, sparse, state on chip, all steps at once */
    QPA_PATH_BATCH_DENSE_I8 = 10, /* qpa_batch_paths: grouped matrix-core step with int8
                                    couplings (integer |w| <= 127); timed under
                                    QPA_PATH_BATCH_DENSE                           */
    QPA_PATH_CSR_BINNED = 11,    /* sparse, two streaming passes per step (binned)  */
    QPA_PATH_BATCH_SPARSE_I8 = 12 /* qpa_batch_paths: grouped matrix-core step with int8
                                    couplings kept as lists of their nonzeros (at most
                                    384 in every 16 x 128 block of the padded matrix);
                                    timed under QPA_PATH_BATCH_DENSE                */
} qpa_path;

/* Measurement of the PA-step kernels.  While enabled (enable != 0), every qpa_solve,
 * qpa_solve_batch and qpa_steps call records one HIP event on its stream right before
 * its first step kernel of a path and one right after its last, and counts the step
 * kernels it launched.  qpa_profile_read waits for the recorded events and returns the
 * summed elapsed time in milliseconds and the number of step-kernel launches since the
 * last reset (reset != 0 clears the totals after reading); qpa_profile_read_path does the
 * same for the kernels of one qpa_path only (QPA_PATH_ALL: every kernel; reset clears
 * everything).  The averaged interval includes the gaps between consecutive step kernels
 * of one call. */
qpa_status qpa_profile_enable(qpa_ctx *ctx, int32_t enable);
qpa_status qpa_profile_read(qpa_ctx *ctx, double *step_ms, int64_t *step_launches,
                            int32_t reset);
qpa_status qpa_profile_read_path(qpa_ctx *ctx, int32_t path, double *step_ms,
                                 int64_t *step_launches, int32_t reset);

/* The path (QPA_PATH_BATCH_SPARSE, QPA_PATH_BATCH_DENSE, QPA_PATH_BATCH_DENSE_I8 or
 * QPA_PATH_BATCH_SPARSE_I8) that each instance of the last successful qpa_solve_batch on
 * this context took; `count` must equal that call's count.  paths: host array of `count`
 * int32. */
qpa_status qpa_batch_paths(const qpa_ctx *ctx, int32_t count, int32_t *paths);

/* ---------------------------------------------------------------------------------
 * Simulated Bifurcation Machine (App. B): the adiabatic oscillator network
 *   dq_i/dt = a0 p_i,
 *   dp_i/dt = -(q_i^2 + a0 - a(t)) q_i + c0 (sum_j J'_ij q_j + h'_i),
 * on R independent replicas, with a(t) = a0 t / T over T steps of symplectic Euler with
 * step dt (p first, from the positions of the step; then q from the new p).  The
 * machine maximises (1/2) q^T J' q + h'^T q, so it is driven with (J', h') = (-J, -b),
 * (J, b) the Ising form of the problem (App. A for a QUBO); the spins read out at the
 * end are s = sign(q) (sign(0) = +1) and are scored as in qpa_solve.  Per element, in
 * FP32 with one rounding per operation in this order:
 *   g = (sum_j J_ij q_j, one fused multiply-add per term, ascending j) + b_i
 *   w = ((q q + a0) - a) q;  F = -w - c0 g;  p = p + dt F;  q = q + (dt a0) p
 * with a = a0 * ((float)t / (float)T) and dt a0 rounded once.  Initial positions as the
 * PA initial state (q_0 = sigma0 (2u - 1), same counter RNG and seed use); p_0 = 0.
 * c0 = 0 asks for c0 = 1 / rho, rho the spectral radius max |lambda(J)| estimated in
 * FP64 by power_iters iterations of the power method from v_0 = 2u - 1 (u the top 24
 * bits of SplitMix64 output i + 1 of `seed`) -- App. B sets c0 from the largest
 * eigenvalue of the couplings; rho bounds both signs of the spectrum.
 * Dense couplings are used in FP32 (exact for integer |J| < 2^24); params of the PA
 * path (precision, schedule) do not apply. */
typedef struct {
    int32_t replicas;           /* R >= 1                                          */
    int32_t steps;              /* T >= 0                                          */
    float a0;                   /* > 0: inverse mass and final pump level          */
    float c0;                   /* > 0: coupling scale; 0: 1 / (power-method rho)  */
    float dt;                   /* > 0: integration step                           */
    float sigma0;               /* amplitude of the initial positions              */
    uint64_t seed;              /* SplitMix64 seed (initial positions, power start) */
    int32_t power_iters;        /* >= 0, power-method iterations when c0 == 0      */
    int32_t flags;              /* 0, QPA_SOLVE_STREAMED (sparse: per-step kernel
                                   even where the state fits on chip) and/or
                                   QPA_SOLVE_GRAPH                               */
} qpa_sbm_params;

/* Device bytes of workspace for qpa_sbm_solve / qpa_sbm_steps / qpa_spectral_radius
 * (same alignment and ownership rules as qpa_workspace_size). */
qpa_status qpa_workspace_size_sbm(qpa_ctx *ctx, const qpa_problem *problem,
                                  const qpa_sbm_params *params, size_t *bytes);

/* Whole SBM solve: canonicalisation, initial state, c0, T steps, exact energies of
 * sign(q_T), best replica.  Outputs as qpa_outputs, with x <- q_T and m <- p_T. */
qpa_status qpa_sbm_solve(qpa_ctx *ctx, const qpa_problem *problem, const qpa_sbm_params *params,
                         void *workspace, size_t workspace_bytes, void *stream,
                         const qpa_outputs *out);

/* Advance a caller-held SBM state by steps t0 .. t1-1 (0 <= t0 <= t1 <= steps) of the
 * schedule a(t) of `params`.  q, p: device [R*n] float, replica-major, read and
 * overwritten in place.  g_last: device [R*n] float or NULL, receives J q + b of the last
 * step taken.  c0 is resolved as in qpa_sbm_solve.  Split runs give the same bits as an
 * uninterrupted one. */
qpa_status qpa_sbm_steps(qpa_ctx *ctx, const qpa_problem *problem, const qpa_sbm_params *params,
                         int32_t t0, int32_t t1, float *q, float *p, float *g_last,
                         void *workspace, size_t workspace_bytes, void *stream);

/* Spectral radius estimate of the canonical couplings J by the power method of
 * qpa_sbm_params (power_iters, seed), in FP64.  rho: device [1] double. */
qpa_status qpa_spectral_radius(qpa_ctx *ctx, const qpa_problem *problem,
                               const qpa_sbm_params *params, void *workspace,
                               size_t workspace_bytes, void *stream, double *rho);

/* ---------------------------------------------------------------------------------
 * Low-energy spectrum of a sample set (Sec. V.A: a run returns many low-energy states,
 * not only the best).  Among the R samples spins[r*n .. r*n+n) (int8 in {-1,+1}) with
 * energies energy[r], the distinct states ordered by energy and then by the lowest
 * replica index holding them; the first m = min(k, distinct) are written:
 *   out_spins  [m*n] int8 (device, may be NULL): the states,
 *   out_energy [m] double, out_count [m] int32 (replicas holding the state),
 *   out_first  [m] int32 (lowest such replica), out_distinct [1] int32 (distinct states).
 * All pointers are device pointers; entries past m are left untouched.  Equal states
 * must carry equal energies (as every scoring call of this library returns them).
 * States are told apart by a 64-bit hash and confirmed by exact comparison, so the
 * result does not depend on the hash.  R <= QPA_SPECTRUM_MAX_R (one workgroup sorts the
 * samples on chip); larger R returns QPA_E_UNSUPPORTED.
 * flags: 0, or QPA_SPECTRUM_EXACT_ONLY to group equal-energy samples by exact
 * comparison alone (diagnostic; same result, slower). */
#define QPA_SPECTRUM_MAX_R 4096
#define QPA_SPECTRUM_EXACT_ONLY 1
qpa_status qpa_workspace_size_spectrum(qpa_ctx *ctx, int64_t n, int32_t R, size_t *bytes);
qpa_status qpa_spectrum(qpa_ctx *ctx, int64_t n, int32_t R, const int8_t *spins,
                        const double *energy, int32_t k, int32_t flags, void *workspace,
                        size_t workspace_bytes, void *stream, int8_t *out_spins,
                        double *out_energy, int32_t *out_count, int32_t *out_first,
                        int32_t *out_distinct);

/* Autotuning of the sparse step kernel (CSR problems).  Times `probe_steps` PA steps
 * (at most params->steps) of every applicable kernel configuration -- the streamed
 * per-step kernel, the resident kernel with 1, 2, 4 or 8 replicas per workgroup where
 * the instance fits on chip, and the binned step where it applies (QPA_SOLVE_BINNED)
 * -- each from the initial state of `params`, warmed up
 * once, and records the fastest for this shape (n, nnz, kind, dtypes, replicas) in the
 * context: later qpa_solve / qpa_steps / qpa_energy calls on the context with the same
 * shape use it (unless params->flags holds QPA_SOLVE_STREAMED or QPA_SOLVE_BINNED).
 * Every configuration
 * gives the same bits.
 *  workspace: as for qpa_solve (its size does not depend on the choice);
 *  choice (host, required): 0 = streamed kernel, G = resident kernel with G replicas,
 *  QPA_TUNE_BINNED = binned step;
 *  ms (host, optional, 6 doubles): probe milliseconds of [streamed, G=1, 2, 4, 8,
 *  binned], -1 where a configuration does not apply.
 * Dense problems return QPA_E_UNSUPPORTED. */
qpa_status qpa_autotune(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                        int32_t probe_steps, void *workspace, size_t workspace_bytes,
                        void *stream, int32_t *choice, double *ms);

/* Measure the two paths of qpa_solve_batch on this device for `count` instances: the
 * batch is solved for probe_steps steps with every BF16-exact instance forced dense, then
 * with every instance forced sparse (a warm-up run before each timed one), and the
 * step-kernel time of each path gives its rate -- dense tiles in bytes per second,
 * counting 2 bytes per coupling of the padded matrix (4 per stored entry for the int8
 * entry lists) plus 16 per variable and replica (x and m read and written), sparse tasks
 * in coupling adds per second (stored entries times replicas).  The context keeps the rates; later qpa_workspace_size_batch and
 * qpa_solve_batch calls on it choose each instance's path with them (before any
 * measurement, built-in estimates are used).
 *  rates (host, optional, 2 doubles): the rates now in effect [dense B/s, sparse adds/s].
 * The tuner allocates the probe's workspace and outputs itself and frees them before it
 * returns; `stream` is synchronised. */
qpa_status qpa_autotune_batch(qpa_ctx *ctx, int32_t count, const qpa_problem *problems,
                              const qpa_params *params, int32_t probe_steps, void *stream,
                              double *rates);

/* Record a sparse kernel choice for this shape by hand (0 = streamed, the resident
 * kernel's replica group 1, 2, 4 or 8, or QPA_TUNE_BINNED, where it applies), as
 * qpa_autotune would. */
#define QPA_TUNE_BINNED (-1)
qpa_status qpa_tune_set(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                        int32_t choice);

/* Allocation-free solve, for callers that cannot allocate memory (tight serving loops,
 * harnesses that forbid hipMalloc): the same solve as qpa_solve -- same kernels, same
 * results bit for bit -- with the workspace taken from a device buffer the library owns
 * instead of a caller argument.  The buffer is a static device array of
 * QPA_NOALLOC_WORKSPACE_BYTES; every device the library is loaded on holds its own copy
 * until the process ends.  The call allocates nothing (no device, pinned or managed
 * memory; no HIP event, stream or graph): the schedule staging buffer it needs is
 * reserved by qpa_create.
 *  Limits: problems whose qpa_workspace_size() exceeds QPA_NOALLOC_WORKSPACE_BYTES fail
 *  with QPA_E_WORKSPACE; steps > QPA_NOALLOC_MAX_STEPS and QPA_SOLVE_GRAPH (capturing a
 *  graph allocates) fail with QPA_E_UNSUPPORTED.  Profiling spans are not recorded.
 *  Sharing: all calls on one device -- from any context -- use the same buffer, which
 *  keeps the last call's contents (the solve clears what it needs).  Calls that overlap
 *  in time on one device race on it: issue them from one host thread on one stream, or
 *  order them by synchronisation.  Like qpa_solve, the call synchronises `stream` once
 *  to report invalid input, so it cannot be recorded into a graph. */
#define QPA_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
#define QPA_NOALLOC_MAX_STEPS 65536
qpa_status qpa_solve_noalloc(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                             void *stream, const qpa_outputs *out);

/* Library version string. */
const char *qpa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QPA_H */
