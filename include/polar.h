/*
 * polar.h -- C-ABI of libpolar: the online part of the method of polarized
 * traces for the 2D Helmholtz equation (Zepeda-Nunez & Demanet, "The method
 * of polarized traces for the 2D Helmholtz equation", 2014) on one AMD
 * Instinct MI355X (gfx950).
 *
 * Problem (paper Section 2.1): -Lap u - omega^2 m u = f, m = 1/c^2, on the
 * PML-padded rectangle with homogeneous Dirichlet data, discretised by the
 * 5-point stencil with the unsymmetric PML alpha = 1/(1 + i sigma/omega),
 * sigma(d) = (C/delta)(d/delta)^2, delta = npml*h.  Physical nodes are
 * x_p = p*h, p = 1..nx (same for z); the padded grid has
 * NX = nx + 2 npml columns (x, fastest) and NZ = nz + 2 npml rows (z).
 *
 * Method: pt_setup runs the offline part (Alg. 1): the z axis is split into
 * L layers (Section 2.2; physical rows split evenly, layer 1 and layer L own
 * the global PML rows, interior sides get npml extension rows), each layer's
 * operator is factored on the GPU line by line (block-tridiagonal Schur
 * recurrence Delta_r = A_r - l_r u_{r-1} Delta_{r-1}^{-1}, appendix B,
 * Def. 10, with dense pivoted inverses of the NX x NX blocks), and the local
 * Green's trace blocks between local rows {0, 1, n, n+1} are extracted
 * (Def. 1, Def. 2).  pt_solve runs the online part (Alg. 2): local solves
 * for the Newton potentials (Def. 3), flexible GMRES on the polarized system
 * closed by jump conditions (Def. 9) preconditioned by n_it Gauss-Seidel
 * sweeps (Alg. 4), then one forced local solve per layer
 * (eq. PDE_version_green_formula) for the volume field.
 *
 * Conventions shared by every entry point:
 *  - complex numbers are interleaved (re, im) float64 pairs (the layout of
 *    C99 double _Complex and numpy complex128);
 *  - a volume field is (nrhs, NZ, NX), x fastest, right-hand sides slowest;
 *  - a polarized trace vector is (nrhs, 2, L-1, 2, NX): [down part d | up part
 *    a], then interface k = 0..L-2 (between layers k and k+1, 0-based), then
 *    the two trace rows (row n and n+1 of layer k = rows 0 and 1 of layer
 *    k+1), then x;
 *  - a layer-local field is (nrhs, sum_l R_l, NX): layer l's R_l local rows
 *    (top extension, owned rows, bottom extension) stacked by layer;
 *  - `on_device` = 1: every data pointer is device memory on the solver's
 *    device (the call is asynchronous on the solver's stream except where
 *    stated); 0: host memory (the call copies and synchronises);
 *  - the caller owns every pointer it passes; pt_setup copies the model and
 *    keeps no caller pointer; the solver owns all its device memory until
 *    pt_free;
 *  - every call returns a pt_status; no exception crosses the ABI; on error
 *    pt_last_error() returns a thread-local message;
 *  - one solver is driven from one host thread at a time (calls on one solver
 *    are not re-entrant); different solvers are independent.
 */
#ifndef POLAR_H
#define POLAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PT_OK = 0,
  PT_EINVAL = 1,     /* invalid argument; outputs untouched                      */
  PT_ENOMEM = 2,     /* device allocation failed                                  */
  PT_EHIP = 3,       /* HIP runtime error                                         */
  PT_ESINGULAR = 4,  /* zero pivot in the local factorisation                     */
  PT_ENOCONV = 5     /* some source did not converge (GMRES reached maxit, or the
                        source is not finite); u holds the last iterate's field,
                        the per-source info says which                           */
} pt_status;

typedef enum {
  PT_F64 = 0,        /* every block apply and local solve in complex float64     */
  PT_F32 = 1,        /* the Gauss-Seidel preconditioner (sweeps and reflection
                        terms) applies float32 copies of the trace blocks
                        (complex float32, float32 accumulation; on the FP32
                        MFMA with more than 4 sources); local solves,
                        the operator A inside GMRES, Krylov vectors, Arnoldi,
                        least squares and true residuals stay float64, so
                        flexible GMRES converges to the float64 solution (both
                        block copies are kept) */
  PT_SPLIT_BF16 = 2, /* mixed: the Gauss-Seidel preconditioner (sweeps and
                        reflection terms) applies the trace blocks as split
                        bfloat16 pairs (hi + lo) on MFMA with float32
                        accumulation; local solves, the operator A inside GMRES
                        and everything else stay float64, so flexible GMRES
                        converges to the float64 solution (both block copies
                        are kept: 1.5x the float64 block memory)            */
  PT_SPLIT_F16 = 3   /* mixed, as PT_SPLIT_BF16 but with float16 pairs on the
                        float16 MFMA (about 22 significant bits per pair
                        instead of 16).  float16 has a 5-bit exponent: every
                        split matrix is stored times one power of two chosen at
                        setup (the largest Frobenius norm of a trace block maps
                        to 2^14) and the inputs are split at 2^12 times their
                        value, sized for unit-norm inputs (GMRES's Krylov
                        vectors; pt_apply and pt_gauss_seidel scale their
                        inputs to unit norm per source and back)             */
} pt_precision;

/* One Helmholtz problem (paper Section 2.1; Alg. 1 inputs m, omega). */
typedef struct {
  int32_t nx, nz;    /* physical nodes along x (fast) and z (layered axis); >= 1   */
  int32_t npml;      /* PML nodes per side, also the layer extension width; >= 1 */
  double h;          /* grid spacing, > 0                                         */
  double omega;      /* angular frequency, > 0                                    */
  double pml_C;      /* PML strength C of sigma = (C/delta)(d/delta)^2, >= 0      */
  int32_t L;         /* number of layers, >= 1; every layer needs >= 2 physical
                        rows (nz >= 2L)                                           */
  const double* c;   /* host velocity on the padded grid, NZ*NX values, > 0,
                        finite, x fastest                                         */
} pt_problem;

typedef struct {
  int32_t precision; /* pt_precision                                              */
  int32_t gs_iters;  /* n_it of the Gauss-Seidel preconditioner (Alg. 4), 0..8;
                        0 = unpreconditioned GMRES. Paper: 2                      */
  double tol;        /* GMRES stop: relative residual of the trace system         */
  int32_t maxit;     /* GMRES iterations (no restart), 1..200                     */
  int32_t max_nrhs;  /* largest nrhs pt_solve will be called with, >= 1           */
  int32_t plr;       /* 1: store and apply the trace blocks in partitioned
                        low-rank form (Alg. 5 / Alg. 6), compressed on the GPU
                        at setup; float64 only                                  */
  double plr_eps;    /* absolute singular-value threshold of a leaf, > 0        */
  int32_t plr_rmax;  /* leaf rank limit, 1..64 (0: ceil(sqrt(NX)))              */
  int32_t use_graph; /* 1: each GMRES iteration's launches (preconditioner,
                        operator, Arnoldi, Givens, convergence flags) are
                        captured once per (nrhs, iteration) into a hipGraph and
                        replayed on later solves; needs a non-null stream; not
                        used while profiling or with the learned stage; pt_tune
                        discards the graphs.  0: plain stream launches.      */
  int32_t presolve;  /* how the pre-solve (Alg. 2, N^l f^l at the trace rows) is
                        formed.  0: forward and backward line-by-line local
                        solves over the layers a source touches.  1: products
                        with the layers' interface Green's functions: the rows
                        j = 0, 1, n, n+1 of (A^l)^-1 over every owned row, kept on
                        the device after setup (Def. 3 with the source restricted
                        to the layer), one launch instead of ~R dependent ones;
                        PT_ENOMEM if they do not fit.
                        2: kept when they take at most a third of the free
                        device memory at setup; used for
                        every pre-solve (passes of more than 4 columns split
                        each product over row ranges).                         */
  int32_t closure;   /* how the polarized system is closed (Section 3.4).
                        0: jump conditions (Def. 9) with the Gauss-Seidel
                        preconditioner of its splitting (Alg. 4).  1: the
                        extrapolation relations (Def. polarized_out_going):
                        the rows at row n / row 1 are kept and the other row
                        of each pair becomes u_{n+1} = E_down u_n,
                        u_0 = E_up u_1, with the one-sided extrapolators taken
                        from the stored factors (E_down = -l Sigma_{n+1}^-1,
                        E_up = -u Delta_0^-1); Gauss-Seidel on its splitting
                        (eq. splitting_out_going), D^-1 as the jump system's
                        sweeps after one extrapolation step.  Same solution;
                        float64 factors without PLR blocks only (PT_EINVAL).   */
} pt_options;

typedef struct {
  int32_t iters;     /* GMRES iterations used                                     */
  int32_t converged; /* 1 if the residual estimate reached tol (0 for a source
                        with a NaN or Inf: it stops at once, est and relres NaN)  */
  double est;        /* GMRES residual estimate at exit (relative)                */
  double relres;     /* true relative residual ||s - A x|| / ||s|| in float64     */
  int32_t learned;   /* 1 if the result came from GMRES with the learned stage    */
  int32_t learned_steps; /* GMRES steps of this RHS that used the network's output    */
} pt_rhs_info;

typedef struct {
  int32_t NX, NZ, L;
  int32_t sumR;      /* rows of a layer-local field                               */
  int64_t ntrace;    /* complex entries of one polarized trace vector, 4(L-1)NX   */
  int32_t R[64];     /* local rows per layer (first min(L,64) layers)             */
  int32_t own_start[64], n_own[64], top_ext[64], bot_ext[64];
  double setup_ms;   /* wall time of pt_setup                                     */
  int64_t block_bytes;  /* device bytes of the trace blocks as applied (PLR storage
                           when plr = 1)                                          */
  int64_t factor_bytes; /* device bytes of the local factors                      */
  int64_t dense_block_bytes; /* device bytes the dense trace blocks take          */
  int64_t plr_leaves;   /* leaves of all compressed blocks (0 without PLR)         */
  int64_t green_bytes;  /* device bytes of the interface Green's functions of the
                           pre-solve (0: line-by-line pre-solve)                 */
  double plr_ms;        /* wall time of the GPU compression inside pt_setup
                           (0 without PLR)                                        */
  int32_t max_nrhs;     /* the options' max_nrhs                                  */
  int32_t plr_rmax;     /* leaf rank limit of the compressed blocks in use (0: none) */
  int32_t precision;    /* the options' pt_precision                              */
} pt_layout;

typedef struct pt_solver pt_solver;

/* Offline part (Alg. 1).  Validates the problem (PT_EINVAL on nx, nz, npml < 1,
 * h or omega <= 0, C < 0, L < 1, a layer with < 2 physical rows, c <= 0 or not
 * finite, NX > 4096), allocates every device buffer for up to opt->max_nrhs
 * right-hand sides, factors the local problems and extracts the trace blocks
 * on the GPU.  `hip_stream` is a hipStream_t (NULL = the null stream) on the
 * current device; it becomes the solver's stream.  Synchronous. */
pt_status pt_setup(const pt_problem* prob, const pt_options* opt, void* hip_stream, pt_solver** out);

/* Online part (Alg. 2): u = H^{-1} f for nrhs fields f (nrhs, NZ, NX).  f is
 * restricted to each layer's owned rows (its PML part is used as given).
 * info (host, nrhs entries, may be NULL) receives per-RHS GMRES data.
 * Returns PT_ENOCONV if any right-hand side missed tol within maxit or is not
 * finite (decided whether or not info is given; u is still written: the
 * field of the last GMRES iterate).  Host-synchronising once per GMRES
 * iteration. */
pt_status pt_solve(pt_solver* s, int32_t nrhs, const double* f, double* u, int32_t on_device,
                   pt_rhs_info* info);

void pt_free(pt_solver* s); /* NULL is a no-op */

/* Several problems' offline parts (Alg. 1) at once, e.g. the problems of an
 * uneven batch: problem i is set up as by pt_setup(&probs[i], &opts[i],
 * hip_streams[i], &out[i]) on its own host thread, on the caller's current
 * device, so the latency-bound factorisation launches of different problems
 * overlap on the GPU when their streams are distinct (hip_streams may be NULL:
 * every problem on the null stream, one after another in effect).  On any
 * failure every solver of the batch is freed, out[] is all NULL, and the
 * first failing problem's status is returned (pt_last_error names it). */
pt_status pt_setup_batch(int32_t nprob, const pt_problem* probs, const pt_options* opts, void* const* hip_streams,
                         pt_solver** out);

/* The offline state of a solver -- the local factors, the trace blocks, the
 * interface Green's functions when kept, the compressed (PLR) blocks and the
 * tuned launch shapes, with the problem and the options -- written to the
 * file `path` (Alg. 1's output, which Alg. 2 reuses for every right-hand
 * side).  Synchronises the solver's stream.  PT_EINVAL if the file cannot be
 * written. */
pt_status pt_save(const pt_solver* s, const char* path);

/* A solver read back from a file written by pt_save, on `hip_stream` of the
 * current device: no factorisation, extraction or compression is repeated,
 * and pt_solve returns bit-identical results to the saved solver's.
 * PT_EINVAL for a file that is not a saved solver of this library version
 * (or is truncated), PT_ENOMEM if the device memory does not suffice. */
pt_status pt_load(const char* path, void* hip_stream, pt_solver** out);

const char* pt_status_str(pt_status st);
const char* pt_last_error(void);

/* ---- stages of the online path, for verification and profiling ---------- */

pt_status pt_get_layout(const pt_solver* s, pt_layout* out);

/* K^l_{j,k} = (A^l)^{-1}_{j,k}, A^l = h^2 H^l, the Green's trace block of layer
 * l between local rows j, k in {0: row 0, 1: row 1, 2: row n, 3: row n+1}
 * (Def. 1: G^l(z_j, z_k) = h K_{j,k}).  Written to host `out` as an NX x NX
 * row-major complex matrix (rows: target x).  PT_EINVAL if the layer has no
 * such row (layer 0 has no rows 0, 1; layer L-1 no rows n, n+1).  Reads the
 * stored float64 blocks. */
pt_status pt_get_block(const pt_solver* s, int32_t layer, int32_t j, int32_t k, double* out);

/* The same block as pt_get_block, expanded from its partitioned low-rank form
 * (Section 5, Alg. 5: the adaptive quadtree of low-rank and dense leaves, built
 * on the GPU at setup when plr = 1): the product U V of every low-rank leaf and
 * the entries of every dense leaf, written to host `out` (NX x NX row-major
 * complex).  `nleaves` and `stored` (either may be NULL) receive the block's
 * leaf count and stored complex entries.  PT_EINVAL if the solver was set up
 * without plr or the block does not exist; allocates one NX x NX device
 * buffer for the call. */
pt_status pt_get_plr_block(const pt_solver* s, int32_t layer, int32_t j, int32_t k, double* out, int32_t* nleaves,
                           int64_t* stored);

typedef enum {
  PT_OP_A = 0,       /* y = A x: polarized system closed by jump conditions (Def. 9) */
  PT_OP_R = 1,       /* y = R x, R = A - D (eq. def_permuted_system_jump)            */
  PT_OP_DINV = 2,    /* y = D^{-1} x: down sweep and up sweep (Section 4.1)          */
  PT_OP_PRECOND = 3, /* y = M^{-1} x: Gauss-Seidel preconditioner, gs_iters (Alg. 4) */
  /* the same four for the system closed by extrapolation (closure = 1 only) */
  PT_OP_A_EXTRAP = 4,
  PT_OP_R_EXTRAP = 5,
  PT_OP_DINV_EXTRAP = 6,
  PT_OP_PRECOND_EXTRAP = 7
} pt_op;

/* y = op(x) on polarized trace vectors (nrhs, 2, L-1, 2, NX); L >= 2. */
pt_status pt_apply(pt_solver* s, int32_t op, int32_t nrhs, const double* x, double* y, int32_t on_device);

/* x = (A^l)^{-1} b for every layer l at once on layer-local fields
 * (nrhs, sumR, NX): the forward/backward block sweep with the stored factors. */
pt_status pt_local_solve(pt_solver* s, int32_t nrhs, const double* b, double* x, int32_t on_device);

/* Right-hand side of the polarized system for sources f (nrhs, NZ, NX):
 * s_down,k = (N f)^k at rows n, n+1; s_up,k = (N f)^{k+1} at rows 0, 1 with
 * N f = (A^l)^{-1} h^2 f^l (Def. 3, Alg. 2).  s: (nrhs, 2, L-1, 2, NX). */
pt_status pt_trace_rhs(pt_solver* s, int32_t nrhs, const double* f, double* out, int32_t on_device);

/* Volume field from sources f and polarized traces x (both as above): one
 * forced local solve per layer with t = d + a (eq. PDE_version_green_formula). */
pt_status pt_reconstruct(pt_solver* s, int32_t nrhs, const double* f, const double* x, double* u,
                         int32_t on_device);

/* Gauss-Seidel on the polarized system as a stand-alone solver (Alg. 3):
 * u^0 = 0, u^{i+1} = D^-1 (s - R u^i) (the sweeps of Section 4.1), stopping
 * when every source's relative update ||u^{i+1} - u^i|| / ||u^{i+1}|| is below
 * tol or after maxit iterations; then the volume field is reconstructed as in
 * pt_solve.  iters (may be NULL): iterations taken; relupd (may be NULL, nrhs
 * entries): each source's last relative update.  PT_ENOCONV if maxit was
 * reached (u holds the last iterate's field).  PT_EINVAL for L = 1. */
pt_status pt_gauss_seidel(pt_solver* s, int32_t nrhs, const double* f, double* u, int32_t on_device, double tol,
                          int32_t maxit, int32_t* iters, double* relupd);

/* Several independent problems at once (problems of uneven size and L):
 * problem i is solved by s[i] for nrhs[i] sources, f[i] -> u[i], info[i]
 * (each as in pt_solve; info[i] may be NULL).  Each problem runs on its own
 * host thread and its solver's stream, so the launches of different problems
 * overlap on the GPU when the solvers were set up on distinct streams (on a
 * shared stream they run one after another, with the same results).  The
 * solvers must be distinct.  Returns PT_OK, or the first non-OK status in
 * problem order (every problem is still attempted; pt_last_error describes
 * that problem's failure). */
pt_status pt_solve_batch(int32_t nprob, pt_solver* const* s, const int32_t* nrhs, const double* const* f,
                         double* const* u, int32_t on_device, pt_rhs_info* const* info);

/* The same batch as one launch sequence from one host thread (Alg. 2 for
 * every problem, in lockstep): each stage -- source activity and pre-solve
 * (the w^l of every layer, its traces), GMRES start, each GMRES iteration
 * of the problems not yet converged, GMRES end and reconstruction,
 * convergence data -- is issued for all problems before the host waits,
 * once per stage.  In the iterations, the block applies (Alg. 4's sweeps
 * and the operator of Def. 9) of problems with the same kernel family (the
 * same block storage and the same side of the form's right-hand-side
 * threshold) share one launch, one segment of the grid per problem with its
 * own block size, right-hand sides and vectors; a lone problem keeps its
 * tuned shape, merged launches take the rules' shapes for their total size.
 * The pre-solve and reconstruction chains run on the problems' own streams
 * when these are distinct (they overlap), otherwise everything runs on
 * s[0]'s stream.  Arguments, results and statuses as pt_solve_batch; every
 * solver on one device and without a learned stage (PT_EINVAL otherwise).
 * Each problem's arithmetic is its pt_solve's up to the launch shapes (the
 * summation order inside a merged launch), so results agree with separate
 * solves to rounding.  Synchronises every solver's stream first and s[0]'s
 * stream before returning. */
pt_status pt_solve_batch_merged(int32_t nprob, pt_solver* const* s, const int32_t* nrhs, const double* const* f,
                                double* const* u, int32_t on_device, pt_rhs_info* const* info);

/* The variant of pt_apply that allocates nothing, for callers that cannot
 * allocate device memory at call time (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same operators and the
 * same result as pt_apply (bit for bit); x and y are device pointers
 * (nrhs, 2, L-1, 2, NX) on the solver's device, and y must not overlap x.
 * Instead of the solver's work buffers, the Gauss-Seidel iterates, the staged
 * input and the k-slice partial tiles of the split-bfloat16 launches live in
 * one fixed 64 MiB device array per GPU (held until the process ends; its
 * address is taken at the first pt_setup on that device).  It needs
 * 3 * nrhs * 4(L-1)NX * 16 bytes (each rounded up to 256) plus the partial
 * tiles; larger calls return PT_EINVAL with the size in pt_last_error().
 * MFMA launches that pt_tune split into k-slices over workgroups keep their
 * partial tiles in the solver's own workspace, allocated by pt_setup.
 * Every call on one GPU shares that array and overwrites it (nothing in it
 * needs to start at zero), so calls that overlap on one GPU, from any
 * solvers or streams, race: serialise them.  Synchronises the solver's
 * stream before returning. */
pt_status pt_apply_noalloc(pt_solver* s, int32_t op, int32_t nrhs, const double* x, double* y);

/* ---- live kernel timing ----------------------------------------------- */

typedef struct {
  int64_t launches;   /* block-apply launches recorded                           */
  double kernel_ms;   /* sum of their durations (HIP events on the solver stream) */
  double alg_bytes;   /* algorithmic bytes: every matrix block once + the vectors
                         each launch must read and write                          */
  double alg_flops;   /* 8 flops per complex multiply-add                          */
} pt_kernel_stats;

/* enable = 1: reset the counters and record a HIP event pair around every
 * block-apply launch (the kernel that streams the Green's blocks and local
 * factors); enable = 0: stop recording (counters kept). */
pt_status pt_profile(pt_solver* s, int32_t enable);
/* Synchronises the solver stream and returns the accumulated counters. */
pt_status pt_profile_read(pt_solver* s, pt_kernel_stats* out);

/* Classes of block-apply launches (for per-class counters and tuning). */
typedef enum {
  PT_CLS_LOCAL = 0,    /* one row step of the local solves (pre-solve, reconstruction)  */
  PT_CLS_SWEEP = 1,    /* one step of the Gauss-Seidel down and up sweeps (Alg. 4)       */
  PT_CLS_REFLECT = 2,  /* the reflection terms of a Gauss-Seidel pass                    */
  PT_CLS_OPERATOR = 3, /* the polarized operator A = D + R, or R alone                   */
  PT_CLS_PRESOLVE = 4, /* pre-solve products with the interface Green's functions; with
                          skipped all-zero input chunks (MFMA form) the counters hold
                          the bytes and flops of the chunks actually streamed            */
  PT_CLS_COUNT = 5
} pt_launch_class;
/* The counters of one launch class (same synchronisation as pt_profile_read). */
pt_status pt_profile_read_class(pt_solver* s, int32_t cls, pt_kernel_stats* out);

/* ---- autotuner ----------------------------------------------------------
 *
 * Tile shapes of the block-apply kernels are chosen per launch by built-in
 * rules.  pt_tune times, for nrhs right-hand sides, every candidate shape of
 * each launch class on one representative launch of that class (HIP events,
 * one warm-up and three timed runs on the solver's own work buffers, whose
 * contents it overwrites) and keeps the fastest if it is at least 2% faster
 * than the built-in rule's shape (else the rule's shape stays, so that shapes
 * within the timing noise of each other do not change from run to run);
 * later calls with the same nrhs use it.  Candidates: MFMA tiles (float64
 * or float32 blocks) of 16, 32 or 64 right-hand sides, with the 16-wide
 * tile's chunks split over 1, 2 or 4 wave groups, or, where the solver's
 * workspace holds the partial tiles (sweep steps and reflection terms of the
 * float64 and float32 forms, operator A of every form; not the local solves'
 * passes), over 2, 4 or 8 workgroups; split tiles of 32 or 64
 * right-hand sides, split over 1..16 k-slices.  Classes with a single form
 * (the row-streaming kernel for <= 4 right-hand sides, compressed blocks) are
 * reported with tried = 1; the pre-solve products are not tuned (tried = 0).
 * With compressed blocks (plr = 1) it first picks the leaf rank limit r_max,
 * the partition threshold of Alg. 5, among ceil(sqrt(NX)) x {1/2, 1, 2, 4}
 * (<= 64) at the solver's eps: each candidate tree is built on the GPU and the
 * compressed-block launches of one GMRES iteration (sweeps, reflection terms,
 * A) are timed; the fastest tree stays in use (pt_get_layout reports it).
 * Every choice goes into a process-wide cache keyed by (NX, L, precision,
 * closure, compressed or not, launch class, nrhs, the launch's job count);
 * pt_tune reuses a cached choice instead of timing (cached = 1), and
 * pt_tune_cache_save / pt_tune_cache_load keep the cache in a text file
 * across processes (load merges; PT_EINVAL, and nothing merged, for a file
 * that is not one or that names a tile shape the kernels do not have).
 * out: PT_CLS_COUNT entries (may be NULL). */
typedef struct {
  int32_t cls;        /* pt_launch_class                                          */
  int32_t tried;      /* candidate shapes timed (0: no launch, or not tuned)       */
  int32_t tile_rhs;   /* right-hand sides per tile of the shape in use, the rule's  */
                      /* when no candidate replaced it (0: single form)            */
  int32_t ksplit;     /* wave groups or k-slices per tile of that shape            */
  double best_us;     /* its mean launch time                                      */
  double default_us;  /* the built-in rule's mean launch time                      */
  int32_t cached;     /* 1: taken from the tuning cache, not timed                 */
} pt_tune_entry;
pt_status pt_tune(pt_solver* s, int32_t nrhs, pt_tune_entry* out);
pt_status pt_tune_cache_save(const char* path);
pt_status pt_tune_cache_load(const char* path);

/* ---- learned preconditioner stage --------------------------------------
 *
 * Not in the paper.  A small 1D convolutional network N along the interface
 * coordinate adds a stage to the Gauss-Seidel preconditioner GS inside
 * flexible GMRES.  For the Krylov vector v of a step with z = GS(v), the
 * residual of that step is r = v - A z, and N(r) estimates A^{-1} r, what z
 * misses of A^{-1} v.  Two ways of using it (pt_learned_mode):
 *   PT_LEARN_CORRECT: every step uses z + c, c = N(r), for a right-hand side
 *     whose float64 residual drops (||r - A c|| < ||r||), else z alone;
 *   PT_LEARN_AUGMENT: steps alternate: a sweep step z = GS(v), then a network
 *     step whose direction is N(r) for the previous step's r; GMRES weighs
 *     the two directions itself.  A network step costs one apply of A and no
 *     sweeps.
 * The network sees each interface separately as 8 real channels ({down, up}
 * x {row n, row n+1} x {re, im}) of r divided by their RMS; its output is
 * scaled back.  Architecture: 4 convolutions 8 -> 32 -> 32 -> 32 -> 8,
 * kernel 5 with dilations 1, 2, 4, 8 (taps (k - 2) d apart: 61 interface
 * points around each output), zero padding, ReLU between layers; bfloat16
 * weights, float32
 * activations and accumulation, float32 master weights trained with Adam.
 * Training pairs (r, e) come from the method's own solves: for every Krylov
 * vector v of a sweep-only GMRES, r = v - A GS(v) and e = A^{-1} r from a
 * tight trace solve.  If a solve with the learned stage misses tol or its
 * float64 true residual exceeds 10 tol, pt_solve repeats it with the sweeps
 * only.  Parameter order (float32): w1 (32x8x5), b1 (32), w2 (32x32x5), b2,
 * w3, b3, w4 (8x32x5), b4 (8); weights are (out, in, k) row-major.
 * A network is used by one thread at a time: training and solves that use it
 * must not overlap. */
typedef enum { PT_LEARN_CORRECT = 0, PT_LEARN_AUGMENT = 1 } pt_learned_mode;
typedef struct pt_learned pt_learned;

/* Network with He-initialised weights (seeded) and room for `capacity`
 * training samples; runs on `hip_stream`. */
pt_status pt_learned_create(int32_t capacity, uint64_t seed, void* hip_stream, pt_learned** out);
void pt_learned_free(pt_learned* net); /* NULL is a no-op */
int64_t pt_learned_num_params(void);
pt_status pt_learned_get_params(const pt_learned* net, float* out);   /* float32 master weights (host) */
pt_status pt_learned_set_params(pt_learned* net, const float* in);     /* also refreshes the bf16 copy  */
/* Loss (mean over samples of ||y - t||^2 / ||t||^2) and its gradient with
 * respect to every parameter, for host inputs x, t of shape (batch, 8, n),
 * computed by the GPU forward/backward kernels with the bf16 weights. */
pt_status pt_learned_gradient(pt_learned* net, int32_t batch, int32_t n, const float* x, const float* t,
                              double* loss, float* grad);
pt_status pt_learned_forward(pt_learned* net, int32_t batch, int32_t n, const float* x, float* y);
/* Training pairs (r, e) from solver s on sources f (nrhs <= max_nrhs of s,
 * host or device array like pt_solve): every Krylov vector of its sweep-only
 * GMRES, up to the fewest iterations any of the nrhs sources took, gives L-1
 * samples (one per interface) until the capacity is reached.  All samples of
 * one network share one interface length NX (PT_EINVAL otherwise); the
 * network itself applies to any NX.  *added: samples added. */
pt_status pt_learned_collect(pt_learned* net, pt_solver* s, int32_t nrhs, const double* f, int32_t on_device,
                             int32_t* added);
pt_status pt_learned_samples(const pt_learned* net, int32_t* count, int32_t* n);
/* `steps` Adam steps on random mini-batches; loss_per_step (host, may be NULL). */
pt_status pt_learned_train(pt_learned* net, int32_t steps, int32_t batch, double lr, double* loss_per_step);
/* Use `net` as the learned stage of s in the given pt_learned_mode (NULL:
 * sweeps only).  The network must outlive its use by s. */
pt_status pt_solver_set_learned(pt_solver* s, pt_learned* net, int32_t mode);
pt_status pt_learned_save(const pt_learned* net, const char* path);
pt_status pt_learned_load(pt_learned* net, const char* path);

#ifdef __cplusplus
}
#endif

#endif /* POLAR_H */
