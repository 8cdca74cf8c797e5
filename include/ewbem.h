/*
 * ewbem: exponential-window frequency-domain BEM for 3-D transient
 * elastodynamics on AMD MI355X (gfx950).
 *
 * The library computes the transient boundary response of an elastic solid
 * by the method of Xiao, Ye and Wen (arXiv:1212.3032):
 *   - Sec. 2.2 / Sec. 3.3: sample the load history, take its damped DFT;
 *   - Sec. 3.1: solve at the complex frequencies s_k = sigma + i k (2 pi / T),
 *     k = 0..N_f/2 (the exponential window's damping sigma);
 *   - Sec. 2.1: collocation BEM with constant flat triangles, system
 *     T u = U t (free term in T), A = T and b = U t for traction loading;
 *   - Sec. 4: the sequence A_k a_k = b_k solved by GMRES with a
 *     block-diagonal preconditioner from an extrapolated initial guess
 *     (Sec. 4.2, solution extrapolation); here A_k is a hierarchical matrix
 *     (cluster tree, admissibility, adaptive cross approximation, dense
 *     near field) instead of the paper's precorrected FFT;
 *   - Sec. 3.2 / 3.3: conjugate fill, Hann or Blackman window, inverse DFT,
 *     de-damping by exp(sigma t).
 *
 * Conventions
 *   - Degree of freedom 3 e + i is Cartesian component i of element e, in
 *     the caller's element order (the internal cluster-tree order is hidden).
 *   - Complex values are interleaved double pairs (ewbem_z), the layout of
 *     numpy/torch complex128.
 *   - Pointers documented "host" must be host memory; "device" must be
 *     device memory on the context's GPU (e.g. a torch tensor's data_ptr()).
 *     Inputs are copied; the caller keeps ownership of every buffer.
 *   - All GPU work is enqueued on the stream given to ewbem_create (borrowed,
 *     never destroyed by the library); calls return when their results are
 *     complete.
 *   - Every call returns EWBEM_OK (0) or a negative status and never aborts;
 *     ewbem_last_error() describes the last failure.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef EWBEM_H
#define EWBEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes */
#define EWBEM_OK 0
#define EWBEM_EINVAL (-1)   /* invalid argument (shape, range, degenerate mesh, NaN) */
#define EWBEM_ENOMEM (-2)   /* device or host allocation failed */
#define EWBEM_EHIP (-3)     /* a HIP runtime call failed */
#define EWBEM_ENOCONV (-4)  /* GMRES reached maxit; outputs hold the best iterate */
#define EWBEM_ESTATE (-5)   /* call out of order (e.g. solve before mesh) or no GPU */

/* ---- operator kinds, storage, windows, preconditioners, guesses */
#define EWBEM_OP_DENSE 0    /* every block dense (no admissible blocks) */
#define EWBEM_OP_HMAT 1     /* hierarchical matrix with ACA far field */
#define EWBEM_STORE_C128 0  /* far factors stored and applied in complex128 */
#define EWBEM_STORE_C64 1   /* far factors stored and applied in complex64 (FP64 accumulation) */
#define EWBEM_WINDOW_NONE 0
#define EWBEM_WINDOW_HANN 1     /* W_k = (1 + cos(2 pi k / N_f)) / 2  (Sec. 3.2) */
#define EWBEM_WINDOW_BLACKMAN 2 /* 0.42 + 0.5 cos(2 pi k/N_f) + 0.08 cos(4 pi k/N_f) */
#define EWBEM_PREC_NONE 0
#define EWBEM_PREC_ELEMENT 1 /* inverse of each element's 3 x 3 diagonal block */
#define EWBEM_PREC_LEAF 2    /* inverse of each leaf cluster's diagonal block */
#define EWBEM_GUESS_ZERO 0
#define EWBEM_GUESS_SEM 1    /* least-squares extrapolation, Sec. 4.2 */
#define EWBEM_GUESS_QUAD 2   /* Lagrange extrapolation 3a1 - 3a2 + a3 */
#define EWBEM_GUESS_LEARNED 3 /* least-squares extrapolation with its part in the learned
                                 basis moved to the trained model's prediction
                                 (ewbem_guess_train) */

typedef struct ewbem_ctx ewbem_ctx; /* opaque, owned by the library */

typedef struct {
  double re, im;
} ewbem_z;

typedef struct {
  int32_t kind;       /* EWBEM_OP_DENSE or EWBEM_OP_HMAT (default HMAT) */
  int32_t leaf_size;  /* max elements per leaf cluster, 1..64 (default 64) */
  double eta_adm;     /* admissibility: min(diam) <= eta * dist (default 1.0) */
  double aca_tol;     /* relative ACA stopping tolerance (default 1e-5) */
  int32_t far_store;  /* EWBEM_STORE_C128 or EWBEM_STORE_C64 (default C128) */
  int32_t self_order; /* polar rule order on the singular element, 4..32 (default 24) */
  int32_t aca_reuse;  /* 1: start each far block's ACA from the rows and columns that gave
                         its pivots at the previously assembled frequency, then continue
                         with ordinary steps until the stopping test holds; 0: from scratch
                         every time (default 1) */
  int32_t autotune;   /* 1: on the first assembled operator (and again after the partition
                         changes), time every pair of matvec task shapes -- 2, 4 or 8 factor
                         columns per phase-1 wavefront, and phase-2 tasks of 1/2048, 1/4096
                         or 1/8192 of all panel columns -- and keep the fastest; 0: 4 and
                         1/4096 (default 1).  The shapes change the summation order only. */
  int32_t aca_batch_mb; /* with far_store C64: 0 approximates every far block at once in
                           complex128 and then converts them (default); > 0 takes the far
                           blocks in index order in batches whose complex128 factors and
                           warm-start work areas need about this many MiB, converting each
                           batch to complex64 as it finishes and reusing its work area, so
                           the complex128 copy never exists for all blocks at once (the
                           meshes whose complex128 far field would not fit).  The factors are
                           the same; only the memory differs.  Not with the pipeline. */
  int32_t mv_mfma;      /* 1: the panel products of a matvec on eight right-hand sides (several
                           loads' lock-step GMRES, the learned guess's training,
                           ewbem_apply_multi) on the FP64 matrix cores, 0: on the vector units
                           (default 1).  The summation order differs, the results agree to
                           rounding. */
  int32_t ws_keep;      /* warm start: 1 (default) keeps every term the core elimination
                           formed, 0 only those up to the first that meets the ACA stopping
                           test.  At least one ordinary step follows either way, with the
                           usual stopping test, and adds what the new frequency needs; 0
                           leaves it more to add (each step reads the block's factors), 1
                           stores a few more terms. */
  double ws_pivot_rel;  /* warm start: the elimination of the cross's core A(I, J) stops at
                           the first pivot whose modulus is at most ws_pivot_rel times the
                           first pivot's; in [0, 1), 0 (default) takes aca_tol.  With ws_keep
                           1 this sets the warm start's rank: a smaller value keeps more
                           terms, a larger one leaves more to the ordinary steps.  (A term's
                           norm |u_t| |v_t| is at least its pivot's modulus.) */
} ewbem_op_opts;

typedef struct {
  double tol;        /* relative residual |b - A x| / |b| target (default 1e-6) */
  int32_t restart;   /* GMRES restart length m, 1..400 (default 100) */
  int32_t maxit;     /* iteration cap per frequency (default 2000) */
  int32_t precond;   /* EWBEM_PREC_* (default EWBEM_PREC_LEAF) */
  int32_t guess;     /* EWBEM_GUESS_* (default EWBEM_GUESS_SEM) */
  int32_t sem_k;     /* K previous solutions used by the guess, 1..8 (default 3) */
  int32_t pipeline;  /* 1: in ewbem_solve_transient, the next frequency's ACA runs on a second
                        stream (library-owned, default priority, from a second host thread)
                        while GMRES solves the current one, into a second factor slot (the
                        far factors' memory doubles); results are unchanged.  0: one
                        frequency after the other (default 0: the overlap gains a few percent
                        on one problem, and several problems solved concurrently already
                        overlap their phases) */
} ewbem_solver_opts;

typedef struct {
  int32_t n_solves;        /* frequencies solved by the call */
  int32_t iters_total;     /* GMRES iterations summed over them */
  int32_t iters_max;
  int32_t matvecs;         /* operator applications (GMRES + guess + residuals) */
  double resid_max;        /* largest final true relative residual */
  double guess_resid_sum;  /* sum of |b - A x0| / |b| of the initial guesses */
  double t_assemble_ms;    /* wall time in operator/RHS/preconditioner assembly (with the
                              pipeline it includes the ACA time that overlapped GMRES) */
  double t_guess_ms;       /* wall time in the initial guess */
  double t_gmres_ms;       /* wall time in GMRES */
  double t_post_ms;        /* wall time in the inverse transform */
  double t_matvec_ms;      /* summed HIP-event time of the matvec kernels */
  double matvec_bytes;     /* algorithmic bytes of one matvec (last operator) */
  double stored_bytes;     /* bytes of the stored operator (near + far) */
  int64_t n_near, n_far;   /* block counts */
  int64_t rank_sum, rank_max; /* far-block ranks of the last operator */
  double t_aca_ms;         /* HIP-event time of the ACA kernels */
  double t_near_ms;        /* HIP-event time of the near-field + self kernels */
  double t_rhs_ms;         /* HIP-event time of the right-hand-side kernels */
  double matvec_bytes_total; /* algorithmic bytes summed over every timed matvec */
  int32_t matvecs_timed;   /* matvecs included in t_matvec_ms */
  int32_t pad0;
  int64_t aca_warm_blocks; /* far blocks whose ACA started from previous pivots */
  int64_t aca_cold_blocks; /* far blocks whose ACA started from scratch (capacity
                              retries, always from scratch, are not counted again) */
  int64_t guess_learned;   /* frequencies whose guess included the network's prediction */
  double pod_energy;       /* ewbem_guess_train: fraction of the training solutions'
                              squared norm inside the reduced basis */
  double train_loss_first; /* ewbem_guess_train: mean squared error of the network on */
  double train_loss_last;  /*   its samples before the first and after the last step */
  int64_t aca_core_blocks[7]; /* warm starts by the size class of the core eliminated (complex
                                 entries of A(I, J)): [5] at most 64 x 64 and [6] at most
                                 128 x 128, in registers; the rest in LDS: [0] at most 2,304,
                                 [1] 4,480, [2] 8,960 entries, [4] at most 64 rows and 1,024
                                 entries; [3] larger or over 128 rows, in global memory */
  int64_t aca_warm_pivots;  /* pivots eliminated in the warm starts' cores, summed */
  int64_t aca_warm_kept;    /* of their terms, those kept (all of them with ws_keep 1), summed */
  int64_t aca_retries;      /* far blocks approximated again with more capacity */
  int64_t aca_steps;        /* lock steps of the ACA after the starts (each adds terms to
                               every still-active block), summed */
  int64_t aca_step_blocks;  /* active blocks summed over those steps */
  int64_t aca_step_first;   /* blocks still active after their start (warm or cold), summed */
} ewbem_stats;

/* Training of the learned initial guess (ewbem_guess_train). */
typedef struct {
  int32_t n_modes;     /* reduced coordinates r: basis size (default 64) */
  int32_t hidden;      /* width of each hidden layer (default 256) */
  int32_t n_hidden;    /* hidden layers, 0..8 (default 3) */
  int32_t epochs;      /* full-batch Adam steps (default 2000) */
  double lr;           /* Adam step size, cosine-decayed to lr / 10 (default 1e-3) */
  int32_t power_iters; /* subspace iterations of the randomized range finder (default 2) */
  int32_t load_kind;   /* 0: each case is nt x 3 tractions; 1: nt pressures (default 0) */
  uint64_t seed;       /* initial weights, the range finder's sketch and the
                          augmentation weights (default 1) */
  int32_t augment;     /* virtual cases per case: random complex combinations of the
                          cases' coordinate sequences (exact, the solution being
                          linear in the load), 0..64 (default 4) */
  int32_t unit_snapshots; /* 1: the basis is the POD of the snapshots scaled to unit
                             norm, so every frequency counts alike (default); 0: of the
                             raw snapshots, which the large low-frequency solutions
                             dominate */
  int32_t lsq_map;     /* 1: the prediction's base is a least-squares map per frequency
                          from the three previous coordinate vectors to the next, fitted
                          over the training loads (regularised, dual form), and the
                          network learns its residual (default); 0: the base is the
                          quadratic extrapolation 3 c1 - 3 c2 + c3 */
  int32_t pad;
  double lsq_reg;      /* the map's regularisation: lam = lsq_reg tr(G) / n with G the
                          n x n Gram matrix of the training histories, (0, 1) (default 1e-8) */
} ewbem_train_opts;

typedef struct {
  int64_t n_elements, n_dof;
  int64_t n_clusters, n_leaves, n_near, n_far;
  int64_t near_entries;    /* complex entries of all dense near blocks */
  int32_t max_leaf, min_leaf;
  int32_t mv_cols;         /* matvec shapes in use: factor columns per phase-1 wavefront */
  int32_t mv_task_div;     /*   phase-2 task size = all panel columns / mv_task_div (>= 96) */
  int32_t mv_tuned;        /*   1 once chosen by timing (ewbem_op_opts.autotune) */
  int32_t mv_tune_cached;  /*   1 when taken from an earlier context of the process on the
                                same device and partition (unknowns, block counts and sizes,
                                factor storage), which timed them: tuned once per problem */
  double mv_tune_best_ms;    /* tuning: one matvec with the chosen shapes, and with the */
  double mv_tune_default_ms; /*   default ones (4, 4096), on the operator it ran on; 0 before */
  int64_t lib_device_bytes;  /* device memory held by the library's buffers, summed over every
                                context of the process (the allocation-free entry point's
                                static array excluded) */
  int64_t far_work_bytes;    /* of this context: the far factors' work areas (complex128 at
                                their capacity, both slots and the retry buffers) and the
                                complex64 store */
  int64_t aca_scratch_bytes; /* of this context: the warm start's cross, substitution panels
                                and norm partials, the ordinary steps' partials */
} ewbem_info_t;

/* Fill option structs with their defaults. */
void ewbem_default_op_opts(ewbem_op_opts* o);
void ewbem_default_solver_opts(ewbem_solver_opts* o);
void ewbem_default_train_opts(ewbem_train_opts* o);

/* Create a context on GPU ``device`` enqueuing on ``hip_stream`` (a
 * hipStream_t, borrowed; NULL = the null stream).  device = -1 creates a
 * host-only context: mesh, tree and partition queries work, every GPU call
 * returns EWBEM_ESTATE. */
int ewbem_create(ewbem_ctx** out, int32_t device, void* hip_stream);
void ewbem_destroy(ewbem_ctx* ctx);
/* Message of the last failure on ctx (valid until the next call on it). */
const char* ewbem_last_error(const ewbem_ctx* ctx);

/* Sec. 2.1: boundary mesh of flat triangles.  xyz: host, nv x 3 doubles;
 * tri: host, nt x 3 vertex indices, counter-clockwise seen from outside each
 * closed surface.  exterior = 1: the solid lies outside the surfaces
 * (cavities), so the outward normal of the solid points into them;
 * exterior = 0: a bounded solid.  EINVAL on bad indices or zero-area
 * triangles. */
int ewbem_set_mesh(ewbem_ctx* ctx, int64_t nv, const double* xyz, int64_t nt,
                   const int32_t* tri, int32_t exterior);

/* Sec. 2.1: density rho, shear modulus mu, Poisson ratio nu (c_s, c_p follow). */
int ewbem_set_material(ewbem_ctx* ctx, double rho, double mu, double nu);

/* Sec. 2.2 / 3.1: period T, N_f samples (even, >= 2; dt = T / N_f),
 * damping sigma >= 0 of the exponential window, spectral window
 * EWBEM_WINDOW_*. */
int ewbem_set_time(ewbem_ctx* ctx, double period, int32_t n_f, double sigma, int32_t window);

/* Sec. 2.1 / 2.2: traction load t(x, t) = t0(x) P(t).  t0: host, nt x 3
 * (caller order); history: host, n_f samples P(n dt). */
int ewbem_set_load_traction(ewbem_ctx* ctx, const double* t0, const double* history);

/* Pressure load: t0 = -p n on each element (n pointing out of the solid), so
 * p > 0 pushes on the solid.  p: host, nt values; history: host, n_f. */
int ewbem_set_load_pressure(ewbem_ctx* ctx, const double* p, const double* history);

/* Sec. 2.1, eq. Aa_b (mixed boundary conditions): bc (host, nt): 0 = the
 * element's traction is given, 1 = its displacement is given (fixed: the
 * given displacement must be zero, else EINVAL).  values (host, nt x 3):
 * the given traction (bc 0) or zero (bc 1); history (host, n_f samples).
 * The unknowns, and the outputs of the solve calls, are then the element's
 * displacement for bc 0 and its traction for bc 1. */
int ewbem_set_load_mixed(ewbem_ctx* ctx, const int32_t* bc, const double* values,
                         const double* history);

/* Scattering of a plane S-wave by the cavity (the boundary integral equation
 * of Sec. 2.1 with the scattered field's traction as the given data; every
 * element traction-free).  The incident field is
 *   u_inc(x, t) = pol f(t - dir . x / c_s),  f(t) = (1 - 2a) exp(-a),
 *   a = (pi ricker_fc (t - t0))^2,
 * with f sampled at n dt (ewbem_set_time first).  In the Laplace domain its
 * traction on a surface of normal n (out of the solid) is
 *   t_inc(s) = -(mu s / c_s) F(s) exp(-s dir . x / c_s) (pol (dir . n) + dir (pol . n)),
 * and the load is the scattered-field traction -t_inc at each element's
 * centroid.  The unknowns and every output are the scattered displacement;
 * the total motion is u_sc + u_inc.  dir and pol (host, 3 each) are
 * normalised; EINVAL if either is zero, if they are not orthogonal
 * (|dir . pol| > 1e-9 after normalising), or for ricker_fc <= 0.  Replaces
 * any earlier load. */
int ewbem_set_load_incident_s(ewbem_ctx* ctx, const double* dir, const double* pol, double ricker_fc,
                              double t0);

/* The same plane S-wave in the total-field formulation: with traction-free
 * cavities the total displacement u = u_sc + u_inc solves the integral
 * equation of Sec. 2.1 with the incident displacement as the right-hand
 * side, (c + T) u = u_inc, because u_inc, regular inside every cavity,
 * satisfies T u_inc - U t_inc = (1 - c) u_inc there (Somigliana's identity
 * for the cavities' interior).  b is then u_inc at the collocation points:
 * O(N) per frequency instead of the O(N^2) sum U t_sc.  The unknowns and
 * every output are the total displacement.  The two formulations agree in
 * the limit of refinement, not element by element.  Arguments and errors as
 * for ewbem_set_load_incident_s; ewbem_solve_transient_incident_loads
 * takes the scattered formulation only (ESTATE after this call). */
int ewbem_set_load_incident_s_total(ewbem_ctx* ctx, const double* dir, const double* pol, double ricker_fc,
                                    double t0);

/* The fast operator for A_k (Sec. 4.1 accelerates the matvec with a fast
 * method and names hierarchical matrices as an alternative to its
 * precorrected FFT; this library builds the hierarchical matrix: cluster
 * tree, admissibility min(diam) <= eta_adm dist, ACA far blocks, dense near
 * blocks).  opts (host) is copied (ewbem_default_op_opts gives the
 * defaults).  EINVAL for NULL or a field out of its documented range (the
 * context is then unchanged).  The tree, partition and device state are
 * rebuilt at the next assembly. */
int ewbem_set_operator(ewbem_ctx* ctx, const ewbem_op_opts* opts);
/* The iterative solver (Sec. 5: GMRES with a block-diagonal
 * preconditioner, stopped at a relative residual; Sec. 4.2: the initial
 * guess by extrapolation from the previous frequencies' solutions, eqs.
 * a0, lsem, a0-solution).  opts (host) is copied
 * (ewbem_default_solver_opts gives the defaults).  EINVAL for NULL or a
 * field out of its documented range (the context is then unchanged).  The
 * solver's device buffers are resized at the next solve. */
int ewbem_set_solver(ewbem_ctx* ctx, const ewbem_solver_opts* opts);

/* Sizes of the discretisation, cluster tree and block partition (host). */
int ewbem_info(ewbem_ctx* ctx, ewbem_info_t* info);

/* Cluster tree and partition (host output).  perm (nt): perm[t] = caller
 * element at tree position t.  near, far: 4 int32 per block (row begin,
 * row end, col begin, col end) as tree positions; either may be NULL.
 * Sizes from ewbem_info. */
int ewbem_get_partition(ewbem_ctx* ctx, int32_t* perm, int32_t* near, int32_t* far);

/* Sec. 3.3 (damped DFT): P_k = (1/N_f) sum_n exp(-sigma n dt) P(n dt)
 * exp(-2 pi i n k / N_f), k = 0..N_f/2.  phat: host, N_f/2+1 values. */
int ewbem_load_spectrum(ewbem_ctx* ctx, ewbem_z* phat);

/* Sec. 2.1: point kernels at Laplace parameter s for n pairs: U_ij(x, y)
 * and T_ij(x, y; n(y)) (i = force direction at x, j = component at y).
 * x, y, nrm: device, n x 3; U, T: device, n x 9 row-major (either NULL). */
int ewbem_kernel_eval(ewbem_ctx* ctx, ewbem_z s, int64_t n, const double* x, const double* y,
                      const double* nrm, ewbem_z* U, ewbem_z* T);

/* Sec. 2.1, eq. T u = U t: dense collocation matrices at s.  T (with the
 * free term) and U: device, N x N row-major in caller order (either NULL).
 * Meant for small meshes and parity checks. */
int ewbem_assemble_dense(ewbem_ctx* ctx, ewbem_z s, ewbem_z* T, ewbem_z* U);

/* Sec. 4 (A_k a_k = b_k): assemble the operator A_k = T(s_k), the right-hand
 * side b_k = P_k U(s_k) t0 and the preconditioner at frequency k. */
int ewbem_assemble(ewbem_ctx* ctx, int32_t k, ewbem_stats* stats);

/* y = A_k x with the assembled operator.  x, y: device, N (caller order). */
int ewbem_apply(ewbem_ctx* ctx, const ewbem_z* x, ewbem_z* y);

/* Y(:, j) = A_k X(:, j), j < nrhs, with the assembled operator read once for
 * all columns (the product that the extrapolation over previous solutions,
 * Sec. 4.2, and several loads' GMRES use).  X, Y: device, N x nrhs
 * column-major (column j starts at j N), caller order, owned by the caller;
 * nrhs in 1..8, else EWBEM_EINVAL; X and Y must not overlap.  With
 * ewbem_op_opts.mv_mfma and nrhs = 8 the panel products run on the FP64
 * matrix cores. */
int ewbem_apply_multi(ewbem_ctx* ctx, const ewbem_z* X, int32_t nrhs, ewbem_z* Y);

/* b_k of the assembled frequency.  b: device, N (caller order). */
int ewbem_get_rhs(ewbem_ctx* ctx, ewbem_z* b);

/* Solve A_k a_k = b_k (assembling first if needed).  x0: device, N, or NULL
 * for the configured guess (Sec. 4.2 uses the solutions of the previous
 * frequencies solved on this context); a: device, N.  ENOCONV if maxit is
 * reached (a holds the last iterate). */
int ewbem_solve_frequency(ewbem_ctx* ctx, int32_t k, const ewbem_z* x0, ewbem_z* a,
                          ewbem_stats* stats);

/* The whole path: solve k = 0..N_f/2 in order, then the inverse transform.
 * u: device, N_f x N doubles (time-major); spec: device, (N_f/2+1) x N
 * complex, or NULL. */
int ewbem_solve_transient(ewbem_ctx* ctx, double* u, ewbem_z* spec, ewbem_stats* stats);

/* Several loads on one mesh: t(x, t) = t0_l(x) P(t) for l < n_loads with the
 * history P of the context's current traction or pressure load.  Every
 * frequency's operator, self terms and preconditioner are assembled once
 * and serve all loads, each with its own right-hand side, extrapolation
 * history and GMRES; the right-hand sides of up to eight loads share one
 * kernel evaluation per element pair, and the loads' GMRES run in lock-step
 * groups of up to eight whose matvecs read the operator once for the
 * group.  Each load's result is that of ewbem_solve_transient with that load
 * on the same operators, to rounding.
 * loads: host, n_loads x nt x 3 tractions (pressure 0) or n_loads x nt
 * pressures (pressure 1), caller order.  u: device, n_loads x n_f x N
 * doubles (load-major, each as in ewbem_solve_transient); spec: device,
 * n_loads x (N_f/2+1) x N complex, or NULL.
 * Memory: per load 16 (N_f/2+1) N bytes of off-diagonal sums (times 4 from
 * 4,096 elements on), the extrapolation history and three vectors; per
 * group up to eight Krylov bases of restart + 1 vectors.
 * The learned guess is not used here (the extrapolation alone).  The
 * context's own load is unchanged.  ESTATE without mesh, time grid and a
 * traction or pressure load; ENOCONV as for ewbem_solve_transient. */
int ewbem_solve_transient_loads(ewbem_ctx* ctx, int32_t n_loads, const double* loads, int32_t pressure,
                                double* u, ewbem_z* spec, ewbem_stats* stats);

/* Several incident plane S-waves on one mesh: the scattered field of each
 * wave of unit direction dirs[3l..3l+2] and polarisation pols[3l..3l+2]
 * (normalised here; each polarisation normal to its direction), all with
 * the wavelet of the context's current incident wave
 * (ewbem_set_load_incident_s), as that call defines the load (Sec. 2.1's
 * equation for the scattered field).  Every frequency is assembled once for
 * all waves, as in ewbem_solve_transient_loads; the right-hand sides of up
 * to four waves share one kernel evaluation per element pair.  dirs, pols:
 * host, n_loads x 3.  u, spec and the results as for
 * ewbem_solve_transient_loads: each wave's result is that of
 * ewbem_solve_transient with that wave, to rounding.  ESTATE without mesh,
 * time grid and an incident wave; EINVAL for a zero or non-normal
 * polarisation. */
int ewbem_solve_transient_incident_loads(ewbem_ctx* ctx, int32_t n_loads, const double* dirs,
                                         const double* pols, double* u, ewbem_z* spec, ewbem_stats* stats);

/* An addition to the method (the paper solves one problem at a time; each
 * problem's own path is Sec. 2.2-4 as in ewbem_solve_transient).
 * Several problems at once (one context each, all distinct): up to
 * per_launch of them run concurrently from host threads, each with its
 * whole frequency loop on its own context's stream (contexts created on the
 * same stream serialise).  u_out[i] (device, n_f x 3 nt of context i) as in
 * ewbem_solve_transient.  stats (optional) sums the contexts' counters and
 * times and takes the maxima of resid_max, iters_max and rank_max.  Returns
 * the first hard error of any context, else ENOCONV if any frequency of any
 * context missed the tolerance (its outputs are still written), else OK;
 * EINVAL for null or repeated contexts or per_launch < 1. */
int ewbem_batch_solve_transient(ewbem_ctx** ctxs, int32_t n, double** u_out, ewbem_stats* stats,
                                int32_t per_launch);

/* An addition to the method, like ewbem_batch_solve_transient: the same
 * problems in lock-step over the frequency index, in groups of per_launch.
 * At each k every problem of a group assembles its operator and forms its
 * initial guess on its own library-owned stream (host threads,
 * concurrently); then the group's GMRES run together on one library-owned
 * stream, and every Arnoldi step applies all their operators with one
 * matvec: their task tables concatenated into one launch of each matvec
 * kernel (the phase-1 factor products, the panel products and the fixed-
 * order reduction), captured once per frequency as a HIP graph and replayed
 * each step.  Problems leave the launch as they converge (the graph is
 * rebuilt for the rest).  Each problem's arithmetic is its lone solve's.
 * Requirements: contexts on one device, H-matrix or dense operators whose
 * far factors share one store type, no pipeline; N_f may differ (a problem
 * leaves the lock-step after its last frequency).  Outputs, stats and return
 * codes as for ewbem_batch_solve_transient; EINVAL also for contexts on
 * different devices. */
int ewbem_batch_solve_transient_lockstep(ewbem_ctx** ctxs, int32_t n, double** u_out, ewbem_stats* stats,
                                         int32_t per_launch);

/* ---- Learned initial guess (an addition to the method; Sec. 4.2 supplies
 * the extrapolation it extends).
 *
 * ewbem_guess_train solves the whole frequency sequence for n_cases loads
 * (same mesh, material, time grid, operator and solver settings, and the
 * load history of the context's current traction or pressure load), then
 *   - takes the r dominant left singular directions of all those solutions
 *     (randomized range finder with power_iters subspace iterations on
 *     r + 16 columns, then the exact eigen-decomposition of the sketch):
 *     the basis Phi, N x r with orthonormal columns;
 *   - forms, for every case and k = 3..N_f/2, the reduced coordinates
 *     c_j = Phi^H a_j of the solutions at k-1, k-2, k-3 and at k;
 *   - (lsq_map) fits, for every k, the least-squares map from the history
 *     h = [c_{k-1}; c_{k-2}; c_{k-3}] to c_k over the n_cases loads in its
 *     dual form: X_k = [h_1 .. h_n], A = (X_k^H X_k + lam I)^{-1},
 *     lam = lsq_reg tr(X_k^H X_k) / n, W_k = [c_k of each case] A, so the
 *     map is c_k ~ W_k X_k^H h (a combination of the training loads'
 *     outcomes, the solution being linear in the load); its prediction of
 *     each training case is the base the network corrects (else the base is
 *     3 c_{k-1} - 3 c_{k-2} + c_{k-3});
 *   - the network's input is [Re, Im of c_{k-1}, c_{k-2}, c_{k-3}] / nu with
 *     nu = |c_{k-1}|, followed by f and f^2 (f = k / (N_f/2)); its target is
 *     [Re, Im of c_k - base] / nu; the samples also come from augment x
 *     n_cases virtual cases, each a combination of the cases' coordinate
 *     sequences (and bases) with complex N(0, 1/n_cases) weights;
 *   - fits a network of n_hidden GELU layers of width hidden (bf16 weights
 *     and activations in the products, fp32 accumulation) by full-batch Adam
 *     on the mean squared error.
 * With EWBEM_GUESS_LEARNED, frequency k >= 3 then takes the least-squares
 * extrapolation x (residual r) and moves its part in the basis to the
 * prediction p = base + nu y (y: network output, base the map's W_k X_k^H h
 * when the model was fitted for the context's N_f, else the quadratic
 * extrapolation) along v = Phi (p - Phi^H x) by the step gamma that
 * minimises |r - gamma A v| (one more operator application), so the guess
 * is never worse in residual than the extrapolation alone; k < 3 uses the
 * extrapolation alone.  The context's own load is
 * unchanged (the training loads run through the multi-load loop of
 * ewbem_solve_transient_loads).  loads: host, n_cases x nt x 3 tractions
 * (load_kind 0) or n_cases x nt pressures (1), caller order.  stats sum the
 * training solves and report pod_energy and the fit's losses.  ESTATE
 * without mesh, time grid and a traction or pressure load; EINVAL if
 * N_f < 6, n_modes exceeds the snapshots n_cases (N_f/2 + 1) or N, or there
 * are more than 65535 snapshots.  ENOCONV if a training solve missed the
 * tolerance (the model is still fitted).  A new mesh drops the model. */
int ewbem_guess_train(ewbem_ctx* ctx, int32_t n_cases, const double* loads, const ewbem_train_opts* opts,
                      ewbem_stats* stats);

/* Serialise the model (basis in caller order, network, least-squares map)
 * into buf (host).  buf = NULL: *len receives the size.  EINVAL if *len is
 * too small (then *len is the size needed); ESTATE without a model.  Layout:
 * 8 bytes "EWBGUESS"; int32 version 2, N, r, L; int32 widths dims[0..L];
 * fp64 pod energy, first and last training loss; fp32 parameters (per layer
 * W_l row-major dims[l+1] x dims[l], then b_l); complex128 basis N x r
 * column-major; int32 n (training loads of the map, 0 for none) and K (the
 * frequency count N_f/2 + 1 it was fitted for, 0 for none); complex128 X_k
 * (3r x n, column-major) for k = 3..K-1, then W_k (r x n) for k = 3..K-1.
 * All little-endian, no padding.  ewbem_guess_load also reads version 1,
 * which ends after the basis (no map). */
int ewbem_guess_save(const ewbem_ctx* ctx, void* buf, size_t* len);

/* Load a model written by ewbem_guess_save (host buffer of len bytes) for
 * a mesh with the same number of unknowns.  EINVAL on a malformed or
 * mismatched buffer; ESTATE without a mesh.  Host-only contexts accept it. */
int ewbem_guess_load(ewbem_ctx* ctx, const void* buf, size_t len);

/* The model's basis size (n_modes, may be NULL) and basis (phi: device,
 * N x r complex column-major in caller order, or NULL). */
int ewbem_guess_basis(ewbem_ctx* ctx, int32_t* n_modes, ewbem_z* phi);

/* The network's kernels on caller data (all arrays device fp32, row-major):
 * n_layers layers of widths dims[0..n_layers] (host), GELU after all but the
 * last, params laid out as in the saved model.  ewbem_mlp_eval: y (batch x
 * dims[L]) = net(x) (x: batch x dims[0]); with target (batch x dims[L]):
 * loss = mean of (y - target)^2 over all batch dims[L] entries and, if grad
 * is given, grad = d loss / d params.  batch = 0 writes nothing (grad zero,
 * loss 0).  ewbem_mlp_train: epochs full-batch Adam steps (beta 0.9, 0.999,
 * eps 1e-8, constant step lr) on that loss, params updated in place;
 * loss_first / loss_last (optional) before the first and after the last
 * step. */
int ewbem_mlp_eval(ewbem_ctx* ctx, int32_t n_layers, const int32_t* dims, const float* params, int64_t batch,
                   const float* x, const float* target, float* y, float* grad, double* loss);
int ewbem_mlp_train(ewbem_ctx* ctx, int32_t n_layers, const int32_t* dims, float* params, int64_t batch,
                    const float* x, const float* target, int32_t epochs, double lr, double* loss_first,
                    double* loss_last);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as ewbem_mlp_eval, with the same arguments and results, that
 * allocates nothing.  Its activations, pre-activations, output gradient,
 * backward work area and loss partials live in one statically sized array
 * of 32 MiB per GPU (held from the first context on that GPU until the
 * process ends), so it needs 2 batch sum(hidden widths) + [target] (batch
 * dims[L] + 256 x 2) + [grad] 2 batch max(width) floats, each part rounded
 * up to 256 bytes, within 32 MiB; larger requests return EINVAL before any
 * work is enqueued.  Every call on a GPU shares that array and leaves its
 * contents behind (nothing there needs clearing: each call writes before it
 * reads), so calls that overlap on one GPU (several host threads, or
 * several streams in flight) race and must be serialised by the caller. */
int ewbem_mlp_eval_noalloc(ewbem_ctx* ctx, int32_t n_layers, const int32_t* dims, const float* params,
                           int64_t batch, const float* x, const float* target, float* y, float* grad,
                           double* loss);

/* Sec. 3.3 (inverse): u(n dt) = Re{exp(sigma n dt) sum_k W_k a_k
 * exp(2 pi i n k / N_f)} with a_{N_f-k} = conj(a_k).  spec: device,
 * (N_f/2+1) x N complex (caller order); u: device, N_f x N doubles. */
int ewbem_mft_inverse(ewbem_ctx* ctx, const ewbem_z* spec, double* u);

#ifdef __cplusplus
}
#endif

#endif /* EWBEM_H */
