/*
 * helm.h -- C ABI of the MI355X shifted-HSS Helmholtz solver.
 *
 * Problem (Sec. 2 of Cotter, Hope-Collins and Knook, "Shifted HSS solvers
 * for the indefinite Helmholtz equation"):  find u in the CG1/Q1 space with
 *
 *     b_delta(u, v) = G[v]  for all v,
 *     b_delta(u, v) = int (-delta + ik)^2 u v* + grad u . grad v*
 *                     - (-delta + ik) int_Gamma u v*,
 *
 * on the unit square (P1 triangles, every cell split along the diagonal
 * from (x_i, y_j) to (x_i+1, y_j+1)) or the unit cube (Q1 hexahedra), with
 * Sommerfeld conditions on Gamma = the whole boundary.  delta >= 0, k > 0.
 *
 * Method: right-preconditioned flexible GMRES in complex FP64 on B_0 (or
 * B_delta), preconditioned by the shifted-HSS preconditioner of Sec. 4
 * (Definition "Shifted HSS iteration for the primal system",
 * eq. (HSSpc primal)) with delta replaced by delta_hat > delta:
 * m*ceil(k) gamma=k HSS steps from u_0 = 0, each inner solve with
 *     L = K + (dh^2 - k^2 - 2i dh k^2) M + (dh - i k^2) M_Gamma
 * approximated by q geometric-multigrid V(nu1,nu2) cycles (q >= 2, chosen
 * per handle from the measured cycle rate unless helm_opts.mg_cycles sets
 * it) with scaled Jacobi smoothing (Sec. 5.3), FE interpolation / its
 * transpose as transfers, and an FP64 dense solve on the coarsest mesh.
 *
 * Data layout (all vectors): complex, interleaved (re, im), one column per
 * right-hand side, column-major [nrhs][N]; nodes lexicographic,
 * node (i, j[, l]) at index i + (n+1) (j + (n+1) l), N = (n+1)^dim.
 * The mixed element (HELM_MIXED_DG0_P1) appends the triangle values of
 * sigma to every column of rhs, x and the preconditioner's vectors:
 * columns of helm_vector_length(h) = N + 4 n^2 values.
 * FP64 vectors are double2, FP32 vectors float2.  Every vector pointer
 * passed to this library is a DEVICE pointer on the device current when
 * helm_create was called; the caller owns it and it is not retained after
 * the call returns.
 *
 * Streams: all device work is ordered on the stream given to helm_create.
 * Calls that report host-visible results (helm_solve) synchronise that
 * stream before returning; the per-step calls only enqueue work.
 * A handle is not thread-safe; distinct handles are independent.
 *
 * Errors: every call returns HELM_OK (0) or a negative HELM_E* code; no
 * exception crosses the ABI; helm_strerror names the code.
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define HELM_OK        0
#define HELM_EINVAL   (-1)  /* invalid argument (sizes, parameters, null)  */
#define HELM_ENOMEM   (-2)  /* host or device allocation failed            */
#define HELM_EDEVICE  (-3)  /* HIP runtime error                           */
#define HELM_ENOCONV  (-4)  /* max_outer reached before the tolerance      */
#define HELM_ENOTSUP  (-5)  /* valid request this build does not implement */

/* ---- mesh / element kinds ---------------------------------------------- */
#define HELM_P1_TRI_RIGHT 1  /* 2D, right-diagonal P1 triangles */
#define HELM_Q1_HEX       2  /* 3D, trilinear hexahedra          */
#define HELM_MIXED_DG0_P1 3  /* 2D mixed formulation of Sec. 2: sigma in
                                [DG0]^2, u in P1 on the right-diagonal mesh.
                                Vectors are [u | sigma]: u at the N nodes,
                                then sigma on the 2 n^2 triangles, triangle
                                e = t n^2 + (p + n q) of cell (p, q) (t = 0:
                                (p,q),(p+1,q),(p+1,q+1); t = 1:
                                (p,q),(p+1,q+1),(p,q+1)), its x and y
                                components at 2e and 2e + 1: N + 4 n^2
                                complex values per column
                                (helm_vector_length)                     */

/* ---- precision modes ---------------------------------------------------- */
#define HELM_FP64     0  /* everything in complex FP64                       */
#define HELM_FP32_MG  1  /* HSS sweeps and V-cycles in complex FP32 (FP32
                            accumulation); outer FGMRES, Arnoldi and the
                            coarsest-mesh solve stay FP64                    */

/* ---- outer iterations (helm_opts.outer) ---------------------------------- */
#define HELM_OUTER_FGMRES      0  /* flexible right-preconditioned GMRES (Sec. 5.1) */
#define HELM_OUTER_RICHARDSON  1  /* preconditioned Richardson, the stationary
                                     iteration of Sec. 4:
                                     x <- x + B~^{-1} (rhs - B x)              */

/* ---- multigrid cycles (helm_opts.cycle) ---------------------------------- */
#define HELM_CYCLE_V_JACOBI   0  /* V(2,2) cycles, scaled Jacobi omega, FP64
                                    dense solve on the coarsest mesh          */
#define HELM_CYCLE_W_GMRES    1  /* the paper's variant (Sec. 5.3): W-cycle
                                    whose smoother on every level, the
                                    coarsest included, is smooth_its
                                    iterations of Jacobi-left-preconditioned
                                    GMRES; no coarse factorisation          */

/* ---- operators for helm_apply (all a K + b M + c M_Gamma) --------------- */
#define HELM_OP_B0      0  /* b_0: K - k^2 M - i k M_Gamma (Sec. 2, delta = 0) */
#define HELM_OP_BDELTA  1  /* b_delta with the handle's delta                 */
#define HELM_OP_BSHIFT  2  /* b_delta_hat                                    */
#define HELM_OP_L       3  /* L of eq. (HSSpc primal), left-hand side        */
#define HELM_OP_N       4  /* N of eq. (HSSpc primal), right-hand operator   */
#define HELM_OP_H       5  /* Gram matrix of the H_primal inner product
                              (Sec. 3.1) with delta_hat: 2 dh k M + k M_Gamma */
#define HELM_OP_M       6  /* mass matrix                                    */
#define HELM_OP_MIXED   7  /* mixed handles, level 0, FP64: the mixed
                              operator A_delta on [u | sigma] (Sec. 2)      */
#define HELM_OP_MIXED_SHIFT 8  /* mixed handles: A_delta_hat                */

typedef struct helm_s helm_t;

typedef struct {
    int dim;     /* 2 or 3                                                  */
    int elem;    /* HELM_P1_TRI_RIGHT (dim 2) or HELM_Q1_HEX (dim 3)         */
    int n;       /* cells per side on the finest mesh, >= 2                  */
    int levels;  /* multigrid levels >= 1; n divisible by 2^(levels-1) and
                    the coarsest mesh n/2^(levels-1) >= 1                    */
} helm_mesh;

typedef struct {
    /* Bit f set means face f carries u = 0 (Dirichlet) instead of the
       impedance (Sommerfeld) condition of Sec. 2: x0=1, x1=2, y0=4, y1=8,
       z0=16, z1=32 (only the first four in 2D).  The nodes of those faces
       are not unknowns: every operator keeps the rows and columns of the
       other nodes (the impedance term lives on the remaining faces) and
       acts as the identity on Dirichlet nodes, the prolongation P drops
       them on both levels, and the coarsest-mesh matrix gets identity rows
       and columns there.  Every vector a call writes is zero on Dirichlet
       nodes; vectors passed to the per-step calls must be zero there too
       (helm_solve, helm_precondition and helm_hss_history take their
       inputs as zero there themselves).  Primal P1/Q1 element with V
       cycles only. */
    unsigned dirichlet_faces;
} helm_bc;

typedef struct {
    int    precision;  /* HELM_FP64 (default) or HELM_FP32_MG               */
    int    nu1, nu2;   /* pre/post Jacobi sweeps; this build needs 2, 2      */
    double omega;      /* Jacobi damping, default 2/3                        */
    int    hss_m;      /* m in m*ceil(k) HSS steps, default 1                */
    int    hss_steps;  /* if > 0, overrides m*ceil(k)                        */
    int    restart;    /* FGMRES basis size; 0 = 3*ceil(k) + 30, max 2000    */
    int    max_outer;  /* outer iteration cap; 0 = 4 * restart               */
    int    x0_given;   /* 1: x holds the initial guess on entry, else x0 = 0 */
    int    profile;    /* 1: time the finest-level smoothing launches of
                          every tenth HSS step with HIP events (2D: the
                          four-sweep passes; 3D: each Jacobi sweep; fills
                          the sweep_* stats).  A timed solve runs its
                          preconditioner eagerly, without the captured
                          graphs                                            */
    int    mg_cycles;  /* V-cycles per inner HSS solve (each after the first
                          starts from the previous iterate).  0 = automatic:
                          with exact inner solves the HSS error contracts by
                          (k-1)/(k+1) per step (Sec. 3.1 proposition); an
                          inexact solve with error E changes the step's map T
                          to T + E (I - T), still a contraction when
                          |E| < (1 - nu)/(1 + nu) = 1/k; the library measures
                          the V-cycle rate rho_V once (power iteration) and
                          uses the smallest q >= 2 with rho_V^q <= 1/k
                          (mixed form: <= 1/n, since sigma is recovered from
                          the gradient of u, which magnifies a u error by
                          ~1/(h k))                                          */
    int    no_graphs;  /* 1: launch the preconditioner's kernels one by one;
                          default 0 replays one captured HIP graph of the
                          whole HSS loop per application (captured on a
                          private stream, launched on the handle's stream)  */
    int    no_small;   /* 1: run every 2D level with per-level kernels; by
                          default the levels from the first one whose
                          vectors fit one workgroup's LDS down to the
                          coarsest run as one LDS-resident kernel per cycle  */
    int    verbose;    /* > 0: print the Arnoldi residual estimate to stderr
                          every `verbose` outer iterations                   */
    int    no_stream;  /* 1: run the large 2D levels with the LDS-tiled
                          kernels and every 3D level with one thread per
                          node; by default the 2D levels >= 16^2 run with
                          the register-streaming kernels (one wavefront
                          marches up a strip of 64 columns, every sweep a
                          pipeline stage one row behind the previous one)
                          and the 3D levels >= 128^3 with the z-marching
                          column-tile kernel                                 */
    int    full_reorth; /* 1: classical Gram-Schmidt twice at every Arnoldi
                          step; by default the second pass runs only for
                          the columns whose first pass kept less than
                          1/sqrt(50) ~ 0.14 of the new vector's norm (the
                          Kahan-Parlett test: one pass leaves an
                          orthogonality error of ~eps times the inverse of
                          that fraction; estimated as |w|^2 - |h|^2 on the
                          device, no host synchronisation)                  */
    int    split;      /* 1: with two or more columns, split them into two
                          groups whose HSS loops run on two streams (one
                          group's finest-level passes can overlap the
                          other's latency-bound coarse levels); by default
                          all columns run as one batch on one stream        */
    int    outer;      /* HELM_OUTER_FGMRES (default) or HELM_OUTER_RICHARDSON.
                          Richardson computes the true residual of every
                          column each iteration and stops a column once it
                          meets the tolerance (restart is ignored; max_outer
                          = 0 means 4 * (3*ceil(k) + 30))                    */
    int    cycle;      /* HELM_CYCLE_V_JACOBI (default) or HELM_CYCLE_W_GMRES.
                          The W variant needs HELM_FP64, runs its kernels
                          one by one (no captured graph), uses mg_cycles
                          W-cycles per HSS step (0 = 1, the paper's choice)
                          and places no limit on the coarsest mesh size    */
    int    smooth_its; /* GMRES iterations per smoothing of the W variant,
                          1..20; 0 = 5 (the paper's primal setting)         */
} helm_opts;

typedef struct {
    int    outer_its;            /* FGMRES iterations (max over columns)     */
    int    restarts;             /* restart cycles performed                 */
    int    hss_steps;            /* HSS steps per preconditioner application */
    long long vcycles;           /* V-cycles applied, summed over columns    */
    int    converged;            /* 1 if every column met the tolerance      */
    double arnoldi_rel_residual; /* max over columns, last Arnoldi estimate  */
    double true_rel_residual;    /* max over columns of ||b - B x|| / ||b||,
                                    recomputed in FP64 after convergence     */
    double solve_ms;             /* wall time of helm_solve                  */
    double precond_ms;           /* device time inside the preconditioner    */
    double sweep_ms;             /* profile=1: summed device time of the
                                    timed smoothing launches (see profile)    */
    long long sweep_launches;    /* profile=1: number of timed launches       */
    double sweep_bytes;          /* profile=1: algorithmic bytes they move per
                                    right-hand side: x and b read, x' written;
                                    2D adds the coarse correction read and the
                                    coarse residual written (a quarter vector
                                    each)                                      */
    int    mg_cycles;            /* V-cycles per inner HSS solve used          */
    double vcycle_rate;          /* measured V-cycle contraction (automatic
                                    mode; 0 when mg_cycles was given)         */
    long long reorth_passes;     /* second Gram-Schmidt passes run, summed
                                    over columns and iterations               */
    double outer_rate;           /* average outer contraction per iteration,
                                    (|r_J| / |r_0|)^(1/J) from the true
                                    residuals before the first and after the
                                    last of a column's J iterations (the
                                    measured rate of Sec. 5.2's tables); max
                                    over columns with J >= 1, else 0         */
} helm_stats;

/* Fill *opts with the defaults listed above. */
void helm_opts_default(helm_opts* opts);

/* Name of a status code (static string). */
const char* helm_strerror(int status);

/* Detail of the last HIP error seen on the calling thread ("" if none);
 * valid until the next call on that thread. */
const char* helm_last_error(void);

/*
 * Build a solver for one mesh and parameter set.
 *   k > 0, delta >= 0, delta_hat > delta: the problem and the shift
 *     (Sec. 2 and Sec. 4; delta_hat > delta as in the shift-preconditioning
 *     iteration of Sec. 4).
 *   bc: NULL means Sommerfeld on every face.
 *   opts: NULL means helm_opts_default.
 *   hip_stream: a hipStream_t (NULL = the null stream), owned by the caller.
 * Builds the level table (n_l = n / 2^l), the per-level operator
 * coefficients, and the coarsest-mesh FP64 inverse of L (host LU, uploaded
 * once).  The handle owns only these (kilobytes to a few MB); solve-time
 * vectors live in the caller's workspace.
 * Errors: HELM_EINVAL for dim not in {2,3}, elem/dim mismatch, n < 2,
 * levels < 1, n not divisible by 2^(levels-1), k <= 0, delta < 0,
 * delta_hat <= delta, hss_m < 1, omega not in (0, 2), out == NULL, an
 * unknown outer or cycle, smooth_its outside 0..20, or (V cycles) a
 * coarsest mesh with more than 4096 nodes, or dirichlet_faces bits beyond
 * the 2 dim faces; HELM_ENOTSUP for Dirichlet faces with the mixed element or the
 * W variant, (nu1, nu2) != (2, 2) with V cycles, or the W variant with
 * HELM_FP32_MG or with the mixed element; HELM_ENOMEM; HELM_EDEVICE.
 * On error *out is set to NULL and nothing is leaked.
 */
int helm_create(const helm_mesh* mesh, double k, double delta, double delta_hat,
                const helm_bc* bc, const helm_opts* opts, void* hip_stream,
                helm_t** out);

/* Release the handle (NULL is accepted). Synchronises its stream first. */
int helm_destroy(helm_t* h);

/* Number of nodes N on the finest mesh, and on level l (0 = finest). */
long long helm_nodes(const helm_t* h, int level);

/* Complex values per column of rhs and x: N, or N + 4 n^2 for
 * HELM_MIXED_DG0_P1 (-1 for NULL). */
long long helm_vector_length(const helm_t* h);

/*
 * Bytes of device workspace helm_solve / helm_precondition / helm_vcycle
 * need for nrhs columns (256-byte aligned base required).  nrhs >= 1.
 */
int helm_workspace_bytes(const helm_t* h, int nrhs, size_t* bytes);

/*
 * Solve B_delta x = rhs for nrhs columns (B_0 when delta = 0), to
 * ||rhs - B x||_2 <= tol ||rhs||_2 per column (Sec. 5.1's relative
 * tolerance; the true residual is recomputed in FP64 at the end).
 *   rhs, x: device, complex FP64 [nrhs][helm_vector_length(h)]; rhs is an
 *     assembled load vector (the preconditioner maps the dual space to the
 *     primal space, Sec. 4), e.g. from helm_load_nodal.  Mixed element:
 *     the mixed system A_delta [u | sigma] = rhs.
 *   workspace: device, helm_workspace_bytes(h, nrhs) bytes.
 *   stats: may be NULL.
 * Returns HELM_OK, or HELM_ENOCONV with x holding the last iterate when
 * max_outer is reached; HELM_EINVAL for tol not in (0, 1), nrhs < 1, NULL
 * pointers, or a non-finite rhs norm.  A zero column gives x = 0.
 */
int helm_solve(helm_t* h, const void* rhs, void* x, int nrhs, double tol,
               void* workspace, helm_stats* stats);

/*
 * b = M f for nodal source values f (real FP64 [nrhs][N]): the load vector
 * of the nodal interpolant of f.  b: device complex FP64 [nrhs][N]; for the
 * mixed element b = [M f / (delta - ik) | 0], [nrhs][N + 4 n^2] (the mixed
 * right-hand side of Sec. 2).
 */
int helm_load_nodal(helm_t* h, const double* f_nodal, void* b, int nrhs);

/* ---- the steps of the hot path, exposed one by one ----------------------
 * prec selects the vector type of x/y/b arguments: HELM_FP64 (double2) or
 * HELM_FP32_MG (float2).  Level l meshes have n / 2^l cells per side.
 * These calls only enqueue work on the handle's stream.
 */

/* y = Op x on level l (Op one of HELM_OP_*), matrix-free. */
int helm_apply(helm_t* h, int op, int level, int prec,
               const void* x, void* y, int nrhs);

/* HSS residual of the correction form of eq. (HSSpc primal) on level 0:
 * rho = (2k/(k+1)) (R - B_shift u).  u == NULL means u = 0. */
int helm_hss_residual(helm_t* h, int prec, const void* R, const void* u,
                      void* rho, int nrhs);

/* One scaled-Jacobi sweep for L on level l (D = diag L):
 * x_out = x_in + omega D^{-1} (b - L x_in); x_in == NULL means x_in = 0.
 * x_out must not alias x_in or b. */
int helm_jacobi(helm_t* h, int level, int prec, const void* x_in,
                const void* b, void* x_out, int nrhs);

/* Residual restriction: b_c = P^T (b - L x) from level l to level l+1. */
int helm_restrict_residual(helm_t* h, int level, int prec, const void* x,
                           const void* b, void* b_coarse, int nrhs);

/* Prolongation and correction: x += P e_c from level l+1 to level l. */
int helm_prolong_correct(helm_t* h, int level, int prec, const void* e_coarse,
                         void* x, int nrhs);

/* Coarsest-mesh solve x = L_c^{-1} b in FP64 arithmetic whatever prec
 * (HELM_ENOTSUP with HELM_CYCLE_W_GMRES, which has no coarse solve). */
int helm_coarse_solve(helm_t* h, int prec, const void* b, void* x, int nrhs);

/* One multigrid cycle for L on level 0 with zero initial guess: V(nu1, nu2)
 * Jacobi, or with HELM_CYCLE_W_GMRES one W-cycle of the paper's variant. */
int helm_vcycle(helm_t* h, int prec, const void* b, void* x, int nrhs,
                void* workspace);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the cycle
 * of helm_vcycle with the level vectors in a scratch array the library
 * holds on each device (HELM_NOALLOC_SCRATCH_BYTES, kept until the process
 * ends) instead of a workspace.  It calls no hipMalloc, hipFree or other
 * allocating routine; segment heights not measured yet on this thread come
 * from the library's model (no timing launches).  Same arguments, layout
 * and result as helm_vcycle, bit for bit; b and x are device vectors on
 * the current device, which must be the handle's.  Every call on a device
 * shares that device's scratch: calls that overlap on one device (two
 * streams, two threads) race and give wrong results.  The scratch needs no
 * clearing (every level vector is written before it is read).
 * Errors: HELM_EINVAL for the arguments helm_vcycle rejects, a current
 * device other than the handle's, or a mesh and column count whose level
 * vectors exceed HELM_NOALLOC_SCRATCH_BYTES (helm_last_error gives the
 * bytes needed); HELM_ENOTSUP with HELM_CYCLE_W_GMRES; HELM_EDEVICE. */
#define HELM_NOALLOC_SCRATCH_BYTES (64u << 20)
int helm_vcycle_noalloc(helm_t* h, int prec, const void* b, void* x, int nrhs);

/* Shifted-HSS preconditioner z = B~^{-1} v (Definition "Shifted HSS
 * iteration for the primal system"), correction form, in the handle's
 * precision mode.  v, z: complex FP64 [nrhs][helm_vector_length(h)]; the
 * mixed element applies the mixed preconditioner (Definition "Shifted HSS
 * preconditioner for the mixed system", sigma eliminated in every step). */
int helm_precondition(helm_t* h, const void* v, void* z, int nrhs,
                      void* workspace);

/* The preconditioner of helm_precondition with the HSS residual recorded:
 * after HSS step s (s = 1 .. hss_steps) of column c,
 *   res[c * (hss_steps + 1) + s] = ||v_c - B_shift u_s||_2
 * (the mixed element: ||v_c - A_delta_hat U_s||_2),
 * and res[c * (hss_steps + 1)] = ||v_c||_2, all in FP64 arithmetic on the
 * iterate u_s in the handle's precision mode (the residual contraction of
 * the HSS iteration that Sec. 5.2 reports as the measured rate).  The
 * steps run eagerly (no captured graph) with one extra residual pass and
 * one device->host copy each, so this is a diagnostic, not the fast path;
 * z receives the same result as helm_precondition.
 *   res: host, nrhs * (hss_steps + 1) doubles, caller-owned.
 * Errors: HELM_EINVAL for NULL pointers or nrhs < 1; HELM_EDEVICE. */
int helm_hss_history(helm_t* h, const void* v, void* z, int nrhs, void* workspace,
                     double* res);

/* ---- serving: continuous batching of independent solves -----------------
 * A server solves a stream of requests (one mesh, k, delta_hat and a set of
 * right-hand sides each).  Requests with the same mesh and parameters form a
 * group that shares one solver handle, one device workspace of `max_cols`
 * column slots and one stream (another group of the same parameters is
 * created when one is full); every column owns a slot (its own Krylov
 * basis and iterate).  All columns of a group advance by one outer FGMRES
 * iteration in the same kernel launches, and every group runs on its own
 * stream at its own pace: helm_server_step polls the groups' in-flight
 * iterations and, for each group whose iteration has finished on the
 * device, completes it on the host, copies out its finished requests,
 * admits queued requests into its free slots and enqueues its next
 * iteration at once, while the other groups keep running; it returns once
 * at least one group has advanced (or no group has work).  Groups are
 * created while their workspace fits the HBM budget (computed from the
 * sizes before anything is built) and idle groups are released when space
 * is needed.  A column's arithmetic does not depend on which other columns
 * share its launches, so a request's result is the same alone and in the
 * mix.
 * The server allocates its workspaces itself (hipMalloc) and owns its
 * streams.  Not thread-safe.
 */
typedef struct helm_server_s helm_server_t;

typedef struct {
    double hbm_budget_bytes;  /* device memory for group workspaces (> 0)      */
    int    max_cols;          /* column slots per group (>= 1)                 */
    int    precision;         /* HELM_FP64 or HELM_FP32_MG                     */
    int    restart;           /* FGMRES basis per column; 0 = 3 ceil(k) + 30   */
    int    max_outer;         /* 0 = 4 * restart                               */
} helm_server_opts;

typedef struct {
    int    status;            /* 0 queued, 1 running, 2 done                   */
    int    converged;         /* every column met its tolerance                */
    int    outer_its;         /* max over the request's columns                */
    double true_rel_residual; /* max over its columns                          */
    double t_submit, t_admit, t_done;  /* seconds since helm_server_create     */
} helm_request_info;

int helm_server_create(const helm_server_opts* opts, helm_server_t** out);

/* Queue a request: solve B_0 x = rhs for nrhs columns on the dim-D unit
 * domain with n cells per side and `levels` multigrid levels, wavenumber k,
 * shift delta_hat.  rhs, x: device, complex FP64 [nrhs][N], caller-owned;
 * rhs must stay valid until the request is admitted, x until it is done.
 * Errors: HELM_EINVAL for invalid sizes or parameters (as helm_create), or
 * nrhs > max_cols (the request could never be admitted). */
int helm_server_submit(helm_server_t* s, int dim, int n, int levels, double k, double delta_hat,
                       const void* rhs, void* x, int nrhs, double tol, long long* id);

/* Advance the groups whose iterations have finished (see above) plus
 * admission; *n_done (nullable) receives the number of requests completed
 * by this call. */
int helm_server_step(helm_server_t* s, int* n_done);

int helm_server_query(const helm_server_t* s, long long id, helm_request_info* info);

/* Queued and running request counts and device bytes held in workspaces. */
int helm_server_load(const helm_server_t* s, int* queued, int* running, double* bytes_in_use);

int helm_server_destroy(helm_server_t* s);

#ifdef __cplusplus
}
#endif

#endif /* HELM_H */
