/*
 * rp4d.h -- C ABI of the MI355X (gfx950) randomized-preconditioned SC-4DVAR hot path.
 *
 * The operations follow Subrahmanya, Rao, Saibaba, "Randomized Preconditioned
 * Solvers for Strong Constraint 4D-Var Data Assimilation" (arXiv:2401.15758):
 *   model / TLM / ADJ            Sec. 2.1 eq. (model), Sec. 2.2, discrete RK adjoints
 *   A, H = A^T A, I + H          Sec. 2.2 eq. (Rhalf)
 *   gradient                     Sec. 2.2 eq. (4dvar_gradient)
 *   GN system                    eqs. (gniter), (gniterf1), (pcgsystem)
 *   Nystrom / RandSVD sketches   Sec. 3.1.1 Alg. 2 / Alg. 1
 *   limited-memory precond.      eq. (woodbury)
 *   reuse test kappa_re          Sec. 3.2 eq. (condtext2)
 *
 * Conventions (all entry points)
 *   - Every vector / block argument is a DEVICE pointer owned by the caller
 *     (e.g. a torch tensor's data_ptr()).  Host pointers are marked "host".
 *   - Blocks of k vectors in state space are row-major (n, k): grid point major,
 *     vector minor (the k vectors are interleaved per grid point).  For the 2-D
 *     model the grid is flattened j*nx + i (x fastest).
 *   - Observation-space blocks are row-major (n_t, n_obs, k), m = n_obs * n_t.
 *   - `dtype` selects the arithmetic of a block call: RP4D_F64 (double buffers)
 *     or RP4D_F32 (float buffers).  The trajectory is always stored in FP64.
 *   - Work is enqueued on the context's HIP stream and ordered on it.  Calls that
 *     return host scalars (J, info structs, kappa) synchronise that stream.
 *   - Handles are opaque, created and freed only by the library (*_create /
 *     *_destroy).  A problem must outlive the trajectories, preconditioners and
 *     GN states made from it; a context must outlive its problems.
 *   - Return value: RP4D_OK (0) or a negative error code; the message of the
 *     last failure on the calling thread is returned by rp4d_last_error().
 *     No C++ exception crosses this boundary.  On error, output buffers are
 *     left in an unspecified state unless stated otherwise.
 *   - Calls on one context must not overlap from several threads.
 */
#ifndef RP4D_H
#define RP4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RP4D_OK          0
#define RP4D_EINVAL     -1   /* bad argument or shape */
#define RP4D_ENOMEM     -2   /* device allocation failed / HBM budget exceeded */
#define RP4D_EUNSTABLE  -3   /* time step outside the RK4 stability interval */
#define RP4D_ENOTSPD    -4   /* Nystrom core matrix not SPD after shift retries */
#define RP4D_ENOCONV    -5   /* PCG reached maxit before rtol (last iterate kept) */
#define RP4D_ENONFINITE -6   /* NaN/Inf detected in a state or result */
#define RP4D_EHIP       -7   /* HIP runtime error */
#define RP4D_ESTATE     -8   /* call out of order (e.g. data not set) */

typedef struct rp4d_ctx rp4d_ctx;
typedef struct rp4d_problem rp4d_problem;
typedef struct rp4d_traj rp4d_traj;
typedef struct rp4d_precond rp4d_precond;
typedef struct rp4d_gn_state rp4d_gn_state;

enum { RP4D_F64 = 0, RP4D_F32 = 1, RP4D_BF16 = 2 };
enum {
    RP4D_NYSTROM = 0,
    RP4D_RANDSVD = 1,
    RP4D_NOPREC = 2,
    RP4D_RANDSVD_ADAPTIVE = 3,
    RP4D_SINGLEVIEW = 4,
    RP4D_SINGLEVIEW_ADAPTIVE = 5,
    RP4D_NYSTROM_ADAPTIVE = 6
};
enum { RP4D_BURGERS1D = 0, RP4D_BVE2D = 1, RP4D_BURGERS1D_WALL = 2 };
/* How a GN step obtains its direction from (I + H) dv = -g_v (eq. (gniterf1)):
 * SketchPrec (PCG preconditioned by eq. (woodbury), Sec. 3.2.2) or SketchSolv
 * (one application of eq. (woodbury), eq. (dxsol), Sec. 3.2.1). */
enum { RP4D_SOLVE_PCG = 0, RP4D_SOLVE_SKETCH = 1 };

/* Problem description (Sec. 2.1): model, window, observation layout, prior.
 *   Burgers:  nx grid points on [0,1) (ny ignored), viscosity nu.
 *   Burgers, wall (the setup of Sec. 5.1): nx interior nodes x_j = (j+1)/(nx+1)
 *     of (0,1) with homogeneous Dirichlet walls, central differences, RK3-TVD
 *     (Shu-Osher form) instead of RK4; node j observed when (j+1) is a multiple
 *     of obs_stride (n_obs = floor(nx/obs_stride)); prior Gamma^{1/2} =
 *     (prior_alpha I - prior_beta Lap*)^{-1}, Lap* = tridiag(1,-2,1) with zero
 *     walls (sigma_b, L_b ignored); nx <= 16384, batches not supported.
 *   BVE:      nx*ny periodic grid on [0,1)^2, viscosity nu.
 *   dt, nsteps: RK4 step and number of steps N of the window.
 *   obs_stride, obs_every: observe every obs_stride-th grid point (2-D: cell in
 *     both directions) at steps s_i = i*obs_every, i = 1..floor(N/obs_every).
 *   sigma_o: R_i = sigma_o^2 I.  sigma_b, L_b: Gaussian prior std and length
 *     (Burgers: L_b in domain units; BVE: L_b in cells).
 *   ckpt_every: 0 or 1 store every state of the trajectory; C > 1 store every
 *     C-th state and recompute segments during the sweeps (bitwise identical).
 *     Burgers only: the 2-D model always stores every state and, per step, its
 *     RK4 stage values and stream functions (7 fields per step).
 * 2-D model (Sec. 5.2, periodic form): vorticity zeta on a square grid
 * (nx == ny = 16 B with B in {2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32}, the
 * sides the line FFTs take, i.e. 32..512; others are RP4D_EINVAL at creation),
 * flattened j*nx + i; stream function
 * psi = L zeta with L the spectral inverse Laplacian (zero mean); RHS
 * -J_A(psi, zeta) + nu lap(zeta) with Arakawa's Jacobian J_A and the 5-point
 * Laplacian; separable prior sigma_b (S_y kron S_x), S the circulant square
 * root of the unit Gaussian kernel exp(-r^2/L_b^2) (r in cells); observations
 * at cells (j, i) with j, i multiples of obs_stride, ordered j-major. */
typedef struct {
    int model;
    int nx, ny;
    double nu;
    double dt;
    int nsteps;
    int obs_stride, obs_every;
    double sigma_o, sigma_b, L_b;
    int ckpt_every;
    double prior_alpha, prior_beta;  /* wall model only: Gamma^{1/2} = (alpha I - beta Lap*)^{-1} */
} rp4d_problem_desc;

typedef struct {
    int iters;            /* PCG iterations = (I+H) products spent */
    int converged;        /* 1 if ||r|| <= rtol ||b|| */
    double relres;        /* recurrence residual ||r_k|| / ||b|| at exit */
    double true_relres;   /* ||b - (I+H) x|| / ||b|| (one extra product; -1 if not computed) */
} rp4d_pcg_info;

/* Counters as in Sec. 5 / Tables 2 and 4: offline TLM/ADJ are spent building
 * sketches; online FWD/TLM/ADJ in cost/gradient evaluations and in PCG. */
typedef struct {
    long long fwd;
    long long tlm_online, adj_online;
    long long tlm_offline, adj_offline;
    long long sketches, reuses;
    long long hv_columns;   /* Hessian-vector columns applied (any purpose) */
} rp4d_counters;

/* Options of one Gauss-Newton step (Sec. 2.2, Sec. 3.2). */
typedef struct {
    int sketch;             /* RP4D_NYSTROM, RP4D_RANDSVD, RP4D_NOPREC (Prec_Gamma),
                               RP4D_RANDSVD_ADAPTIVE (Alg. 4, FP64), RP4D_SINGLEVIEW (Alg. 3),
                               RP4D_SINGLEVIEW_ADAPTIVE (Alg. 5, FP64) or RP4D_NYSTROM_ADAPTIVE
                               (FP64; the adaptive options as for Alg. 4) */
    int ell;                /* sketch size l (adaptive: the initial size; SingleView: l1) */
    uint64_t seed;          /* Philox seed for Omega when omega == NULL */
    const double* omega;    /* device (n, ell) test matrix -- adaptive: (n, ell_max) -- or NULL */
    int sketch_dtype;       /* RP4D_F64 or RP4D_F32 sweeps for the sketch */
    double rtol;            /* PCG relative residual tolerance */
    int maxit;              /* PCG iteration cap (<= 0: n) */
    double reuse_eps;       /* eps_re of eq. (condtext2); <= 0: always re-sketch */
    const double* vhat;     /* device unit vector for kappa_re (and for kappa_sk with the
                               adaptive sketch), or NULL (Philox) */
    int ell_hat;            /* adaptive sketch: columns per extension (SingleView: l1_hat) */
    int ell_max;            /* adaptive sketch: largest size (SingleView: of the range sketch) */
    double eps_sk;          /* adaptive sketch: stop once kappa_sk <= eps_sk (eq. (condtext)) */
    int ell2;               /* SingleView: co-range sketch size l2 (0: min(2 l1 + 1, m)) */
    const double* psi;      /* SingleView: device (m, ell2) test matrix -- adaptive: (m, l2_max),
                               see rp4d_sv_adaptive_opts -- or NULL (Philox) */
    int ell2_hat;           /* adaptive SingleView: co-range columns per extension (0: 2 ell_hat) */
    int solve;              /* RP4D_SOLVE_PCG or RP4D_SOLVE_SKETCH (needs a sketch; no PCG, so
                               pcg_iters = 0, pcg_converged = 1 and pcg_relres = -1) */
    int line_search;        /* 1: Armijo backtracking on the v-form cost, J(v + a dv) <= J(v) +
                               1e-4 a g.dv with a = 1, 1/2, ... (at most 20 trials, the last taken
                               if none passes; one FWD each); 0: a = 1 */
    int exact_lmp;          /* SketchPrec with RP4D_NYSTROM / RP4D_RANDSVD.  0 (default): PCG applies
                               the preconditioner in factored form, (I + W^T W)^{-1} = I - F F^T,
                               F = W^T chol(I + W W^T)^{-T} (eq. (randsvdsv)), with W the RandSVD W
                               or, for Nystrom, W = B^T of Alg. 2 (H_hat = B B^T keeps the shift nu:
                               at most nu from eq. (woodbury) in norm); no eigendecomposition is
                               formed.  1: eq. (woodbury) with Alg. 1/2's V_hat, Lambda_hat. */
} rp4d_gn_opts;

typedef struct {
    double J;               /* cost at the start of the step (v-form) */
    double gnorm_inf;       /* ||g_v||_inf at the start of the step */
    int pcg_iters;
    int pcg_converged;
    double pcg_relres;
    int sketched;           /* 1 if a new sketch was built in this step */
    int reused;             /* 1 if the resident preconditioner was kept */
    double kappa_re;        /* value of the reuse test, or -1 if not run */
    int sketch_ell;         /* size of the preconditioner in use (0 without one) */
    double kappa_sk;        /* last kappa_sk of an adaptive sketch built in this step, or -1 */
    double alpha;           /* step length taken */
    int ls_trials;          /* line-search trials (FWD solves), 0 without a line search */
} rp4d_gn_info;

/* Thread-local message of the last failing call ("" if none). */
const char* rp4d_last_error(void);
/* Library version string. */
const char* rp4d_version(void);

/* Context on HIP device `device`, enqueueing on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  The stream must outlive the context.
 * hbm_budget_bytes caps the device memory held through the context's objects
 * (problems, trajectories, preconditioners, GN states, batches and their
 * workspaces; counted when allocated, released when freed, whichever object is
 * destroyed first): an allocation that would exceed it fails with RP4D_ENOMEM
 * and leaves the objects usable.  0 = no cap (the device's memory).  The
 * admission of work by footprint (Sec. 3.2 serving) reads the count with
 * rp4d_ctx_hbm. */
int rp4d_ctx_create(int device, void* hip_stream, size_t hbm_budget_bytes, rp4d_ctx** out);
/* Device bytes currently held through the context (used) and its budget
 * (0 = none), host outputs (either may be NULL). */
int rp4d_ctx_hbm(const rp4d_ctx* ctx, size_t* used, size_t* budget);
int rp4d_ctx_destroy(rp4d_ctx* ctx);
/* Change the stream subsequent calls are enqueued on. */
int rp4d_ctx_set_stream(rp4d_ctx* ctx, void* hip_stream);

/* Create a problem.  Fails with RP4D_EUNSTABLE when 4 nu dt / dx^2 > 2.785 or
 * the advective CFL number exceeds 2.8 for |u| <= 10 (RK4 stability).  The
 * background x_b and observations y must be set with rp4d_problem_set_data
 * before any call that needs them (fwd innovations, gradient, gn_step). */
int rp4d_problem_create(rp4d_ctx* ctx, const rp4d_problem_desc* desc, rp4d_problem** out);
int rp4d_problem_destroy(rp4d_problem* p);
/* Host outputs: n (state size), n_obs, n_t. */
int rp4d_problem_dims(const rp4d_problem* p, int* n, int* n_obs, int* n_t);
/* Caller-chosen identity of a problem (default 0).  Batched calls derive each
 * problem's random draws (Omega, kappa_re test vectors) from (seed, id), so a
 * problem's results do not depend on its position in a batch. */
int rp4d_problem_set_id(rp4d_problem* p, uint64_t id);
/* Copy x_b (n) and y (n_t, n_obs) from device buffers into the problem. */
int rp4d_problem_set_data(rp4d_problem* p, const double* xb, const double* y);

/* Trajectory storage for one problem (every state, or checkpoints). */
int rp4d_traj_create(rp4d_problem* p, rp4d_traj** out);
int rp4d_traj_destroy(rp4d_traj* t);

/* FWD (eq. (model)): run the nonlinear RK4 model from x0 (n) over the window,
 * storing the trajectory in `traj`.  If data are set, also records the
 * innovations d_i = R^{-1/2}(O x_{s_i} - y_i) and, if J_obs != NULL (host),
 * returns 1/2 sum_i |d_i|^2 (synchronises).  Counts one online FWD. */
int rp4d_fwd(rp4d_problem* p, const double* x0, rp4d_traj* traj, double* J_obs);

/* y_out (n_t, n_obs) = O x_{s_i}: observations of the stored trajectory. */
int rp4d_observe(rp4d_problem* p, const rp4d_traj* traj, double* y_out);

/* U (n,k) = Gamma^{1/2} V (n,k): the symmetric square root of the Gaussian prior
 * (circulant Gaussian square-root kernel; 2-D separable). */
int rp4d_bhalf(rp4d_problem* p, int k, const void* V, void* U, int dtype);

/* Z (n_t,n_obs,k) = A V = [R^{-1/2} O M_i Gamma^{1/2} V]_i (eq. (Rhalf)):
 * k tangent-linear sweeps around the stored trajectory. */
int rp4d_tlm(rp4d_problem* p, const rp4d_traj* traj, int k, const void* V, void* Z, int dtype);

/* U (n,k) = A^T W = Gamma^{1/2} sum_i M_i^T O^T R^{-1/2} W_i: k adjoint sweeps
 * (discrete RK4 adjoint) with observation forcing, W shaped (n_t,n_obs,k). */
int rp4d_adj(rp4d_problem* p, const rp4d_traj* traj, int k, const void* W, void* U, int dtype);

/* HV (n,k) = (add_identity ? V : 0) + A^T A V: block GN Hessian product
 * (eq. (Rhalf), (pcgsystem)); one TLM and one ADJ sweep per column.  V and HV
 * must not alias. */
int rp4d_hessian_block(rp4d_problem* p, const rp4d_traj* traj, int k, const void* V, void* HV,
                       int dtype, int add_identity);
/* The block Hessian product of rp4d_hessian_block, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, layouts, kernels and results
 * (bitwise) as rp4d_hessian_block, 1-D models only (EINVAL for the 2-D model).
 * Its workspaces (two blocked copies of the block, the k observation columns,
 * the prior's Gram scratch and, with checkpoints, one recomputed segment) live
 * in a static 64 MiB scratch array that each GPU holds from library load until
 * the process ends; the call allocates and frees nothing, and returns EINVAL
 * when the workspaces of (n, m, k) exceed 64 MiB (about k * (2 n + m) * w bytes
 * with w = 8 for FP64, 4 for FP32).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (two streams, two threads) race.  The
 * caller still owns V and HV.  Kernel timing is suspended during the call. */
int rp4d_hessian_block_noalloc(rp4d_problem* p, const rp4d_traj* traj, int k, const void* V, void* HV,
                               int dtype, int add_identity);

/* g (n) = v + A^T d: gradient of the v-form cost (eq. (4dvar_gradient) times
 * Gamma^{1/2}) using the innovations recorded by the last rp4d_fwd on `traj`.
 * Counts one online ADJ. */
int rp4d_gradient(rp4d_problem* p, const rp4d_traj* traj, const double* v, double* g);

/* Build the low-rank preconditioner {V_hat, Lambda_hat} by Nystrom (Alg. 2) or
 * RandSVD (Alg. 1) with `ell` test vectors; omega is a device (n, ell) Gaussian
 * matrix or NULL (drawn on device with Philox4x32-10 + Box-Muller from `seed`).
 * sketch_dtype selects FP64 or FP32 sweeps; post-processing is FP64.
 * Counts ell offline TLM and ell offline ADJ.  RP4D_ENOTSPD if the shifted
 * Nystrom core matrix stays indefinite after 3 tenfold shift increases. */
int rp4d_build_precond(rp4d_problem* p, const rp4d_traj* traj, int method, int ell, uint64_t seed,
                       const double* omega, int sketch_dtype, rp4d_precond** out);
/* Nystrom approximation (Sec. 3.1.1, Alg. 2) of a symmetric operator of the
 * problem's size from a caller-supplied sketch: omega (n, ell) and Y = H omega
 * (n, ell), both device buffers, row-major FP64, read only (the caller keeps
 * them).  The shift nu = sqrt(n) 2^-52 ||Y||_2 is retried tenfold, at most 3
 * times, while the shifted core omega^T (Y + nu omega) is not numerically
 * positive definite; then RP4D_ENOTSPD.  No sweep runs and no counter moves.
 * EINVAL on null arguments or ell outside [1, min(128, n)]. */
int rp4d_build_precond_from_sketch(rp4d_problem* p, int ell, const double* omega, const double* Y,
                                   rp4d_precond** out);
/* Adaptive RandSVD (Sec. 3.1.2, Alg. 4): start from ell0 Gaussian columns and
 * add ell_hat columns while kappa_sk = ||(I + H)(I + H_hat)^{-1} v||_2
 * (eq. (condtext), (I + H_hat)^{-1} by eq. (randsvdsv)) exceeds eps_sk and the
 * sketch stays within ell_max.  Each new block is orthogonalised twice against
 * the accumulated basis and factored by Cholesky QR; each kappa_sk costs one
 * single-vector Hessian product.  FP64.  Counts every sketch column and every
 * kappa_sk product as offline TLM + ADJ. */
typedef struct {
    int ell0;               /* initial sketch size, >= 1 */
    int ell_hat;            /* columns added per extension, >= 1 */
    int ell_max;            /* largest sketch, ell0 <= ell_max <= min(128, n, m) */
    double eps_sk;          /* stop once kappa_sk <= eps_sk (> 0; the paper uses 1.01) */
    uint64_t seed;          /* Philox seed of Omega's blocks and of v when omega / vtest are NULL */
    const double* omega;    /* device (n, ell_max) row-major: columns [0, ell0) the first block, then
                               ell_hat columns per extension; or NULL */
    const double* vtest;    /* device (n) test vector (normalised here), or NULL */
} rp4d_adaptive_opts;
typedef struct {
    int ell;                /* final sketch size */
    int nkappa;             /* evaluations of kappa_sk */
    double kappa_sk;        /* the last value */
    double kappa[16];       /* the first 16 values */
} rp4d_adaptive_info;
int rp4d_build_precond_adaptive(rp4d_problem* p, const rp4d_traj* traj, const rp4d_adaptive_opts* opts,
                                rp4d_precond** out, rp4d_adaptive_info* info);
/* Adaptive Nystrom (Sec. 3.1.2; the paper gives the loop for RandSVD and calls
 * the Nystrom form similar): the same options and stopping rule as
 * rp4d_build_precond_adaptive.  Each round sweeps only the new block through
 * the block Hessian, appends it to Omega and H Omega, forms Alg. 2 on all
 * columns so far and evaluates kappa_sk with the new preconditioner.  FP64;
 * counts every column and every kappa_sk product as offline TLM + ADJ. */
int rp4d_build_precond_nystrom_adaptive(rp4d_problem* p, const rp4d_traj* traj, const rp4d_adaptive_opts* opts,
                                        rp4d_precond** out, rp4d_adaptive_info* info);
/* SingleView (Sec. 3.1.1, Alg. 3): the range sketch Y = A Omega (l1 TLM columns)
 * and the co-range sketch Z = A^T Psi (l2 ADJ columns) are independent; the
 * approximation is A_SV = Q_Y (Psi^T Q_Y)^+ Z^T (eq. (singleviewlr)), returned
 * as H_hat = A_SV^T A_SV = V_hat Lambda_hat V_hat^T (l1 columns).  Thin QRs by
 * Cholesky QR2 (shifted Cholesky QR3 when the Gram matrix is numerically
 * indefinite), FP64 post-processing.  On the 1-D model the ADJ block runs on a
 * second stream beside the TLM block unless `serial` is set.  H_hat need not
 * satisfy H_hat <= H.  Counts l1 offline TLM and l2 offline ADJ.  RP4D_ENOTSPD
 * if Y or M = Psi^T Q_Y is numerically rank deficient. */
typedef struct {
    int ell1;               /* range sketch size l1, 1 <= l1 <= min(128, n, m) */
    int ell2;               /* co-range sketch size l2, l1 <= l2 <= m; 0: min(2 l1 + 1, m) */
    uint64_t seed;          /* Philox seed of Omega (and, through a fixed mix, of Psi) when NULL */
    const double* omega;    /* device (n, l1) row-major, or NULL */
    const double* psi;      /* device (m, l2) row-major, rows ordered (n_t, n_obs) like the
                               observations, or NULL */
    int sketch_dtype;       /* RP4D_F64 or RP4D_F32 sweeps */
    int serial;             /* 1: both sketches on the problem stream */
} rp4d_singleview_opts;
int rp4d_build_precond_singleview(rp4d_problem* p, const rp4d_traj* traj, const rp4d_singleview_opts* opts,
                                  rp4d_precond** out);
/* Adaptive SingleView (Sec. 3.1.2, Alg. 5): start from Alg. 3 with (l1, l2)
 * columns and, while kappa_sk (eq. (condtext); H_hat = W^T W, eq. (randsvdsv))
 * exceeds eps_sk and l1 + l1_hat <= l1_max, draw l1_hat more range and l2_hat
 * more co-range columns: the new TLM block is orthogonalised twice against
 * Q_Y and factored by Cholesky QR, its ADJ partner runs on a second stream
 * (1-D model, unless `serial`), M = Psi^T Q_Y is refactored and W formed anew.
 * The algorithm's RandSVD-style lines A^T Q_hat / W <- [W; W_hat] are read as
 * the co-range sketch of the new Psi block followed by the SingleView W.
 * FP64.  Counts every column and every kappa_sk product offline; info->ell is
 * the final l1 (the final l2 is ell2 + (info->nkappa - 1) ell2_hat). */
typedef struct {
    int ell1, ell2;         /* initial sizes (ell2 = 0: min(2 ell1 + 1, m)), ell1 <= ell2 */
    int ell1_hat, ell2_hat; /* columns per extension (ell2_hat = 0: 2 ell1_hat), ell1_hat <= ell2_hat */
    int ell1_max;           /* largest range sketch, <= min(128, n, m) */
    double eps_sk;          /* stop once kappa_sk <= eps_sk (> 0) */
    uint64_t seed;          /* Philox seed of the blocks and of v when omega / psi / vtest are NULL */
    const double* omega;    /* device (n, ell1_max) row-major: ell1 columns, then ell1_hat per extension */
    const double* psi;      /* device (m, l2_max) row-major, l2_max = ell2 + ell2_hat *
                               floor((ell1_max - ell1) / ell1_hat) (<= m): ell2, then ell2_hat per extension */
    const double* vtest;    /* device (n) test vector (normalised here), or NULL */
    int serial;             /* 1: every sweep on the problem stream */
    int qr_update;          /* 1: keep the thin QR of M = Psi^T Q_Y by the update of Alg. 6 (needs
                               ell1_max + ell2_hat <= max(n, m)); 0: refactor M every round */
} rp4d_sv_adaptive_opts;
int rp4d_build_precond_singleview_adaptive(rp4d_problem* p, const rp4d_traj* traj, const rp4d_sv_adaptive_opts* opts,
                                           rp4d_precond** out, rp4d_adaptive_info* info);
int rp4d_precond_destroy(rp4d_precond* pc);
/* Host outputs (each nullable): ell, lambda_hat (ell, descending), Nystrom shift nu. */
int rp4d_precond_info(const rp4d_precond* pc, int* ell, double* lambda_host, double* nu_host);
/* Copy V_hat (n, ell) row-major into a device buffer. */
int rp4d_precond_basis(const rp4d_precond* pc, double* V_out);
/* Z (n,k) = (I + V_hat Lambda_hat V_hat^T)^{-1} R = R - V_hat diag(lam/(1+lam)) V_hat^T R
 * (eq. (woodbury)). */
int rp4d_precond_apply(const rp4d_precond* pc, int k, const double* R, double* Z);

/* PCG on (I + H) x = b (eq. (pcgsystem)) preconditioned by `pc` (NULL: identity,
 * the paper's Prec_Gamma), x0 = 0, stop when ||r_k|| <= rtol ||b||.  FP64.
 * Returns RP4D_ENOCONV (with x = last iterate and info filled) at maxit. */
int rp4d_pcg_solve(rp4d_problem* p, const rp4d_traj* traj, const rp4d_precond* pc,
                   const double* b, double* x, double rtol, int maxit, rp4d_pcg_info* info);

/* kappa_re = ||(I + H) (I + H_hat)^{-1} v||_2 for the unit vector v (eq. (condtext2));
 * host output. */
int rp4d_kappa_re(rp4d_problem* p, const rp4d_traj* traj, const rp4d_precond* pc,
                  const double* v, double* kappa);

/* Gauss-Newton iterate state: control vector v (starts at 0), state x = x_b +
 * Gamma^{1/2} v, its trajectory and a resident preconditioner. */
int rp4d_gn_state_create(rp4d_problem* p, rp4d_gn_state** out);
int rp4d_gn_state_destroy(rp4d_gn_state* s);
/* Copy v and/or x (each nullable, device, n) out of the state. */
int rp4d_gn_state_get(const rp4d_gn_state* s, double* v, double* x);
/* Copy the last GN direction dv (device, n). */
int rp4d_gn_state_last_step(const rp4d_gn_state* s, double* dv);

/* One GN step (Sec. 2.2 / 3.2): FWD at x, gradient, optional kappa_re reuse test
 * of the resident preconditioner, sketch, PCG, v <- v + dv, x <- x_b + Gamma^{1/2} v.
 * On the 1-D model part of the work runs on a second stream of the context (the
 * gradient; with a Nystrom or RandSVD sketch and every trajectory row stored, the
 * FWD too, launch by launch ahead of the sketch's TLM sweep); it is joined back to
 * the context stream before the PCG, so the step stays ordered on that stream.
 * Returns RP4D_ENOCONV if PCG hit maxit (the step is still applied). */
int rp4d_gn_step(rp4d_problem* p, rp4d_gn_state* s, const rp4d_gn_opts* opts, rp4d_gn_info* info);

/* Cost counters of a problem (host output) and their reset. */
int rp4d_counters_get(const rp4d_problem* p, rp4d_counters* out);
int rp4d_counters_reset(rp4d_problem* p);

/* Fill `count` doubles (device buffer `out`) with standard normals from
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11: ten rounds, multipliers
 * 0xD2511F53 / 0xCD9E8D57, key bumps 0x9E3779B9 / 0xBB67AE85) and Box-Muller.
 * Pair q = i / 2 of the output uses the counter (q mod 2^32, q >> 32, 0, 0)
 * under the key (seed mod 2^32, seed >> 32); of its output words (x0..x3),
 * a = ((x0 << 21) ^ (x1 >> 11)) mod 2^53 and b = ((x2 << 21) ^ (x3 >> 11)) mod 2^53
 * give u1 = (a + 1) 2^-53 in (0, 1] and u2 = b 2^-53, and the pair is
 * (r cos(2 pi u2), r sin(2 pi u2)) with r = sqrt(-2 ln u1); an odd count drops
 * the last sine.  Every random draw of the library (Omega, Psi, test vectors)
 * comes from this generator.  Stream-ordered; EINVAL on null arguments. */
int rp4d_philox_normal(rp4d_ctx* ctx, uint64_t seed, size_t count, double* out);

/* Problem synthesis (Sec. 5.1 'Data and Background'), all device buffers:
 * xb_out (n) = x_true + Gamma^{1/2} xi;  y_out (n_t, n_obs) = O M(x_true) + sigma_o eta
 * (perfect model: the truth is propagated by the same FWD).  Does not set the
 * problem's data (call rp4d_problem_set_data with the outputs). */
int rp4d_problem_synthesize(rp4d_problem* p, const double* x_true, const double* xi, const double* eta,
                            double* xb_out, double* y_out);

/* 2-D model only: psi = L zeta for k fields, in and out row-major (n x k) in
 * `dtype` on the device (in == out allowed).  L is the spectral inverse
 * Laplacian (Sec. 5.2), diagonal in the 2-D Fourier basis, applied by FFT:
 * the fields go through row, column (times the diagonal) and inverse row
 * transforms as ceil(k/2) complex pairs.  RP4D_EINVAL for a 1-D problem. */
int rp4d_bve_inv_laplacian(rp4d_problem* p, int k, const void* in, void* out, int dtype);

/* Reset a GN state to v = 0, x = x_b and drop its resident preconditioner. */
int rp4d_gn_state_reset(rp4d_gn_state* s);

/* Kernel timing with HIP events recorded on the context stream (any call clears
 * the statistics): enable = 1 records an event pair around every launch of the
 * timed kernel classes; enable = 2 records one pair around each Burgers sweep's
 * loop of launches (classes TLM, ADJ, TLM1, ADJ1, FWD; the others per launch),
 * so that timing barely perturbs what it measures -- per-launch averages are
 * then span time / launches and include the gaps between the sweep's launches;
 * enable = 0 stops timing.
 * Classes: RP4D_K_TLM, RP4D_K_ADJ (block sweeps, k > 1), RP4D_K_FWD, RP4D_K_BHALF,
 * RP4D_K_TLM1, RP4D_K_ADJ1 (single-vector sweeps, k = 1) and RP4D_K_EIG (the
 * small symmetric eigensolves of the sketch post-processing; flops reported 0),
 * and for the 2-D model RP4D_K_SPECTRAL (= RP4D_K_GEMM, its earlier name: the
 * column passes of the TLM/ADJ stages' spectral solves and the whole FFT solves
 * of the prior root and the FWD) and RP4D_K_STENCIL (the fused row passes of
 * the TLM/ADJ stages -- row FFT halves, Arakawa / Laplacian stencils, RK update
 * or adjoint combine -- and the FWD stage kernels); 2-D FFT work is counted as
 * FFT-equivalent flops, 5 N log2 N per complex transform of N points.
 * rp4d_ctx_kernel_stats synchronises the stream and returns the number of
 * launches, their summed duration (ms) and the algorithmic flops they performed
 * (owned grid points only; FP64 or FP32 as launched). */
enum {
    RP4D_K_TLM = 0, RP4D_K_ADJ = 1, RP4D_K_FWD = 2, RP4D_K_BHALF = 3,
    RP4D_K_TLM1 = 4, RP4D_K_ADJ1 = 5, RP4D_K_EIG = 6, RP4D_K_GEMM = 7, RP4D_K_SPECTRAL = 7, RP4D_K_STENCIL = 8,
    RP4D_K_COUNT = 9
};
int rp4d_ctx_set_timing(rp4d_ctx* ctx, int enable);

/* PCG solves (rp4d_pcg_solve, rp4d_gn_step) that run past two iterations
 * capture the iteration body -- the Hessian product, the dot products, the
 * x/r/p updates and the preconditioner -- once into a HIP graph on a
 * library-owned stream and replay it on the context stream for the remaining
 * iterations (results are bitwise those of the eager loop).  Off by default:
 * capture must not overlap legacy-stream operations (synchronous copies,
 * frees) issued by other threads of the process, so enable it only where one
 * thread drives the device. */
int rp4d_ctx_set_graphs(rp4d_ctx* ctx, int enable);

/* Precision of the tall-skinny Gram products in the sketch post-processing
 * that feed an eigenvalue estimate or an eigendecomposition (Alg. 2's shift
 * estimate lambda_max(Y^T Y) and the Gram B^T B of its eigendecomposition; the
 * Gram W W^T of the randomized EVD's eigendecomposition): RP4D_F64 (default)
 * or RP4D_BF16 (operands rounded to bfloat16 on the BF16 matrix cores, FP32
 * accumulation per row chunk, chunks summed in FP64: relative errors of order
 * 2^-8 in those Grams, which cost PCG iterations, not correctness).  The Grams
 * that are Cholesky-factored (the Nystrom core Omega^T Y_nu, Cholesky-QR, the
 * factored preconditioner's I + W W^T) stay FP64.  RP4D_EINVAL for another dtype. */
int rp4d_ctx_set_gram_precision(rp4d_ctx* ctx, int dtype);
int rp4d_ctx_kernel_stats(rp4d_ctx* ctx, int kind, long long* launches, double* total_ms, double* alg_flops);

/* ---------------------------------------------------------------------------
 * Batches: many independent Burgers problems (uneven n and window length)
 * advanced together.  Each phase is one launch over all problems (the sweeps:
 * one fused launch per time interval covering every problem's tiles); per-problem
 * reductions use one workgroup per problem with a fixed order, so each result is
 * the same whatever else shares the batch.  Batched sweeps need full trajectory
 * storage (ckpt_every <= 1).  Arrays are indexed like the batch's problems.
 * ------------------------------------------------------------------------- */
typedef struct rp4d_batch rp4d_batch;
/* Group `nprob` problems of one context (the batch does not own them). */
int rp4d_batch_create(rp4d_ctx* ctx, int nprob, rp4d_problem* const* probs, rp4d_batch** out);
int rp4d_batch_destroy(rp4d_batch* b);
/* Tiling of the batched sweeps (mode RP4D_MODE_TLM / RP4D_MODE_ADJ with dtype, or
 * RP4D_MODE_FWD for the forward sweep, dtype RP4D_F64, kc ignored): points per
 * thread, vectors per region, threads per workgroup, steps per launch and the
 * region shape xch (RP4D_XCH_WAVE, the default: one region of 64*ppt points per
 * wave, threads 64/128/256; RP4D_XCH_LDS: one region of threads*ppt points per
 * workgroup).  Each problem's tile is the region minus 2*(4*steps+4) points (at
 * most n).  Values <= 0 keep the defaults (wave regions, 12 steps; ppt 4 and
 * kc 2 for the block sweeps, ppt 2 for the forward sweep; 256 threads).
 * Results do not depend on the tiling. */
int rp4d_batch_set_tiling(rp4d_batch* b, int mode, int dtype, int ppt, int kc, int threads, int steps, int xch);
/* As rp4d_batch_set_tiling for k = 0; k = 1 sets the tiling of the batch's
 * single-vector TLM/ADJ sweeps (the gradient and the PCG products; kc <= 1),
 * which takes precedence over the k = 0 entry for them.  Default of those
 * sweeps: wave regions, 4 points per lane, 256 threads, 16 steps per launch.
 * RP4D_EINVAL for another k, for k = 1 with the FWD mode or kc > 1. */
int rp4d_batch_set_tiling_k(rp4d_batch* b, int mode, int dtype, int k, int ppt, int kc, int threads, int steps,
                            int xch);
/* FWD of every problem from x0[i] (device, n_i) into trajs[i]; J_obs (host, nprob,
 * nullable) receives 1/2 |d_i|^2. */
int rp4d_batch_fwd(rp4d_batch* b, const double* const* x0, rp4d_traj* const* trajs, double* J_obs);
/* HV[i] (n_i, k) = (add_identity ? V[i] : 0) + H_i V[i] for every problem. */
int rp4d_batch_hessian_block(rp4d_batch* b, rp4d_traj* const* trajs, int k, const void* const* V, void* const* HV,
                             int dtype, int add_identity);
/* One GN step for every problem (states[i] belongs to problem i): batched FWD,
 * gradient, kappa_re reuse test (when opts->reuse_eps > 0 and a preconditioner is
 * resident), Nystrom sketches (opts->sketch = RP4D_NYSTROM, omega must be NULL:
 * Omega drawn with Philox from seed ^ (0x9E3779B97F4A7C15 * (id + 1))) or none
 * (RP4D_NOPREC), lockstep FP64 PCG, update.
 * infos (host, nprob, nullable).  RP4D_ENOCONV if some PCG hit maxit. */
int rp4d_batch_gn_step(rp4d_batch* b, rp4d_gn_state* const* states, const rp4d_gn_opts* opts, rp4d_gn_info* infos);

/* Sweep tiling of a problem's block sweeps (used by the autotuner): points per
 * thread `ppt`, vectors per region `kc`, threads per workgroup `threads`,
 * tile length `tile` (grid points owned per region), steps per launch `steps`
 * and the region's neighbour exchange `xch`:
 *   RP4D_XCH_LDS  - one region per workgroup (threads * ppt points), edge
 *                   values through LDS with a barrier per RK stage;
 *   RP4D_XCH_WAVE - one region per 64-lane wave (64 * ppt points), edge values
 *                   through lane shifts; `threads` (64, 128 or 256) only groups
 *                   waves into workgroups.
 * Both give bitwise the same results.  `mode` selects the sweep: 0 both,
 * RP4D_MODE_TLM or RP4D_MODE_ADJ, or RP4D_MODE_FWD for the single nonlinear
 * forward sweep (dtype, k and kc ignored); `dtype`/`k` select the entry (k = 0:
 * every k).  Any argument <= 0 restores the built-in heuristic for that field;
 * all <= 0 removes the entry.  Invalid tilings are reported by the sweep call
 * that uses them (RP4D_EINVAL). */
enum { RP4D_MODE_TLM = 1, RP4D_MODE_ADJ = 2, RP4D_MODE_FWD = 3 };
enum { RP4D_XCH_LDS = 1, RP4D_XCH_WAVE = 2 };
int rp4d_set_sweep_tiling(rp4d_problem* p, int mode, int dtype, int k, int ppt, int kc, int threads,
                          int tile, int steps, int xch);
/* Host output: the tiling the next sweep of `mode` (0 = TLM) with (dtype, k) would use. */
int rp4d_get_sweep_tiling(const rp4d_problem* p, int mode, int dtype, int k, int* ppt, int* kc, int* threads,
                          int* tile, int* steps, int* xch);

#ifdef __cplusplus
}
#endif
#endif /* RP4D_H */
