/*
 * libstokesmg -- matrix-free multigrid for the 3D Stokes problem discretized
 * with H(div)-conforming DG (Raviart-Thomas RT_k velocity, DG Q_k pressure,
 * symmetric interior penalty), after Cui & Kanschat, "Multigrid methods for
 * the Stokes problem on GPU systems" (arXiv 2410.09497).  AMD Instinct MI355X
 * (gfx950), HIP.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Mesh: the unit cube, n^3 equal cubes per level (Sec. 2.1), n a power of two.
 * Degree k in 1..5.  N1 = n (k+1).
 *
 * Vector layout (one level): [u_x | u_y | u_z | p], contiguous, no padding.
 *   u_x[ix + (N1-1) (iy + N1 iz)]  ix = interior continuous node g-1
 *                                  (g = 1 .. N1-1), iy, iz = cell (k+1) + Gauss index
 *   u_y[ix + N1 (iy + (N1-1) iz)]  continuous index in y
 *   u_z[ix + N1 (iy + N1 iz)]      continuous index in z (iz < N1-1)
 *   p  [ix + N1 (iy + N1 iz)]      all indices discontinuous
 * Offsets: 0, nc, 2 nc, 3 nc with nc = (N1-1) N1^2; total 3 nc + N1^3.
 * The normal velocity nodes on the boundary are eliminated (u.n = 0 is part
 * of the space, Sec. 2.1).  The continuous direction uses Lagrange
 * polynomials on the k+2 Gauss-Lobatto points; the discontinuous directions
 * and the pressure use Lagrange polynomials on the k+1 Gauss points.
 *
 * Operator: K = [[A, B^T], [B, 0]] with A the interior-penalty form of
 * Eq. bilinear (penalty gamma = penalty_factor (k+1)^2 / h, interior faces
 * gamma [u].[v] - {{d_n u}}.[v] - [u].{{d_n v}}, boundary faces
 * 2 gamma u.v - d_n u.v - u.d_n v) and B_{PX} = -(psi_P, div phi_X)
 * (Eq. weak_form written with the symmetric sign of Eq. block_A).
 *
 * Memory: every vector argument is a DEVICE pointer owned by the caller.
 * The library allocates no device memory: the caller queries
 * stokesmg_workspace_size() and hands a device buffer of at least that size
 * to stokesmg_set_workspace(); the library never frees caller memory.
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Every
 * entry point is asynchronous on that stream unless stated otherwise.
 *
 * Errors: every int-returning call returns STOKESMG_OK (0) or a negative
 * code; stokesmg_last_error() returns a message for the last failure on that
 * handle.  No exception or exit() crosses this boundary.
 */
#ifndef STOKESMG_H
#define STOKESMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STOKESMG_OK            0
#define STOKESMG_EINVAL       -1   /* bad argument: level, dtype, size, aliasing, NULL */
#define STOKESMG_EHIP         -2   /* a HIP runtime error; the message keeps its text */
#define STOKESMG_ENOMEM       -3   /* no workspace set, or it is too small */
#define STOKESMG_ENOTCONV     -4   /* solve reached max_it; info is still filled */
#define STOKESMG_EUNSUPPORTED -5   /* combination not built (e.g. degree out of range) */

#define STOKESMG_F64 0
#define STOKESMG_F32 1

typedef struct stokesmg stokesmg_t;

typedef struct {
    int    n_cells;         /* cells per direction on the finest level; power of two, >= 1 */
    int    k;               /* polynomial degree, 1..5 */
    int    n_levels;        /* levels of the hierarchy; coarsest has n_cells >> (n_levels-1) cells
                               per direction (>= 1) */
    double penalty_factor;  /* gamma = penalty_factor (k+1)^2 / h; must be 2.0, the method's value
                               (the kernels carry it as a compile-time constant): other values
                               return STOKESMG_EUNSUPPORTED */
    double cg_rtol;         /* local Schur-complement CG: stop when ||r|| <= cg_rtol ||r_0|| (a value
                               below 16 eps of the arithmetic -- 1.9e-6 in FP32, 3.6e-15 in FP64 --
                               is raised to it; the iteration also stops if d.Sd <= 0) ... */
    int    cg_max_it;       /* ... or after cg_max_it iterations (Sec. 3.3: about 15 on average) */
} stokesmg_config;

/* Builds every level's 1D tables on the host (FP64, Sec. 2 and the
 * separable structure of Sec. 2.2).  No device memory is touched until
 * stokesmg_set_workspace().  Returns EINVAL for an invalid config.
 * Caller owns *out and releases it with stokesmg_destroy(). */
int stokesmg_create(const stokesmg_config* cfg, stokesmg_t** out);

/* Releases the handle (not the caller's workspace).  NULL is ignored. */
void stokesmg_destroy(stokesmg_t* h);

/* Message of the last error on this handle ("" if none).  The string is
 * owned by the handle and valid until the next call on it. */
const char* stokesmg_last_error(const stokesmg_t* h);

/* Number of levels, and sizes of level `level` (0 = coarsest,
 * n_levels-1 = finest): unknowns per velocity component, pressure unknowns
 * and total.  Any output pointer may be NULL. */
int stokesmg_num_levels(const stokesmg_t* h);
int stokesmg_sizes(const stokesmg_t* h, int level, int64_t* n_u_comp, int64_t* n_p, int64_t* n_total);

/* Device bytes the library needs (tables and internal vectors).  The
 * buffer passed to stokesmg_set_workspace() must be 256-byte aligned. */
int stokesmg_workspace_size(const stokesmg_t* h, size_t* bytes);

/* Hands the caller-owned device buffer to the library and uploads the
 * tables into it (asynchronously on `stream`).  The buffer must stay alive
 * and untouched by the caller while the handle uses it.  ENOMEM if smaller
 * than stokesmg_workspace_size(). */
int stokesmg_set_workspace(stokesmg_t* h, void* dev_ptr, size_t bytes, void* stream);

/* y = K_level x: the matrix-free operator of Alg. 1 (cell terms, interior-
 * face and boundary-face terms of Eq. bilinear, and both divergence blocks),
 * evaluated through its separable form (Sec. 2.2) by one fused kernel.
 * dtype: STOKESMG_F64 (double) or STOKESMG_F32 (float); x and y have the
 * layout above at that level.  x and y must not overlap (EINVAL). */
int stokes_apply(stokesmg_t* h, int level, int dtype, const void* x, void* y, void* stream);

/* r = b - K_level x (the residual of Alg. 2), fused into the same kernel.
 * r may alias neither x nor b (EINVAL). */
int stokes_residual(stokesmg_t* h, int level, int dtype, const void* b, const void* x, void* r,
                    void* stream);

/* One or more sweeps of the colourized multiplicative vertex-patch smoother
 * (Alg. 2) on level `level` (n >= 2 cells per direction): for each colour
 * c = 0..7 in ascending order, r = b - K x over the whole level, then every
 * patch j of colour c adds R_j^T A_j^{-1} R_j r to x in parallel (the DoF sets
 * of one colour are disjoint).  The local solve is the Schur complement
 * (Sec. 3.2): CG on S = B_j A_j^{-1} B_j^T over mean-zero patch pressures, with
 * A_j^{-1} applied by fast diagonalization; with a tight cg_rtol it equals the
 * pseudo-inverse solve (Sec. 3.3).  x is updated in place; b is read only.
 * x and b must not overlap each other or the workspace (EINVAL).
 * Degrees 1..5. */
int patch_smooth(stokesmg_t* h, int level, int dtype, void* x, const void* b, int n_sweeps, void* stream);

/* For callers that cannot allocate device memory at the call site (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): patch_smooth with the same arguments and the same kernels, whose
 * per-call scratch -- the residual vector of the colour loop and the two CG
 * counters -- lives in a static device array of the library
 * (STOKESMG_NOALLOC_SCRATCH_BYTES per device, held until the process ends)
 * instead of the workspace.  The level tables still come from the workspace
 * set at setup (ENOMEM without one).  The call allocates nothing.
 * Limit: 256 + (level unknowns) x (8 for F64, 4 for F32) bytes must fit the
 * array (32 MiB: e.g. 32^3 cells at k = 2 in F64), else EINVAL.
 * cg_iterations (host pointer, may be NULL): if given, the total local CG
 * iterations of this call; the call then synchronizes `stream`.
 * All calls on one device share its array and keep the last call's contents:
 * calls that overlap in time on one device (two streams, two threads) race. */
#define STOKESMG_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int patch_smooth_noalloc(stokesmg_t* h, int level, int dtype, void* x, const void* b, int n_sweeps,
                         int64_t* cg_iterations, void* stream);
/* *bytes = STOKESMG_NOALLOC_SCRATCH_BYTES (no device needed). */
int stokesmg_noalloc_scratch_size(size_t* bytes);

/* Total local CG iterations and local solves performed by patch_smooth since
 * the last reset (reset = 1 zeroes them after reading).  Synchronizes
 * `stream`. */
int stokesmg_cg_stats(stokesmg_t* h, int64_t* iterations, int64_t* solves, int reset, void* stream);

/* x = P_L^{-1} b: one V-cycle (Sec. 3) from x = 0 on the finest level:
 * pre-smoothing (one patch_smooth sweep), coarse-grid correction with
 * restriction P^T, recursion, prolongation P (the canonical embedding of the
 * coarse space), post-smoothing (one sweep); on the coarsest level the dense
 * pseudo-inverse of K_0 (FP64 matrix also inside an FP32 cycle).  dtype F64
 * or F32 for b and x (finest-level vectors).  Requires a coarsest level with
 * at most 1000 unknowns (EUNSUPPORTED otherwise); every degree 1..5.  The
 * local solver is the one set by stokesmg_set_local_solver (exact by default). */
int vcycle(stokesmg_t* h, int dtype, const void* b, void* x, void* stream);

#define STOKESMG_MAX_HISTORY 512
typedef struct {
    int    iterations;        /* FGMRES steps (V-cycle applications) */
    int    converged;         /* relative residual estimate reached rtol */
    double rel_residual;      /* ||b - K x|| / ||b|| of the returned x, recomputed in FP64 */
    double nu;                /* fractional iteration count -8 / log10(rbar) (Sec. 3.3) */
    double history[STOKESMG_MAX_HISTORY];   /* residual estimate / ||b|| after each step; [0] = 1 */
    long long cg_iterations;  /* local Schur CG iterations during the solve */
    long long local_solves;   /* local patch solves during the solve */
    double seconds;           /* wall time of the solve call */
    int    fallback_iteration;/* learned local solver: FGMRES steps done with it before the exact solver
                                 took over for the rest of the solve (-1: never) */
} stokesmg_info;

/* Bytes of the caller-owned solve workspace for FGMRES(restart), 1 <= restart <= 60,
 * with the V-cycle in vcycle_dtype: restart + 1 FP64 Krylov vectors V, restart
 * preconditioned vectors Z in the V-cycle's precision (FP32 for an FP32 cycle),
 * and three more finest-level vectors.  solve() uses a shorter restart when the
 * workspace it is given holds fewer vectors (at least one step must fit). */
int stokesmg_solve_workspace_size(const stokesmg_t* h, int restart, int vcycle_dtype, size_t* bytes);

/* Solves K x = b on the finest level by right-preconditioned restarted FGMRES
 * (GMRES preconditioned by the V-cycle, Sec. 3.3), x_0 = 0, until the
 * Euclidean residual estimate satisfies ||r|| <= rtol ||b|| or max_it steps.
 * The outer loop is FP64; vcycle_dtype F32 runs the whole V-cycle in FP32 and
 * converts at its entry and exit (Sec. 4.3).  b and x are FP64 device vectors;
 * the returned pressure has zero integral mean.  Synchronizes `stream` a few
 * times per step (Hessenberg scalars).  ENOTCONV when max_it is reached (info
 * and x are still filled).  info may be NULL. */
int solve(stokesmg_t* h, const double* b, double* x, double rtol, int max_it, int restart, int vcycle_dtype,
          void* solve_ws, size_t solve_ws_bytes, stokesmg_info* info, void* stream);

/* Right-hand side of a manufactured problem on level `level` (FP64 device
 * vector): (f, phi) + the boundary terms 2 gamma <g, phi> - <g, d_n phi> of
 * Eq. bilinear for the tangential data g = u, by Gauss quadrature with k+2
 * points per direction; pressure rows zero.
 * STOKESMG_PROBLEM_SINE: u = curl(sin(pi x) sin(pi y) sin(pi z) (1,1,1)),
 * p = cos(pi x) cos(pi y) cos(pi z), f = -Laplace u + grad p. */
#define STOKESMG_PROBLEM_SINE 0
int stokesmg_rhs_manufactured(stokesmg_t* h, int level, int problem, double* b, void* stream);

/* L2 errors ||u - u_h|| (velocity) and ||p - p_h|| (pressure, both with zero
 * integral mean) over the unit cube of the FP64 level vector x against the
 * manufactured solution `problem`, by Gauss quadrature with k+3 points per
 * direction in every cell.  Uses the workspace scratch; synchronizes
 * `stream`.  For the error-versus-time study of the solver (Sec. 3.3). */
int stokesmg_l2_error(stokesmg_t* h, int level, int problem, const double* x, double* err_u, double* err_p,
                      void* stream);

/* Right-hand side (f, phi) of a smooth random body force (FP64 device
 * vector on level `level`), no boundary data, pressure rows zero:
 * f_c(x) = sum_m amp[c][m] cos(pi kappa[c][m] . x + theta[c][m]), c = 0..2,
 * m < n_modes.  kappa: host int array [3][n_modes][3]; amp, theta: host double
 * arrays [3][n_modes].  Gauss quadrature with k+2 points per direction
 * (the force is expanded into separable products of cosines and sines).
 * Synchronizes `stream`. */
int stokesmg_rhs_fourier(stokesmg_t* h, int level, int n_modes, const int* kappa, const double* amp,
                         const double* theta, double* b, void* stream);

/* ------------------------------------------------------------------------
 * Learned local solver (an extension; the paper's local solvers are exact).
 *
 * One network per degree, shared by every interior patch of every level: a
 * patch whose 8 cells touch no boundary face (vertex v with 2 <= v_d <= n-2)
 * has, after scaling, the same local problem on every level (A_j ~ h,
 * B_j ~ h^2 for the separable forms of Sec. 2.2).  Patch-local vectors follow
 * X_j of Sec. 3.1: [U_x | U_y | U_z | P], each the box of that component's
 * index grid starting at (v_d - 1)(k+1), 2k+1 entries in the component's own
 * direction and 2k+2 in the others (and for P), lexicographic with x fastest;
 * d = 3 (2k+1)(2k+2)^2 + (2k+2)^3 entries.
 * Normalized pair: input x = (F/h, G/h^2) / s with s = ||(F/h, G/h^2)||_2 of
 * the patch residual (F, G) = R_j r, target t = (U, h P) / s of the exact
 * correction (U, P) = K_j^+ (F, G) (Sec. 3.1); a zero residual gives x = t = 0.
 * Network: y = GELU(GELU(x W1 + b1) W2 + b2) W3 + b3, hidden width 256,
 * GELU(z) = z Phi(z) with the normal CDF Phi; row-major weights [in x out].
 * Parameter vector (FP32, P = mlp_num_params): W1 | b1 | W2 | b2 | W3 | b3.
 * Products run on the matrix cores with FP32 accumulation; mode
 * STOKESMG_MLP_BF16 rounds the operands to BF16 (production),
 * STOKESMG_MLP_F32 keeps them in FP32 (checks).
 * Memory: an MLP workspace (device, caller-owned, 256-byte aligned) sized by
 * mlp_workspace_size() holds the parameters, gradients, Adam moments and
 * the activations of up to max_rows rows; set it with mlp_set_workspace().
 * ------------------------------------------------------------------------ */
#define STOKESMG_MLP_HIDDEN 256
#define STOKESMG_MLP_BF16 0
#define STOKESMG_MLP_F32  1

#define STOKESMG_LOCAL_EXACT 0   /* Schur complement + fast diagonalization (Sec. 3.2) */
#define STOKESMG_LOCAL_MLP   1   /* network on interior patches, exact solve on the others; the
                                    learned patch pressure is projected to zero coefficient mean,
                                    as the exact correction (orthogonal to the kernel of K_j) is */
#define STOKESMG_LOCAL_MLP_WARM 2 /* exact solve everywhere; on interior patches the Schur CG starts
                                    from the pressure the network predicts instead of zero, with the
                                    same stopping test (relative to the cold-start residual): the
                                    exact solver judges, the network only saves iterations */
#define STOKESMG_LOCAL_DIRECT 3  /* the "Direct" solver of Sec. 3.3 on every patch: the patch
                                    pseudo-inverse as one dense matrix per patch type (the same on
                                    every level in the normalized variables of the gather), applied
                                    to all patches of a colour in one kernel that gathers the patch
                                    residuals, multiplies them on the matrix cores (BF16 or FP32
                                    operands per mlp_mode, FP32 accumulation) and adds the
                                    corrections; no local iteration.  Needs stokesmg_direct_setup(). */

#define STOKESMG_LOCAL_EXACT_BF16 4 /* the exact Schur CG of Sec. 3.2 on every patch, with the in-plane
                                    eigenbasis products of the fast diagonalization (S_x (x) S_y per
                                    velocity component, all z-slices as one GEMM) on the matrix cores:
                                    BF16 operands, FP32 accumulation (Sec. 4.3's mixed precision
                                    carried into the local solver); the z factor and the eigenvalue
                                    scaling in FP32.  FP32 cycles only (an FP64 sweep returns
                                    EINVAL), degrees 1..3 (EUNSUPPORTED).  mlp_mode is ignored. */

/* d (network width in and out) and P (parameter count) for the handle's degree. */
int mlp_dims(const stokesmg_t* h, int64_t* d, int64_t* n_params);

/* Bytes of the MLP workspace for batches of up to max_rows rows (training
 * batches, or the interior patches of one colour per chunk in the learned
 * smoother); for degrees 1..3 it includes the Direct solver's 28 maps, padded
 * to whole tiles, in FP32 and in BF16 (99 MB at k = 2, 718 MB at k = 3). */
int mlp_workspace_size(const stokesmg_t* h, int64_t max_rows, size_t* bytes);
int mlp_set_workspace(stokesmg_t* h, void* dev_ptr, size_t bytes, int64_t max_rows);

/* Parameters drawn from a counter-based generator (SplitMix64): weights
 * uniform in +-sqrt(3 / fan_in), biases zero; Adam moments and step reset. */
int mlp_init(stokesmg_t* h, uint64_t seed, void* stream);

/* Checkpoint: state = parameters | Adam first moments | Adam second moments
 * (3 P floats, device) and the Adam step count. */
int mlp_get_state(stokesmg_t* h, float* state, int64_t* step, void* stream);
int mlp_set_state(stokesmg_t* h, const float* state, int64_t step, void* stream);

/* Y = network(X) for n rows (X, Y: device, row-major n x d FP32). */
int mlp_forward(stokesmg_t* h, int mode, const float* X, float* Y, int64_t n, void* stream);

/* Gradients of the loss mean((network(X) - T)^2) over all n d entries with
 * respect to the parameter vector: grads (P floats, device), loss (one
 * float, device).  n <= max_rows. */
int mlp_backward(stokesmg_t* h, int mode, const float* X, const float* T, int64_t n, float* grads, float* loss,
                 void* stream);

/* One Adam step (Kingma & Ba: beta1 0.9, beta2 0.999, eps 1e-8) on the
 * handle's parameters with gradient `grads` (device, P floats). */
int mlp_adam_step(stokesmg_t* h, const float* grads, float lr, void* stream);

/* Pair capture: one FP64 V-cycle x = P^{-1} b with the exact local solver
 * (as vcycle()), recording the normalized pair of every interior patch
 * solved on the finest level (pre- and post-smoothing, all colours) into
 * rows *n, *n + 1, ... of X and T (device, cap x d FP32); *n is advanced,
 * pairs beyond cap are dropped.  b, x: FP64 finest-level device vectors. */
int mlp_collect_pairs(stokesmg_t* h, const double* b, double* x, float* X, float* T, int64_t cap, int64_t* n,
                      void* stream);

/* Training: `epochs` passes over the n pairs in batches of `batch` rows
 * (batch <= max_rows; a permutation per epoch from SplitMix64(seed, epoch)),
 * Adam with cosine decay lr_t = lr (1 + cos(pi t / T)) / 2 over the
 * T = epochs ceil(n / batch) steps.  loss_hist (host, epochs floats, may be
 * NULL) receives each epoch's mean batch loss.  Synchronizes once per epoch. */
int mlp_train(stokesmg_t* h, int mode, const float* X, const float* T, int64_t n, int epochs, int batch, float lr,
              uint64_t seed, float* loss_hist, void* stream);

/* Local solver used by patch_smooth, vcycle and solve from now on, the
 * network's precision, and a damping factor in (0, 1] applied to the learned
 * corrections (1 = undamped; unused by STOKESMG_LOCAL_MLP_WARM and
 * STOKESMG_LOCAL_DIRECT).  The two learned solvers need an MLP workspace with
 * parameters; the Direct solver needs stokesmg_direct_setup(). */
int stokesmg_set_local_solver(stokesmg_t* h, int local_solver, int mlp_mode, double mlp_damping);

/* The Direct solver's matrices (Sec. 3.3 "Direct solver"), one per patch
 * type: t = M x with x = (F / h, G / h^2) and t = (U, h P) for the patch
 * residual (F, G) and its exact correction (U, P) = K_j^+ (F, G); the same on
 * every level.  The type says which outer faces of the vertex patch lie on
 * the domain boundary: type = t_x + 3 t_y + 9 t_z with t_d = 0 (neither),
 * 1 (the lower face: vertex coordinate 1), 2 (the upper face: vertex n - 1);
 * type 27 is the single patch of the 2^3-cell mesh (both faces everywhere).
 * Built on the host in FP64 from the fast-diagonalization tables via the
 * Schur complement of Sec. 3.2 and checked between two levels.
 * stokesmg_direct_matrix writes the matrix of one type to host memory (d x d
 * doubles, row-major [out][in], d from mlp_dims; no device needed; EINVAL
 * for a type outside 0..27).  stokesmg_direct_setup builds all 28 (on host
 * threads) and uploads them, padded to whole tiles, in FP32 and rounded to
 * BF16 (nearest even) into the MLP workspace, which must be set (ENOMEM);
 * synchronizes `stream`.  Degrees 1..3 (EUNSUPPORTED). */
int stokesmg_direct_matrix(const stokesmg_t* h, int type, double* M);
int stokesmg_direct_setup(stokesmg_t* h, void* stream);

/* Smoothing sweeps of the V-cycle (vcycle, solve, mlp_collect_pairs): pre
 * sweeps before the coarse-grid correction (the first from x = 0) and post
 * sweeps after it, each one patch_smooth sweep over the 8 colours in
 * ascending order.  Default 1 / 1, the single pre- and post-smoothing step of
 * Sec. 3; the iteration counts the paper prints (Table 1 in 2D, at most three
 * steps from k = 3 in 3D, Sec. 3.3) are met with 2 / 2 in this
 * implementation.  0..16 each, at least one in total (EINVAL). */
int stokesmg_set_smoothing(stokesmg_t* h, int pre_sweeps, int post_sweeps);

/* Fallback of the learned solver inside solve(): with the MLP local solver,
 * after FGMRES step j with contraction rho_j = res_j / res_{j-1} of the
 * residual estimate, the rest of the solve uses the exact local solver when
 * rho_j >= max(2 rho_ref, 1e-3) (rho_ref > 0: the plain method's measured
 * contraction) or, for rho_ref <= 0, when rho_j >= 1 (no progress).  A
 * preconditioned vector with non-finite entries also triggers it (that step
 * is dropped).  FGMRES then restarts from the current iterate. */
int stokesmg_set_fallback(stokesmg_t* h, double rho_ref);

#ifdef __cplusplus
}
#endif

#endif /* STOKESMG_H */
