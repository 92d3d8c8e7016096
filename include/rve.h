/*
 * rve.h -- C ABI of librve: the RVE corrector path on one AMD Instinct MI355X
 * (gfx950), hand-written HIP kernels.
 *
 * Problem (Khoromskaia, Khoromskij, Otto, "Numerical study in stochastic
 * homogenization for elliptic PDEs", Sec. 2 eqns. RHS_grad1/scaled_setting
 * and Sec. 4.3 eqn. wg03): on the periodic n x n grid of Q1 finite elements,
 * for a per-cell coefficient field a > 0, find the correctors phi_1, phi_2
 * with  int grad psi . a (e_i + grad phi_i) = 0  for every test function psi,
 * then the homogenized 2x2 matrix (Sec. 4.1 eqns. A_hom_m, Ahom_m_entry;
 * Sec. 4.3 eqn. wg01 and the symmetry argument for wg02).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Grid: n periodic nodes and n cells per axis. Cell (i, j) spans nodes
 *   i..i+1 along x1 and j..j+1 along x2 (mod n). Arrays are row-major
 *   [i][j] with x2 contiguous (the paper's big-endian index map, Sec. 3.2).
 * - Supported n: multiples of 64 from 64 to 4096.
 * - The discrete problem depends only on the cell array a: the Q1 stiffness
 *   is h-independent in 2D, so the library solves in grid units and returns
 *   phi multiplied by the mesh width h. A_hom does not depend on h.
 * - A_hom is reported in the energy form
 *     A_ij = < (e_j + grad phi_j) . a (e_i + grad phi_i) >
 *   (symmetric by construction; its error is quadratic in the solver error),
 *   optionally beside the flux form A_ij = < a (delta_ij + d_j phi_i) > of
 *   eqn. Ahom_m_entry. < . > is the average over the torus.
 * - Solver (Sec. 3.5, eqn. DD_Eqn): preconditioned CG from x0 = 0 with the
 *   constant-coefficient periodic Q1 operator a0 * A_Delta as preconditioner,
 *   a0 = (max a + min a) / 2 (proof of Lemma Cond_Number), applied as its
 *   pseudo-inverse (the paper's shift delta -> 0 on the mean-zero subspace).
 *   Stop when ||r||_2 / ||f||_2 <= tol. phi is returned with zero mean.
 * - Memory: every pointer argument named *_dev is device memory owned by the
 *   caller, on the context's device; *_host is host memory. The library
 *   allocates only inside the context (workspace, transform tables), grows
 *   that workspace on demand, and frees it in rve_destroy.
 * - Streams: all work is enqueued on the context's stream, in order. Calls
 *   return after enqueueing, except where a host output or a convergence
 *   poll needs the device (documented per call).
 * - Errors: every call returns an int status (enum rve_status); nothing
 *   throws across the ABI. Argument errors are detected on the host before
 *   any work is enqueued. Batch calls also write a per-item status.
 * - Threads: a context must not be used by two host threads at once.
 *   Contexts are independent of each other.
 */
#ifndef RVE_H
#define RVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum rve_status {
  RVE_OK = 0,             /* converged */
  RVE_NOT_CONVERGED = 1,  /* maxit reached; outputs and relres still written */
  RVE_BREAKDOWN = 2,      /* p^T A p <= 0 or not finite during PCG */
  RVE_EINVAL = -1,        /* invalid argument (host), or a coefficient <= 0 / NaN (device) */
  RVE_EHIP = -2,          /* a HIP runtime error */
  RVE_ENOMEM = -3         /* device allocation failed */
};

/* Arithmetic of the preconditioner's transform GEMMs (Q X Q on MFMA). The
 * residual r, the iterate x, q = A p, the stencil arithmetic, the CG dot
 * products and the A_hom reductions are FP64 in every mode; in the mixed
 * modes the search directions p and the preconditioned residual z are
 * stored in FP32 (they only steer the iteration: r = f - A x still holds to
 * FP64 rounding, so the stopping test is unaffected). */
enum rve_precision {
  RVE_FP64 = 0,      /* FP64 MFMA, FP64 intermediates */
  RVE_MIX_FP32 = 1,  /* FP32 MFMA, FP32 intermediates */
  RVE_MIX_BF16 = 2,  /* BF16 MFMA operands, FP32 accumulation, BF16 intermediates. Its 8-bit
                        significand, amplified by 1/E in the lowest modes, costs iterations as
                        n grows (measured, contrast 10: 38 against 35 in FP64 at n = 512, about
                        100 against 36 at n = 2048) and at high contrast; RVE_MIX_FP16 runs at
                        the same MFMA rate and stays within one or two iterations of FP64 at
                        every size measured, so it is the faster mixed mode from n = 1024 on */
  RVE_MIX_FP16 = 3   /* FP16 MFMA operands, FP32 accumulation, FP16 intermediates; the
                        residual copy is scaled per system to 0.25 sqrt(N)/||r|| and the
                        symbol's reciprocal stored as E_min/E, so every intermediate stays
                        below the 2-norm of the scaled residual (in rve_apply_precond*,
                        where no residual norm is at hand, the caller's r is used unscaled
                        and must keep its 2-norm below about 6e4) */
};

/* Arithmetic of the operator apply inside PCG. With RVE_STENCIL_FP32 the
 * coefficients, the direction p (rounded to FP32 before use) and q = A p are
 * FP32 while the p.Ap partial sums stay FP64; since q is then only an FP32
 * approximation of A p, the residual is recomputed as r = f - A x in FP64
 * from the current iterate every RVE_DIRECTION_RING iterations, which keeps
 * the stopping test on the true residual to within FP32 rounding of the last
 * few steps. */
enum rve_stencil_precision {
  RVE_STENCIL_FP64 = 0,
  RVE_STENCIL_FP32 = 1
};

/* Discretisation. RVE_SCHEME_Q1: the consistent Q1 Galerkin operator
 * (Sec. 3.1 eqn. FEM_discr; nine-point stencil) with the Q1 constant
 * coefficient preconditioner a0 (K (x) M + M (x) K). RVE_SCHEME_FD5: the
 * lumped form of Sec. 3.2 (eqns. Lapl_Kron_D, As_Kron: each cell contributes
 * a_e (k (x) d + d (x) k) with the lumped mass d = diag(1/2, 1/2); a
 * five-point stencil whose edges carry the mean of their two cells), with the
 * finite-difference Laplacian a0 (Delta_1 (x) I + I (x) Delta_2) of eqn.
 * Lap_Kron as preconditioner. Both have the same right-hand sides; A_hom and
 * its gradient use the scheme's own quadrature (edges for RVE_SCHEME_FD5). */
enum rve_scheme {
  RVE_SCHEME_Q1 = 0,
  RVE_SCHEME_FD5 = 1
};

/* The PCG iterate is not updated every iteration: the search directions of
 * RVE_DIRECTION_RING consecutive iterations are kept, and x += sum_j
 * alpha_j p_j is applied once per that many iterations and at the end, in
 * the order of the plain recurrence (Sec. 3.5 PCG; the result is the same
 * to the last bit). Device memory: that many direction vectors per system. */
#define RVE_DIRECTION_RING 8

typedef struct rve_opts {
  double tol;        /* relative residual target ||r||_2/||f||_2, > 0 */
  int maxit;         /* maximum PCG iterations per system, >= 1 */
  int prec;          /* enum rve_precision */
  int flexible;      /* 1: flexible (Polak-Ribiere) beta; 0: standard beta.
                        Negative: automatic (standard). */
  int check_every;   /* host polls the all-converged flag every this many
                        iterations, rounded up to a multiple of
                        RVE_DIRECTION_RING; <= 0: every RVE_DIRECTION_RING */
  int stencil_prec;  /* enum rve_stencil_precision */
  int scheme;        /* enum rve_scheme (RVE_SCHEME_FD5 needs RVE_STENCIL_FP64) */
} rve_opts;

typedef struct rve_ctx rve_ctx;

/* Fill *opts with defaults: tol 1e-10, maxit 2000, FP64, automatic beta,
 * automatic polling, FP64 operator apply, Q1 scheme. */
void rve_default_opts(rve_opts* opts);

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream). */
int rve_create(rve_ctx** out, int device, void* hip_stream);
int rve_destroy(rve_ctx* ctx);
int rve_set_stream(rve_ctx* ctx, void* hip_stream);

/*
 * One realization, synchronous (Sec. 2, corrector problem eqn. RHS_grad1 /
 * scaled_setting; Sec. 4.1 eqns. A_hom_m and Ahom_m_entry): the coefficient
 * field in, the two correctors (optionally) and the homogenized matrix out.
 *
 *   n              as for rve_solve_batch
 *   a_dev          [n][n] FP64 per-cell coefficients on the device, each > 0
 *   h              mesh width (> 0); phi is returned in physical units (x h)
 *   phi_dev        [2][n][n] FP64 correctors (device, mean zero), or NULL
 *   ahom_host      [2][2] FP64 energy-form A_hom (host, required)
 *   ahom_flux_host [2][2] FP64 flux-form A_hom (host), or NULL
 *   iters_host     [2] PCG iterations per direction (host), or NULL
 *   relres_host    [2] final recursive ||r||/||f|| per direction (host), or NULL
 *
 * Returns the realization's status: RVE_OK, RVE_NOT_CONVERGED or
 * RVE_BREAKDOWN (host outputs written), RVE_EINVAL for a bad argument
 * (nothing enqueued) or for a coefficient <= 0 / NaN found on the device
 * (host outputs written, with phi = 0), RVE_EHIP / RVE_ENOMEM (outputs
 * undefined). Blocks until the host outputs are written.
 */
int rve_solve(rve_ctx* ctx, int n, double h, const double* a_dev, const rve_opts* opts, double* phi_dev,
              double* ahom_host, double* ahom_flux_host, int* iters_host, double* relres_host);

/*
 * Solve B independent realizations of equal size n (one batch: every kernel
 * launch covers all 2B corrector systems).
 *
 *   a_dev         [B][n][n] FP64 per-cell coefficients, each > 0
 *   h             mesh width (> 0); phi is returned in physical units (x h)
 *   phi_dev       [B][2][n][n] FP64 correctors phi_1, phi_2 (mean zero), or NULL
 *   ahom_dev      [B][2][2] FP64 energy-form A_hom (required)
 *   ahom_flux_dev [B][2][2] FP64 flux-form A_hom, or NULL
 *   iters_dev     [B][2] int PCG iterations per direction, or NULL
 *   relres_dev    [B][2] FP64 final recursive relative residual, or NULL
 *   status_dev    [B] int per-item status (enum rve_status), or NULL
 *
 * Returns the worst status over items (EINVAL/EHIP/ENOMEM before warnings).
 * Blocks the host on polls of the convergence flag (every check_every
 * iterations) and at the end, when it reads the per-item statuses.
 * The iterations run in chunks of RVE_DIRECTION_RING, each replayed from a
 * HIP graph captured on first use (see rve_set_graphs); a solve may run up
 * to one chunk past the iteration where its last system stopped (those
 * launches find no active system and return at once).
 */
int rve_solve_batch(rve_ctx* ctx, int B, int n, double h, const double* a_dev,
                    const rve_opts* opts, double* phi_dev, double* ahom_dev,
                    double* ahom_flux_dev, int* iters_dev, double* relres_dev,
                    int* status_dev);

/*
 * Three-dimensional corrector problems (d = 3): the setting of Sec. 2 with
 * a(x) times the 3 x 3 identity, the trilinear Q1 discretisation (eqn.
 * As_Kron_d: the element stiffness k (x) m (x) m + m (x) k (x) m + m (x) m (x) k)
 * and the constant-coefficient preconditioner a0 A_Delta of Sec. 3.5,
 * diagonalised by Hartley transforms along the three axes (six transform
 * GEMMs per apply). B realizations of equal size n, 3B systems.
 *
 *   n             64 <= n <= 256, n % 64 == 0 (grid n x n x n, x3 contiguous;
 *                 cell (i,j,k) spans nodes i..i+1, j..j+1, k..k+1 mod n)
 *   a_dev         [B][n][n][n] FP64 per-cell coefficients, each > 0
 *   h             mesh width (> 0); phi is returned in physical units (x h)
 *   phi_dev       [B][3][n][n][n] FP64 correctors (mean zero), or NULL
 *   ahom_dev      [B][3][3] FP64 energy-form A_hom (required)
 *   ahom_flux_dev [B][3][3] FP64 flux-form A_hom, or NULL
 *   iters_dev     [B][3] int PCG iterations per direction, or NULL
 *   relres_dev    [B][3] FP64 final recursive relative residual, or NULL
 *   status_dev    [B] int per-item status, or NULL
 *
 * opts as for rve_solve_batch, with stencil_prec = RVE_STENCIL_FP64 and
 * scheme = RVE_SCHEME_Q1 (anything else: RVE_EINVAL). Same iteration chunks,
 * graph replay, polling and return convention as rve_solve_batch.
 */
int rve_solve_batch_3d(rve_ctx* ctx, int B, int n, double h, const double* a_dev,
                       const rve_opts* opts, double* phi_dev, double* ahom_dev,
                       double* ahom_flux_dev, int* iters_dev, double* relres_dev,
                       int* status_dev);

/* out = A u for B three-dimensional fields: a_dev [B][n][n][n] cells,
 * u_dev and out_dev [B][n][n][n] nodes (one operand per realization;
 * u_dev != out_dev); n as for rve_solve_batch_3d. Asynchronous. */
int rve_apply_operator_3d(rve_ctx* ctx, int B, int n, const double* a_dev,
                          const double* u_dev, double* out_dev);

/* z = (a0 A_Delta)^+ r for the three systems of each realization:
 * r_dev, z_dev [B][3][n][n][n] FP64, a0 from a_dev as in the solver,
 * transforms in `prec` (enum rve_precision). Asynchronous. */
int rve_apply_precond_3d(rve_ctx* ctx, int B, int n, const double* a_dev,
                         const double* r_dev, double* z_dev, int prec);

/*
 * Realizations of different sizes in one call (packed input).
 *
 *   n_host[B]          grid size of item b (host)
 *   cell_off_host[B+1] element offsets of item b's cells in a_dev (host);
 *                      item b occupies a_dev[cell_off[b] .. cell_off[b]+n_b^2)
 *   phi_dev            packed like a_dev but with 2 n_b^2 nodes per item at
 *                      offset 2*cell_off[b], or NULL
 *   other outputs      as rve_solve_batch, indexed by item
 * Items are grouped by n (each group one batch as in rve_solve_batch) and
 * all groups iterate together: one captured chunk of iterations covers
 * every size, and one convergence poll serves the whole call. Offsets must
 * be non-overlapping.
 */
int rve_solve_uneven(rve_ctx* ctx, int B, const int* n_host,
                     const int64_t* cell_off_host, double h, const double* a_dev,
                     const rve_opts* opts, double* phi_dev, double* ahom_dev,
                     double* ahom_flux_dev, int* iters_dev, double* relres_dev,
                     int* status_dev);

/*
 * Derivative of the energy-form A_hom with respect to every cell value
 * (vector-Jacobian product). The energy form is stationary in the
 * correctors (eqn. wg03), so d A_ij / d a_e = (1/n^2) int_e (e_i + grad
 * phi_i) . (e_j + grad phi_j) and no adjoint solve is needed. The
 * derivative in the inclusion value (Sec. 2, eqns. Stoch-decomp and
 * ahm_coef: the covered set carries one value, which moves all its cells
 * together) is the sum of the per-cell derivative over the covered cells.
 *
 *   a_dev           [B][n][n] coefficients used for the solve (device)
 *   phi_dev         [B][2][n][n] correctors as returned by rve_solve_batch (x h)
 *   h               the same mesh width
 *   G_dev           [B][2][2] upstream weights G_ij
 *   grad_a_dev      [B][n][n] output: sum_ij G_ij d A_ij / d a_e
 *   incl_mask_dev   [B][n][n] bytes, nonzero on the covered cells (device);
 *                   or NULL: the covered cells are those with a_e == a_in
 *   a_in            inclusion value, read only when incl_mask_dev is NULL
 *                   and an inclusion derivative is asked for (must be finite)
 *   grad_in_dev     [B] output: sum_ij G_ij d A_ij / d a_in per realization,
 *                   or NULL
 *   grad_in_sum_dev [1] output: the sum of those B values (fixed order), for
 *                   one inclusion value shared by the batch; or NULL
 *   scheme          enum rve_scheme the correctors were computed with
 * Asynchronous. Scratch for the partial sums comes from the context's
 * workspace (allocated or grown on demand).
 */
int rve_grad(rve_ctx* ctx, int B, int n, const double* a_dev,
             const double* phi_dev, double h, const double* G_dev,
             double* grad_a_dev, const unsigned char* incl_mask_dev, double a_in,
             double* grad_in_dev, double* grad_in_sum_dev, int scheme);

/*
 * rve_grad without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments, kernels and results as rve_grad; the partial
 * sums go to a fixed scratch array of 4 MiB per GPU (a static device array,
 * held by the process until it ends) instead of the context's workspace.
 * Needs 8 B (n/64)^2 per realization when an inclusion derivative is asked
 * for (plus 8 B per realization when only its sum is); a call needing more
 * than 4 MiB returns RVE_EINVAL (and says so on stderr) with nothing
 * enqueued. All calls on one GPU share that GPU's array: calls that overlap
 * on one GPU (different streams or threads without ordering) race. Every
 * scratch byte a call reads it writes first. Asynchronous.
 */
int rve_grad_noalloc(rve_ctx* ctx, int B, int n, const double* a_dev,
                     const double* phi_dev, double h, const double* G_dev,
                     double* grad_a_dev, const unsigned char* incl_mask_dev, double a_in,
                     double* grad_in_dev, double* grad_in_sum_dev, int scheme);

/*
 * Coefficient fields of the two-valued model from their covered sets (Sec. 2,
 * eqns. Stoch-decomp and ahm_coef): a_dev[b][e] = a_in_dev[b] where
 * mask_dev[b][e] != 0, else a_bg. cells = cells per field (n^2, or n^3 in
 * three dimensions); mask_dev [B][cells] bytes, a_in_dev [B], a_dev
 * [B][cells] (all device). 1 <= B <= 65535, a_bg > 0 and finite (the
 * values a_in_dev[b] are checked by the solver like any coefficient).
 * Asynchronous.
 */
int rve_field_from_mask(rve_ctx* ctx, int B, long long cells, const unsigned char* mask_dev,
                        const double* a_in_dev, double a_bg, double* a_dev);

/*
 * Ensemble statistics of N homogenized matrices at RVE size L (Sec. 4.2
 * eqn. A_hom_Empir; Sec. 5 eqns. Var1, Var2; Sec. 5.3 eqn. quartic).
 *
 *   ahom_dev [N][2][2] FP64, N >= 2
 *   out_dev  [26] FP64: mean[4] (A11 A12 A21 A22), centred variance[4]
 *            (1/(N-1)), std_a12 and std_(a11-a22) (uncentred, 1/N), then
 *            the 4x4 quartic tensor q[(i,k),(j,l)] = L^2 cov(A_ij, A_kl),
 *            row-major.
 */
int rve_stats(rve_ctx* ctx, int N, double L, const double* ahom_dev, double* out_dev);

/*
 * The two linear maps of the PCG, one call each, for checking them alone.
 *
 * rve_apply_operator: out = A u for the stiffness of each field in scheme
 * `scheme` (grid units; Q1: Sec. 3.1 eqn. FEM_discr, assembled there by the
 * Kronecker sums of Sec. 3.2, applied here matrix-free as a 9-point stencil;
 * FD5: the lumped five-point form).
 *   a_dev [B][n][n] cells; u_dev, out_dev [B][2][n][n] nodes (distinct).
 *
 * rve_apply_precond: z = (a0 A_Delta)^+ r (Sec. 3.5) with a0 = (max a +
 * min a)/2 of each field, A_Delta the scheme's constant-coefficient operator
 * and the transform GEMMs in precision `prec` (enum rve_precision).
 *   a_dev [B][n][n]; r_dev, z_dev [B][2][n][n] (distinct).
 */
int rve_apply_operator(rve_ctx* ctx, int B, int n, const double* a_dev, const double* u_dev,
                       double* out_dev, int scheme);
int rve_apply_precond(rve_ctx* ctx, int B, int n, const double* a_dev, const double* r_dev,
                      double* z_dev, int prec, int scheme);

/* Static string for a status code. */
const char* rve_status_string(int status);

/*
 * Autotuner. With mode 1 (the default), the first solve of each
 * (n, precision, floor(log2 B)) times the candidate kernel variants on the
 * live data and keeps the fastest: the shape of the operator apply (V = 1, 2
 * or 4 grid columns per lane, H = 16 or 64 rows per wave strip, D = 1, 2 or 4
 * rows of loads in flight per wave), the shape of the residual update that
 * recomputes A p (FP64 apply, two dimensions; same shape set, timed on
 * passes that leave the residual unchanged) and the transform-GEMM
 * variant (64 x 64
 * tiles, or for BF16 128 x 128 tiles when n % 128 == 0; the even/odd-folded
 * variant is used only through rve_force_variants, since its saving per
 * apply is outweighed by extra iterations). Choices are cached in the context
 * and, if the environment variable RVE_TUNE_CACHE names a file, appended
 * there as JSON lines and read back by rve_create. Mode 0 uses fixed
 * defaults. The 16-bit transform tile variants the tuner chooses among
 * (1, 4, 5, 6; the 64 x 64 kernel only where none of them fits) give
 * identical results, so that choice never changes a solve; the operator-apply
 * and residual-update shapes set the summation order of the PCG dot
 * products' partial sums, so their choice changes results at rounding level
 * only.
 *
 * rve_get_tuned: *choice for kind 0 (FP64 operator-apply shape, encoded as
 * V + 8 (H / 16) + 64 (D - 1) for D = 1, 2 and V + 8 (H / 16) + 128 for
 * D = 4), 1 (GEMM variant: 0 = 64 x 64, 1 = 128 x 128, 2 = folded
 * 128 x 128, 3 = 128 x 128 loaded straight into LDS, 4 = 256 x 128,
 * 5 = 256 x 256, 6 = 256 x 256 from 8 waves), 2 (FP32 operator-apply
 * shape), 3 (five-point operator-apply shape), 4 (shape of the recomputing
 * residual update, nine-point) or 5 (the same, five-point), every shape
 * encoded as kind 0, of a shape,
 * or -1 with return value RVE_NOT_CONVERGED if not tuned yet. Cached choices
 * that are not valid for a shape are ignored and tuned again.
 */
int rve_set_autotune(rve_ctx* ctx, int mode);

/*
 * Spectral density of the stiffness matrix (Appendix, eqns. DOS and
 * DOS_gauss): phi_eta(t) = (1/m) sum_j g_eta(t - lambda_j), m = n^2, g_eta the
 * Gaussian of width eta, estimated with probe vectors v (for example with
 * entries +-1): (1/m) tr g(t - A) ~ mean_v v^T g(t - A) v / m, expanded in
 * Chebyshev polynomials of Ahat = A / c - I, c = lmax / 2.
 *
 * rve_dos_moments: mu_dev [B][nv][K] (device) receives
 * mu_k = v^T T_k(Ahat) v / m for the operator of field b (scheme: enum
 * rve_scheme) and its probes v_dev [B][nv][n][n] (device, nv even). lmax
 * must bound the largest eigenvalue (e.g. 16/3 max a for RVE_SCHEME_Q1 and
 * 8 max a for RVE_SCHEME_FD5, by Gershgorin). About K/2 operator applies
 * per probe.
 *
 * rve_dos_eval: phi_dev [B][nt] (device) receives
 * sum_k a_k(t) mubar_k at the points t_dev [nt] (device), mubar the mean of
 * the nv probes' moments and a_k(t) the Chebyshev coefficients of
 * x -> g_eta(t - c (1 + x)) by a Chebyshev-Gauss rule with Q >= K nodes
 * (Q <= 0: Q = 4 K).
 *
 * rve_dos_plan: the spectral bound and the moment count for fields a_dev
 * [B][n][n] (device) and width eta > 0: *lmax_host = (16/3) max a (Q1) or
 * 8 max a (five-point), the Gershgorin bound of every eigenvalue, and
 * *K_host = min(20000, max(64, floor(6 lmax / eta))), about six moments per
 * width over the spectrum. RVE_EINVAL if a cell is <= 0 or NaN. Blocks until
 * the results are on the host.
 *
 * rve_dos_probes: v_dev [B][nv][n][n] (device) receives probe vectors with
 * entries +1 or -1: entry i (flat index) is -1 iff bit i mod 32 of word
 * (i div 32) mod 4 of Philox4x32-10 (Salmon et al., SC'11) with counter
 * (i div 128 mod 2^32, i div 2^39, 0, 0x50524F42) and key (seed mod 2^32,
 * seed div 2^32) is set. Asynchronous.
 */
int rve_dos_moments(rve_ctx* ctx, int B, int n, int scheme, const double* a_dev, int nv,
                    const double* v_dev, double lmax, int K, double* mu_dev);
int rve_dos_eval(rve_ctx* ctx, int B, int nv, int K, const double* mu_dev, double lmax,
                 double eta, int Q, int nt, const double* t_dev, double* phi_dev);
int rve_dos_plan(rve_ctx* ctx, int B, int n, int scheme, const double* a_dev, double eta,
                 double* lmax_host, int* K_host);
int rve_dos_probes(rve_ctx* ctx, int B, int nv, int n, uint64_t seed, double* v_dev);

/*
 * Sample B coefficient fields of the random inclusion model (Sec. 2, covered
 * domain eqn. Stoch-decomp, coefficient eqn. ahm_coef) on the device, for
 * realizations first .. first + B - 1, into a_dev [B][n][n] (FP64, device).
 *
 * Lattice law: each of the n^2 sites (i, j) is independently the centre of
 * a side x side square with probability occ_threshold / 2^32 (for Poisson
 * centres with mean mu per site, occ_threshold = round(2^32 (1 - exp(-mu)));
 * with mu = ln 2 / side^2 half the cells are covered on average). Site
 * s = i n + j of realization r is a centre iff word (s mod 4) of
 * Philox4x32-10 (Salmon et al., SC'11) with counter (s div 4, r mod 2^32,
 * r div 2^32, 0) and key (seed mod 2^32, seed div 2^32) is below
 * occ_threshold. A square centred at s covers cells s - side/2 + u,
 * u = 0 .. side-1, in each direction (mod n); covered cells take a_in, the
 * others a_bg. Integer arithmetic only: a realization's field does not
 * depend on the batch it is drawn in or on the device.
 *
 * Requires n as for rve_solve_batch, 1 <= side <= min(32, n),
 * 1 <= B <= 65535, first >= 0, a_in and a_bg > 0 and finite.
 */
int rve_sample_lattice(rve_ctx* ctx, int B, int n, int side, uint64_t seed, int64_t first,
                       uint32_t occ_threshold, double a_in, double a_bg, double* a_dev);

/*
 * The paper's own law (Sec. 2, eqn. Stoch-decomp: exactly L^2 squares of side
 * 2 alpha; Sec. 3.1: centres at grid nodes): B fields a_dev [B][n][n] (FP64,
 * device) for realizations first .. first + B - 1, each with exactly K
 * side x side squares (side = 2 alpha m0 cells, K = L^2) whose centres are
 * drawn independently and uniformly from the n^2 nodes. Centre k of
 * realization r is node floor(v n^2 / 2^64), v = w0 + 2^32 w1 from words 0 and
 * 1 of Philox4x32-10 with counter (k, r mod 2^32, r div 2^32, 0x46495843) and
 * key (seed mod 2^32, seed div 2^32); a square centred at node s covers cells
 * s - side/2 + u, u = 0 .. side-1, in each direction (mod n), as in
 * rve_sample_lattice. Needs B n^2 bytes of the context's workspace.
 * Requires n as for rve_solve_batch, 1 <= side <= min(32, n),
 * 1 <= B <= 65535, first >= 0, K >= 0, a_in and a_bg > 0 and finite.
 */
int rve_sample_fixed_count(rve_ctx* ctx, int B, int n, int side, uint64_t seed, int64_t first, int K,
                           double a_in, double a_bg, double* a_dev);

/* Site-occupancy threshold of rve_sample_lattice for Poisson centres with
 * mean mu per lattice site: round(2^32 (1 - exp(-mu))) (ties to even),
 * clamped to [0, 2^32 - 1]; 0 for mu <= 0 or NaN. Host only. */
uint32_t rve_occupancy_threshold(double mu);

/* Use these kernel variants instead of the autotuner's or default choice
 * (-1: no override): an operator-apply shape as encoded for rve_get_tuned
 * kind 0 / 2; a shape for the recomputing residual update (the same codes;
 * -1 with an operator-apply shape given: that shape); and a transform-GEMM
 * variant (0: 64 x 64 tiles; 1: 128 x 128
 * 16-bit tiles, n % 128 == 0; 2: even/odd-folded 128 x 128 BF16 tiles, half
 * the MFMA work, n % 256 == 0; 3: 128 x 128 16-bit tiles with the operands
 * loaded straight into LDS, n % 128 == 0, the same results as 1; 4: 256 x 128
 * 16-bit tiles for all transforms but the one scaling by 1/E (BF16; FP16:
 * the first and third), n % 256 == 0; 5: 256 x 256 16-bit tiles for all four,
 * n % 256 == 0; 6: the same tiles from 8 waves of 128 x 64 instead of 16 of
 * 64 x 64, n % 256 == 0, the same z as 5; 7: the tiles of 6 with the operands
 * loaded straight into LDS through a four-stage ring of 32-wide K slices,
 * n % 256 == 0, the same z as 5). An
 * override that is not valid for a shape is
 * ignored for that shape. Applies to rve_solve_* and rve_apply_precond. */
int rve_force_variants(rve_ctx* ctx, int stencil_choice, int gemm_variant, int update_choice);

/* Single-workgroup solver (default on): when every batch of a solve has
 * n = 64 in two dimensions with FP64 transforms and the FP64 apply, each
 * corrector system is solved by one workgroup in one launch (the cells, the
 * Hartley matrix and the vectors stay on the chip), instead of the batched
 * iteration chunks. Same iteration and stopping rule; results agree with the
 * batched path to rounding. mode 0 turns it off, 1 on; anything else
 * RVE_EINVAL. */
int rve_set_small_solver(rve_ctx* ctx, int mode);

/* Where the next search direction p_{k+1} = z_{k+1} + beta_k p_k is formed:
 * mode 1 (the default) in the epilogue of the preconditioner's last
 * transform wherever that is a 16-bit tile variant, the standard beta and
 * the FP64 operator apply are used (beta is summed between the second and
 * the third transform; the operator apply then reads p_k alone); mode 0
 * always in the operator apply, from z_k and p_{k-1}. Both round p to its
 * storage type in the same way, so results are identical to the last bit
 * (with rve_set_direction_bf16 mode 0; see there). Anything else:
 * RVE_EINVAL. */
int rve_set_direction_update(rve_ctx* ctx, int mode);

/* Storage type of the search directions where the last transform forms
 * them (rve_set_direction_update mode 1, 16-bit transforms, n <= 512,
 * contrast <= 20): mode
 * 1 (the default) BF16, p_{k+1} = z_{k+1} + beta_k p_k formed in FP64 and rounded
 * once; mode 0 FP32, as the operator apply forms them. Sec. 3.5's PCG with
 * the direction rounded before use: x += alpha p and r -= alpha A p see the
 * same rounded p, so r = f - A x holds to FP64 rounding and the stopping
 * test and A_hom keep their accuracy; only the conjugacy of successive
 * directions is perturbed (a few percent more iterations), against 2 bytes
 * less per node and system in each of four passes over them. Larger grids,
 * and solves holding a field of contrast max a / min a above 20, keep FP32
 * directions: over their longer iterations the perturbation adds up (n =
 * 4096 with BF16 transforms stalled near a relative residual of 2e-7; at
 * contrast 100 the extra iterations cost more than the bytes save).
 * Anything else: RVE_EINVAL. */
int rve_set_direction_bf16(rve_ctx* ctx, int mode);

/* Chunks of PCG iterations: mode 1 (the default) captures each distinct
 * chunk (same batches, pointers, kernel choices and options) once as a HIP
 * graph, cached in the context, and replays it; mode 0 launches every
 * kernel one by one. Both run the same kernels in the same order, so the
 * results are identical to the last bit. While kernel timing is on
 * (rve_set_timing) chunks are always launched one by one. */
int rve_set_graphs(rve_ctx* ctx, int mode);
int rve_get_tuned(rve_ctx* ctx, int kind, int n, int prec, int B, int* choice);

/* Event timing of kernel classes on the context's stream. rve_set_timing
 * turns recording on (1) or off (0) and clears the accumulators; while it is
 * on, every launch of a class is bracketed by HIP events.
 * rve_last_timing returns the totals since the last rve_set_timing in
 * out_ms[7] and out_counts[7], one entry per kernel: [0] the operator apply
 * fused with the search-direction update, [1]..[4] the four transform GEMMs
 * of the preconditioner in order, [5] the residual update, [6] the iterate
 * update x += sum alpha_j p_j, applied once per RVE_DIRECTION_RING iterations
 * and once at the end of a solve. */
int rve_set_timing(rve_ctx* ctx, int enable);
int rve_last_timing(rve_ctx* ctx, double* out_ms, long long* out_counts);

#ifdef __cplusplus
}
#endif

#endif /* RVE_H */
