/*
 * glm.h -- C ABI of the gfx950 PCG-Aug solver for SUR generalized least squares.
 *
 * The method (Foschi, "Preconditioned Conjugate Gradient methods for the
 * estimation of General Linear Models"):
 *   - a SUR model  y = vec(Y),  X = X_1 (+) ... (+) X_G,  Sigma = Omega (x) I_M
 *     (SUR section, eq. SURdefs), optionally with linear restrictions
 *     R_c beta = r (restricted GLM section, eq. RGLM);
 *   - the GLS estimate is the beta-block of the augmented system
 *       [Sigma X; X^T 0] [u; beta] = [y; 0]                       (eq. aug1)
 *     which stays well posed for a singular PSD Omega as long as Sigma is
 *     positive definite on the null space of X^T (eq. SigmaPosXNull) or y is
 *     consistent;
 *   - the system is solved by preconditioned conjugate gradients with the
 *     indefinite preconditioner K = [D X; X^T 0]^-1 (eq. invprec, eq. prec),
 *     D = alpha I with alpha = max_i omega_ii, whose application is one OLS
 *     step per equation through thin QR factors X_i = Q_i R_i (Algorithm
 *     "The PCG-Aug method"; SUR section).
 *
 * Conventions shared by every entry point
 *   - A batch holds B independent instances.  Instance b has G_b equations,
 *     M_b observations, K_b right-hand sides (1 <= K_b <= 16), k_b restriction
 *     rows (0 = unrestricted) and columns n_{b,1..G_b}; n_b = sum_i n_{b,i}.
 *   - Every batched array is the concatenation, in instance order, of the
 *     per-instance arrays below (no gaps, no per-instance offsets):
 *        X      M_b x n_b     row-major, the blocks side by side [X_1 ... X_G]
 *        Rc     k_b x n_b     row-major (instances with k_b = 0 contribute nothing)
 *        Omega  G_b x G_b     row-major, symmetric positive semi-definite
 *        y, u   M_b x G_b x K_b   row-major: element (t, i, k) = observation t
 *                                 of equation i for right-hand side k
 *        r, uc  k_b x K_b     row-major
 *        beta   n_b x K_b     row-major, blocks stacked in equation order
 *   - All array arguments are DEVICE pointers (HBM of the current device)
 *     unless marked "host".  Double precision throughout the interface.
 *   - Every call enqueues its work on `stream`.  glm_qr_factor does not
 *     block the host.  glm_gls_solve and glm_gls_backward block the calling
 *     thread while they iterate (they poll convergence flags every few
 *     iterations) and return once all results are written.
 *   - Nothing throws across the boundary and nothing calls exit/abort.
 *     Host-detectable problems return a negative code immediately, before
 *     any work is enqueued; device-detected conditions are reported per
 *     (instance, right-hand side) in `info`.
 *   - The library never allocates or frees device memory: the caller
 *     provides one workspace (size from glm_workspace_bytes) that holds the
 *     factors, the iteration vectors and all partial sums.  It allocates a
 *     small pinned host buffer per factor handle for convergence polling.
 *   - A handle and its workspace serve one call at a time.
 */
#ifndef GLM_H
#define GLM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes --------------------------------------------------------- */
#define GLM_OK             0
#define GLM_EINVAL        -1   /* bad shape, NULL where required, K outside 1..16 */
#define GLM_EWORKSPACE    -2   /* workspace too small or NULL                   */
#define GLM_EHIP          -3   /* a HIP runtime call failed                     */
#define GLM_EUNSUPPORTED  -4   /* valid request outside what this build handles */

/* ---- per (instance, right-hand side) outcome written to `info` ------------- */
#define GLM_INFO_CONVERGED   0  /* stopping test met                                   */
#define GLM_INFO_STAGNATED   1  /* c_i stopped decreasing (terminated, as the paper
                                   allows, at the attainable accuracy)                */
#define GLM_INFO_NOCONV    -10  /* iteration limit reached; outputs hold the last
                                   iterate                                             */
#define GLM_INFO_BREAKDOWN -11  /* d_i <= 0 or not finite; outputs hold beta recovered
                                   from the current u (Algorithm PCG-Aug, termination) */
#define GLM_INFO_RANK      -12  /* an X_i (or [X; R_c]) is numerically rank deficient;
                                   nothing was solved for this instance               */

typedef enum glm_precision {
  GLM_FP64 = 0,   /* every step in double precision                               */
  GLM_MIXED = 1,  /* inner PCG with single-precision Q_i, vectors and Omega
                     (single-precision accumulation, double-precision dot
                     products), inside double-precision iterative refinement;
                     QR, refinement residual and the beta/u updates in double   */
  GLM_REDUCED = 4, /* flag, OR-ed into GLM_FP64 or GLM_MIXED for
                     glm_workspace_bytes and glm_qr_factor: SUR model reduction
                     (the remark on reducing the SUR model in the SUR section).
                     One Householder QR of W = [X_1 ... X_G] = Q [R; 0] per
                     instance (double precision) rotates every equation by Q^T;
                     the solve then runs PCG-Aug on the first Mr = min(M, n + 1)
                     rotated observations, which give the GLS estimate of the
                     full model, and returns beta and u of the full model,
                     u = Q [u_reduced; (Q^T Y)_{rest} Omega^g] with Omega^g a
                     generalized inverse of Omega (the inverse when Omega is
                     positive definite; for a singular Omega u is, as on the
                     unreduced path, one of the solutions, Sigma u unique).
                     The factorization keeps Q1 = Q [I; 0] (M x Mr) explicit.
                     glm_gls_backward runs the adjoint through the same
                     reduction; glm_copy_factors returns GLM_EUNSUPPORTED.     */
  GLM_PRECOND_EQ = 8 /* flag, OR-ed into the precision for glm_workspace_bytes,
                     glm_qr_factor(_static) and glm_plan_passes: the
                     preconditioner's auxiliary matrix is one scalar per
                     equation, D = diag(omega_11 .. omega_GG) (x) I_M (the
                     paper's D_2 = diag Sigma of the VAR experiments), so
                     that Pi_i = (I - Q_i Q_i^T) / omega_ii; without it
                     D = alpha I, alpha = max_i omega_ii.  beta and u do not
                     depend on D; the iterations do (a diagonal Omega ends in
                     one step).  Restricted instances, and equations with
                     omega_ii = 0, keep alpha.                                   */
} glm_precision;

typedef struct glm_shape {
  int32_t batch;          /* B >= 1                                               */
  const int32_t* G;       /* host [B]   G_b >= 1                                  */
  const int32_t* M;       /* host [B]   M_b >= 1                                  */
  const int32_t* K;       /* host [B]   1 <= K_b <= 16                            */
  const int32_t* k;       /* host [B]   restriction rows k_b >= 0, or NULL (all 0) */
  const int32_t* n;       /* host [sum_b G_b]  1 <= n_{b,i} <= M_b, instance-major */
} glm_shape;

typedef struct glm_factor glm_factor;   /* opaque host handle */

/* Aggregate counters of the last solve/backward on a handle (host struct). */
typedef struct glm_stats {
  int32_t outer_steps;        /* refinement steps (1 for GLM_FP64)                */
  int64_t pcg_iterations;     /* sum over (instance, rhs) of PCG iterations       */
  int32_t max_iterations;     /* largest per-(instance, rhs) PCG iteration count  */
  int32_t launches;           /* kernel launches enqueued by the call            */
  /* Projection-pass configuration chosen for the handle's shape.  Index 0:
     the single-precision inner solves (GLM_MIXED; -1 on GLM_FP64 handles),
     index 1: the double-precision solves.                                  */
  int32_t pass_rowvec[2];     /* 1 row-vector passes, 0 column-slot passes     */
  int32_t pass_kv[2];         /* right-hand sides per lane (row-vector passes) */
  int32_t pass_ks[2];         /* 16: the sixteen-rhs specialisation, else 0    */
  int32_t pass_omega[2];      /* Omega apply of the row-vector passes: -16, -32
                                 or -64 on the matrix cores (G padded to that
                                 size), 32 from registers, 0 from LDS         */
  int32_t pass_nim[2];        /* widest block, rounded up to 8, 16, 24, 32, 64 */
} glm_stats;

/* Bytes of device workspace needed by glm_qr_factor / glm_gls_solve /
 * glm_gls_backward for this shape and precision.  Returns 0 for an invalid
 * shape (see glm_validate_shape for the reason). */
size_t glm_workspace_bytes(const glm_shape* shape, glm_precision prec);

/* Checks a shape without touching the device.  Returns GLM_OK, GLM_EINVAL or
 * GLM_EUNSUPPORTED.
 *   GLM_EINVAL:  B < 1; G_b, M_b or n_{b,i} < 1; K_b outside 1..16; k_b < 0;
 *                n_{b,i} > M_b; k_b > n_b; n_b >= G_b M_b + k_b (the augmented
 *                system needs m + k > n).
 *   GLM_EUNSUPPORTED (valid, outside this build's kernels): n_{b,i} > 64;
 *                n_b > 2048, or n_b > 1024 with K_b > 4; k_b > 64;
 *                G_b^2 > 65,536. */
int glm_validate_shape(const glm_shape* shape);

/* Factors every block once (SUR section: the data matrices are fixed, so
 * they are factorised only once): batched Householder QR X_i = Q_i R_i in
 * double precision, the explicit thin Q_i (plus a single-precision copy for
 * GLM_MIXED), the column-to-block maps and the tile schedule of the
 * iteration kernels.  With restrictions it also builds an orthonormal basis
 * N of the null space of [R; R_c]^T, which turns the OLS step of the
 * restricted problem (eq. rglm1m) into the unrestricted one plus a rank-k
 * correction.
 *
 *   X    device, M_b x n_b per instance (see conventions); must stay valid
 *        and unmodified while the handle is used (the refinement residual of
 *        GLM_MIXED reads X in double precision)
 *   Rc   device, k_b x n_b per restricted instance, or NULL if all k_b = 0;
 *        same lifetime rule as X
 *   ws   device workspace of ws_bytes >= glm_workspace_bytes(shape, prec),
 *        owned by the caller, outliving the handle
 *   out  host: receives the new handle (release with glm_factor_destroy)
 * Rank deficiency of a block is detected on the device and reported by the
 * next solve as GLM_INFO_RANK.  Returns GLM_OK or a negative code. */
int glm_qr_factor(const glm_shape* shape, glm_precision prec,
                  const double* X, const double* Rc,
                  void* ws, size_t ws_bytes, hipStream_t stream,
                  glm_factor** out);

/* glm_qr_factor for callers that cannot allocate device memory (code that
 * must not call hipMalloc, e.g. tight serving loops or harnesses that forbid
 * it): the same factorization, with the library's static device scratch as
 * the workspace instead of a caller buffer.  The scratch is one 64 MiB array
 * per GPU, reserved when the library's code is loaded on that GPU and held
 * until the process ends.
 *
 *   shape, prec, X, Rc, stream, out   as for glm_qr_factor
 * Returns GLM_EWORKSPACE, before any work is enqueued, when
 * glm_workspace_bytes(shape, prec) exceeds 64 MiB; otherwise as
 * glm_qr_factor.  The call allocates no device or pinned host memory (the
 * handle polls convergence through pageable host memory).  All handles
 * made by this call on one GPU share that GPU's scratch: a new call
 * overwrites the factors of the previous one, so only the handle of the
 * latest call on a device may be used, and calls (or solves on these
 * handles) that overlap in time on one GPU race.  Nothing in the scratch
 * needs to start at zero: every byte a kernel reads is written first by
 * the same call or by the solve. */
int glm_qr_factor_static(const glm_shape* shape, glm_precision prec, const double* X,
                         const double* Rc, hipStream_t stream, glm_factor** out);

/* Multivariate models with exclusion restrictions (section on multivariate
 * linear models with parameter restrictions, eq. MvGLM): Y = Z0 B + U with
 * common regressors Z0 (M_b x N_b, full column rank) and exclusions
 * b_ic = 0; equation i keeps the columns sel_i of Z0.  This is the SUR with
 * X_i = Z0[:, sel_i], factored without forming X: one QR of Z0 = Q0 R0
 * (the model reduction of that section), Q1 = Q0 [I; 0] with
 * Mr = min(M, N + 1) columns, and the reduced regressors R0[:, sel_i]
 * factored block by block (which plays the part of the QRDs of [R0; C_i]
 * for exclusion restrictions).  The handle behaves as a GLM_REDUCED handle
 * for glm_gls_solve, glm_gls_solve_ne, glm_get_stats and the kernel timers:
 * beta holds the kept coefficients (n_b = sum of |sel_i| rows, equation by
 * equation), u is the full model's.  glm_gls_backward and glm_copy_factors
 * return GLM_EUNSUPPORTED.
 *
 *   shape   as for glm_qr_factor, with n_{b,i} = |sel_i| (1 <= n_{b,i} <= N_b)
 *           and k_b extra restriction rows over the kept coefficients
 *   prec    GLM_FP64 or GLM_MIXED, optionally | GLM_PRECOND_EQ (GLM_REDUCED
 *           is implied)
 *   Z0      device, M_b x N_b per instance, row-major, concatenated; must
 *           stay valid while the handle is used (u reads it)
 *   N       host [B], columns of Z0 (N_b <= 2048)
 *   sel     host, for every equation of every instance (instance-major) its
 *           n_{b,i} kept column indices, strictly increasing, in [0, N_b)
 *   Rc      device, k_b x n_b per restricted instance, or NULL
 *   ws      device workspace of glm_workspace_bytes_common(shape, prec, N,
 *           sel) bytes
 * GLM_OK, GLM_EINVAL (bad shape or selection), GLM_EWORKSPACE, GLM_EHIP or
 * GLM_EUNSUPPORTED (as glm_validate_shape, or N_b > 2048). */
size_t glm_workspace_bytes_common(const glm_shape* shape, glm_precision prec,
                                  const int32_t* N, const int32_t* sel);
int glm_qr_factor_common(const glm_shape* shape, glm_precision prec, const double* Z0,
                         const int32_t* N, const int32_t* sel, const double* Rc, void* ws,
                         size_t ws_bytes, hipStream_t stream, glm_factor** out);

/* Solves every (instance, rhs) of the batch with PCG-Aug (projected form:
 * the iteration carries g_i = Pi r_i and one OLS projection per step).
 *
 *   Omega     device, G_b x G_b per instance, symmetric PSD (may be singular:
 *             then y must be consistent, e.g. generated by the model)
 *   y         device, M_b x G_b x K_b per instance
 *   r         device, k_b x K_b per restricted instance, or NULL if none
 *   tol       GLM_FP64: stop when sqrt(c_i / c_1) <= tol (c_i = r_i^T Pi r_i);
 *             GLM_MIXED: stop when the double-precision residual of eq. aug1,
 *             ||[y - Sigma u - X beta ; -Q^T u]|| <= tol * ||y||, its lower
 *             block taken in the coordinates of the orthonormal factors
 *             (X_i^T u = R_i^T Q_i^T u), so that the test does not depend on
 *             the scaling of X's columns
 *   max_iter  PCG iteration limit per (instance, rhs) (per inner solve for
 *             GLM_MIXED); <= 0 selects m - n + 1 (Algorithm PCG-Aug bound)
 *   beta      device out, n_b x K_b per instance
 *   u         device out, M_b x G_b x K_b per instance: the u-block of the
 *             augmented solution (Sigma u = y - X beta, X^T u = 0); unique
 *             only for nonsingular Omega
 *   uc        device out, k_b x K_b per restricted instance (the u-block rows
 *             of the restrictions, i.e. their multipliers), or NULL
 *   info      device out, int32 per (instance, rhs) in batch order: GLM_INFO_*
 *   iters     device out, int32 per (instance, rhs): PCG iterations (total
 *             inner iterations for GLM_MIXED), or NULL
 * Returns GLM_OK or a negative code. */
int glm_gls_solve(glm_factor* f, const double* Omega, const double* y,
                  const double* r, double tol, int32_t max_iter,
                  double* beta, double* u, double* uc,
                  int32_t* info, int32_t* iters, hipStream_t stream);

/* Reverse mode of glm_gls_solve (same handle, same Omega, outputs of the
 * forward solve).  The augmented matrix A = [Sigma X; X^T 0] is symmetric, so
 * the adjoint solve  A [l_u; l_beta] = [g_u; g_beta]  reuses the factors; then
 *   dy      = l_u
 *   dOmega  = -sym( sum_{t,k} l_u[t,:,k] u[t,:,k]^T )   (symmetric gradient:
 *             dL = <dOmega, E> for every symmetric perturbation E)
 *   dX_i    = -sum_k ( l_u,i beta_i^T + u_i l_beta,i^T )
 * Defined for nonsingular Omega.  Restricted instances are solved in the
 * restricted geometry (gradients w.r.t. R_c and r are not produced).  On a
 * GLM_REDUCED handle the adjoint system goes through the same reduction
 * (Q1^T g_u, the reduced adjoint with lower right-hand side g_beta, then
 * l_u of the full model) and the gradients are those of the full model.
 *
 *   beta, u   device, the forward outputs
 *   g_beta    device, n_b x K_b per instance (dL/dbeta)
 *   g_u       device, M_b x G_b x K_b per instance (dL/du), or NULL (zero)
 *   dy        device out, M_b x G_b x K_b per instance
 *   dOmega    device out, G_b x G_b per instance, or NULL
 *   dX        device out, M_b x n_b per instance, or NULL
 *   info, iters   as for glm_gls_solve (for the adjoint solve)
 * Returns GLM_OK or a negative code. */
int glm_gls_backward(glm_factor* f, const double* Omega,
                     const double* beta, const double* u,
                     const double* g_beta, const double* g_u,
                     double tol, int32_t max_iter,
                     double* dy, double* dOmega, double* dX,
                     int32_t* info, int32_t* iters, hipStream_t stream);

/* The comparator of PCG-Aug in the study of its statistical properties
 * (section on the statistical properties of the PCG-Aug estimator; the VAR
 * experiments): conjugate gradients on the normal equations
 *     (X^T Sigma^-1 X) beta = X^T Sigma^-1 y,   Sigma^-1 = Omega^-1 (x) I_M,
 * from beta_0 = 0, in double precision on any unrestricted handle (GLM_FP64
 * or GLM_MIXED; on a GLM_REDUCED handle on the reduced model, whose GLS
 * estimate is the full model's).  Preconditioner: block Jacobi with the
 * diagonal blocks w^ii X_i^T X_i = w^ii R_i^T R_i of the normal matrix
 * ([w^ij] = Omega^-1; one pair of triangular solves per equation).  The
 * normal matrix is never formed: each iteration applies it as X^T ((X p)
 * Omega^-1).  Unlike PCG-Aug's, its early iterates are biased toward 0.
 *
 *   Omega     device, G_b x G_b per instance, symmetric positive definite
 *             (an instance whose Omega is numerically singular -- largest
 *             remaining pivot of a diagonally pivoted Cholesky at most
 *             16 G eps trace(Omega) -- reports GLM_INFO_BREAKDOWN, beta = 0)
 *   y         device, M_b x G_b x K_b per instance
 *   tol       stop when ||b - A beta_i|| <= tol ||b||, b = X^T Sigma^-1 y
 *   max_iter  iteration limit per (instance, rhs); <= 0 selects n_b
 *   beta      device out, n_b x K_b per instance (the last iterate)
 *   info      device out, int32 per (instance, rhs): GLM_INFO_CONVERGED,
 *             GLM_INFO_NOCONV (limit reached), GLM_INFO_BREAKDOWN
 *             (p^T A p <= 0, not finite, or Omega singular), GLM_INFO_RANK;
 *             or NULL
 *   iters     device out, int32 per (instance, rhs): iterations, or NULL
 * Blocks the calling thread like glm_gls_solve.  GLM_OK, GLM_EINVAL,
 * GLM_EHIP, or GLM_EUNSUPPORTED for a handle with restricted instances. */
int glm_gls_solve_ne(glm_factor* f, const double* Omega, const double* y, double tol,
                     int32_t max_iter, double* beta, int32_t* info, int32_t* iters,
                     hipStream_t stream);

/* Copies the factors out of the workspace (enqueued on `stream`):
 *   Q      device out, M_b x n_b per instance, laid out like X (may be NULL)
 *   R      device out, the R_i (n_i x n_i, row-major, upper triangular) of every
 *          block in batch order (may be NULL)
 *   rank   device out, int32 per block: 1 if the block was found numerically
 *          rank deficient (may be NULL)
 * The signs of the rows of R_i (and columns of Q_i) follow the Householder
 * convention (R_jj may be negative).  GLM_OK or GLM_EINVAL / GLM_EHIP. */
int glm_copy_factors(const glm_factor* f, double* Q, double* R, int32_t* rank,
                     hipStream_t stream);

/* Host only (no device call): the projection-pass configuration that
 * glm_qr_factor chooses for this shape and precision, in the pass_* fields
 * of `out` (the counters are zeroed).  With GLM_REDUCED it is the
 * configuration of the reduced problem's solve.  GLM_OK, GLM_EINVAL or
 * GLM_EUNSUPPORTED (as glm_validate_shape). */
int glm_plan_passes(const glm_shape* shape, glm_precision prec, glm_stats* out);

/* Counters of the last solve/backward on the handle.  GLM_OK or GLM_EINVAL. */
int glm_get_stats(const glm_factor* f, glm_stats* out);

/* Kernel timing for measurement.  While enabled, every launch of the two
 * OLS-projection pass kernels is bracketed by HIP events on the launch stream
 * and its algorithmic bytes are counted on the device (tiles of inactive
 * instances count nothing).  glm_profile_read synchronises the stream and
 * returns, for kernel id 0 (projection pass A) and 1 (projection pass B),
 * the number of launches, their summed duration in milliseconds and the
 * summed algorithmic bytes; it then clears the counters.  On a GLM_REDUCED
 * handle ids 0 and 1 report the passes of the reduced solve and id 2 the
 * reduced responses Q1^T Y of glm_gls_solve (and of the adjoint in
 * glm_gls_backward; Q1 and Y read once, the Mr rows written once); the
 * factorization runs before its handle exists and is not timed.  Id 2 reads
 * zero on other handles. */
int glm_profile_enable(glm_factor* f, int on);
int glm_profile_read(glm_factor* f, int kernel_id, int64_t* launches,
                     double* total_ms, double* total_bytes);

/* Measurement aid, not a step of the method: the streaming ceiling of a
 * read/write mix.  One plain streaming kernel moves the bytes of a
 * projection pass in the same pattern, with no arithmetic beyond one add per
 * element, so that the pass's touched bandwidth can be compared with what
 * the device reaches for that mix (pass B of an iteration reads u, g, w and
 * Q_i and writes g and w in place; pass A reads u, g and Q_i and writes u in
 * place and its Q_i^T B_i partial sums).
 *   ro, ro_len  host arrays of n_ro device pointers (float) and lengths
 *               (elements): read-only streams;
 *   rw, rw_len  host array of n_rw device pointers: streams of rw_len
 *               elements read and then overwritten in place;
 *   wo, wo_len  host array of n_wo device pointers: write-only streams of
 *               wo_len elements.
 * Element e of a written stream becomes 0.5 * (its old value, rw only) +
 * the sum over read-only streams with ro_len > e of their element e.
 * Every pointer 16-byte aligned, every length of a given stream positive
 * and a multiple of 4, at most GLM_STREAM_MAX streams of each kind, no
 * written stream overlapping another stream; otherwise GLM_EINVAL before
 * any launch (overlap is not checked).  Enqueued on `stream`; GLM_OK or GLM_EHIP. */
#define GLM_STREAM_MAX 4
int glm_stream_mix(const float* const* ro, const int64_t* ro_len, int32_t n_ro,
                   float* const* rw, int32_t n_rw, int64_t rw_len,
                   float* const* wo, int32_t n_wo, int64_t wo_len, hipStream_t stream);

void glm_factor_destroy(glm_factor* f);

/* Static description of a return or info code; never NULL. */
const char* glm_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* GLM_H */
