// Internal descriptors and launch helpers shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace glm {

constexpr int NT = 256;          // threads per workgroup of the tile kernels
constexpr int KMAX = 16;         // right-hand sides per instance
constexpr int QR_NMAX = 64;      // widest block the QR kernel factors
constexpr int NMAX_INST = 8 * NT; // widest instance (n = sum of n_i) of any path
// doubles of LDS of the full-model u kernel: Omega^g when G <= 32, then one or
// more rows of X (n) and Y (G K); the reduction plans reject shapes whose row
// does not fit
constexpr int RED_U_LDS = 5120;

// Per-(instance, rhs) iteration status.
enum : int {
  ST_ACTIVE = 0,
  ST_CONVERGED = 1,
  ST_BREAKDOWN = 2,
  ST_STAGNATED = 3,
  ST_MAXITER = 4,
  ST_RANK = 5,
  ST_IDLE = 6,     // not part of the current (inner) solve
};

struct InstDesc {
  int G, M, K, kc, n;
  int blk0;        // first block (equation) index in the BlockDesc table
  int rhs0;        // first (instance, rhs) state index
  int tile0;       // first tile of this instance
  int ntiles;
  int rs_t[2];     // rows per LDS-staged sub-tile of the passes (FP32, FP64)
  int rpar_t[2];   // row groups per workgroup of the passes (FP32, FP64)
  int tps_t[2];    // per-tile partial slots of pass A's Q^T B (FP32, FP64): the
                   // row groups, or fewer where pass A combines them in-kernel
  int rsa_t[2];    // rows per sub-tile of pass A (FP32, FP64)
  int maxit;       // PCG iteration bound m - n + 1
  int nimax;       // largest n_i of the instance
  int64_t tp_stride;  // elements per tile partial: max(tps n K, G G)
  int64_t q_off;   // Q / X (M x n)
  int64_t v_off;   // vectors (M x G x K)
  int64_t om_off;  // Omega (G x G)
  int64_t b_off;   // beta-like (nsub x K)
  int64_t t_off;   // reduced projections ((n + kc) x K)
  int64_t col_off; // column -> block map (n)
  int64_t c_off;   // restriction vectors (kc x K)
  int64_t rc_off;  // R_c (kc x n)
  int64_t nb_off;  // null-space basis N ((n + kc) x kc)
};

struct BlockDesc {
  int inst, eq, col, ni;
  int64_t r_off;   // R_i (ni x ni, row-major, upper triangular)
};

struct TileDesc {
  int inst, row0, rows, part;  // part = index of the tile within its instance
  int64_t tp_off;              // element offset of this tile's partial projection (n x K)
};

struct QRJob {
  int64_t a_off;   // first element of the block inside the factored array
  int rows, cols, ld;
  int flag;        // index into the rank-flag array
  int64_t r_off;   // where R (cols x cols) goes, or -1
};

struct RhsState {
  double c, c1, d, lam, mu, cmin;
  double rnorm2, ynorm2;       // refinement residual and reference norms (mixed)
  double itol;                 // inner tolerance of an FP64 refinement solve (0: default)
  int status, iters, since, total_iters;
  int esc;                     // mixed path: inner solves continue in FP64
  int pad;
};

// Pass geometry of precision T (index 0 = FP32, 1 = FP64).
template <typename T>
__host__ __device__ inline int rows_of(const InstDesc& in) {
  return in.rs_t[sizeof(T) == 8];
}
template <typename T>
__host__ __device__ inline int rows_a_of(const InstDesc& in) {
  return in.rsa_t[sizeof(T) == 8];
}
template <typename T>
__host__ __device__ inline int rpar_of(const InstDesc& in) {
  return in.rpar_t[sizeof(T) == 8];
}
template <typename T>
__host__ __device__ inline int tps_of(const InstDesc& in) {
  return in.tps_t[sizeof(T) == 8];
}
// Matrix-core passes (FP32, sixteen rhs): the partial slots pass A writes per
// tile for G padded to gp.  gp <= 16: the rows of a wave are summed by lane
// shuffles, one slot per wave; gp = 32 and 64: one slot per row group (64 / gp;
// summing the two waves of gp = 32 through LDS cost pass A more time than it
// saved in partial traffic).
__host__ __device__ inline int mf_partial_slots(int gp) { return gp <= 16 ? 4 : 64 / gp; }

struct RedChunk {
  int inst, p0;
};

// Model reduction of one SUR instance: W = [X_1 ... X_G] = Q [R; 0] by
// Householder panels of 32 columns; the reduced model keeps Mr = min(M, n + 1)
// rotated observations.
struct RedDesc {
  int M, n, G, K, Mr;
  int kr;          // reflectors: min(M, n)
  int rhs0;        // first (instance, rhs) index
  int inst;        // batch index of the instance
  int nseg0;       // row segments of the first panel's TSQR (ceil(M / 256))
  int nsub;        // columns of the reduced regressors (sum of n_i); n (the
                   // columns of W) is equal except for common regressors
  int sel_off;     // common regressors: first entry of the instance's column
                   // selection (sum of n_i entries); otherwise 0
  int64_t leaf_off;  // T factors of the TSQR leaves (panels x nseg0 x 32 x 32)
  int64_t stk_off;   // stacked R factors / tree reflectors (panels x nseg0 x 32 x 32)
  int64_t w_off;   // W copy: reflectors and R (M x n, row-major); also X and dX
  int64_t q1_off;  // Q1 = Q [I; 0] (M x Mr)
  int64_t b_off;   // beta-like (nsub x K)
  int64_t v_off;   // full vectors (M x G x K)
  int64_t xr_off;  // reduced regressors (Mr x nsub)
  int64_t vr_off;  // reduced vectors (Mr x G x K)
  int64_t tau_off; // reflector scalars (n)
  int64_t t_off;   // block-reflector factors T (panels x 32 x 32)
  int64_t om_off;  // Omega (G x G)
  int64_t zp_off;  // per-segment dOmega partials of the reverse mode
                   // (ceil(M / RED_SEG) x G G)
};

// One 64 x 64 output tile of a batched product with Q1 (inst < 0: padding).
struct GemmTile {
  int inst, i0, j0, pad;
};
constexpr int RED_PANEL = 32;    // columns per Householder panel
constexpr int RED_SEG = 512;     // rows per workgroup of the reverse-mode dOmega partials
constexpr int RED_LEAF = 256;    // rows per TSQR leaf segment

// Arguments of the two projection-pass kernels (host side).
template <typename T>
struct PassLaunch {
  const InstDesc* insts;
  const TileDesc* tiles;
  int ntiles;
  const BlockDesc* blks;
  const int* colblk;
  const int* inst_active;
  const T* Q;
  const T* Om;
  const double* alpha;
  const double* deq;   // per-block D scalars (D = diag(d) (x) I_M), or null: D = alpha I
  const RhsState* st;
  const T* y;
  T* w;
  T* g;
  T* u;
  const T* Tm;
  T* Tpart;
  double* dpart;
  double* cpart;
  unsigned long long* bytes;
  int w_nonzero;
  int kc_t;        // K bucket (1, 2, 4, 8, 16)
  int sl;          // column slots per thread (1, 2, 3, 4, 8)
  size_t lds;      // dynamic LDS bytes
  int rowpass;     // row-vector passes (otherwise the column-slot passes)
  int kv;          // row-vector passes: right-hand sides per lane (1, 2, 4)
  int ks;          // row-vector passes: 16 when every instance has K = 16, else 0
  int gr;          // row-vector passes: Omega column in registers up to this G (0: LDS)
  int nim;         // row-vector passes: bound on n_i (8, 16, 24, 32, 64)
};

// Row-vector projection passes: workgroup size, per-thread staging capacity
// (vector chunks of kv elements, Q scalars) and the register budget of the
// per-lane projection slice (n_i bound x kv x 32-bit words per element).
constexpr int PROJ_NT = 256;
constexpr int PROJ_NV = 8;
constexpr int PROJ_NQ = 8;
constexpr int PROJ_NQA = 16;         // Q scalars per thread in pass A (two vector slabs)
constexpr int PROJ_NVB = 10;         // vector chunks per thread in pass B (three slabs)
constexpr int PROJ_NQB = 10;         // Q scalars per thread in pass B
constexpr int PROJ_QPAD = QR_NMAX;   // zeros after the staged Q rows
constexpr int kProjSliceRegs = 128;


// ---- launchers (defined next to their kernels) ----------------------------
hipError_t launch_qr(const QRJob* d_jobs, int njobs, int nmax, double* A, double* R,
                     int* flags, hipStream_t s);
hipError_t launch_to_float(const double* src, float* dst, int64_t count, hipStream_t s);
hipError_t launch_nullbasis_input(const InstDesc* insts, const int* rinst, int nr,
                                  const BlockDesc* blks, const double* R, const double* Rc,
                                  double* Nb, hipStream_t s);
template <typename T>
hipError_t launch_pass_a(const PassLaunch<T>& p, int mode, hipStream_t s);
template <typename T>
hipError_t launch_pass_b(const PassLaunch<T>& p, int mode, hipStream_t s);
template <typename T>
hipError_t launch_proj(const PassLaunch<T>& p, bool pass_a, int mode, hipStream_t s);
template <typename T>
hipError_t launch_reduce_t(const InstDesc* insts, const TileDesc* tiles, const int* inst_active,
                           const void* chunks, int nchunks, const T* Tpart, T* Tm,
                           int use_rpar, hipStream_t s);
template <typename T>
hipError_t launch_scalar_a(const InstDesc* insts, const TileDesc* tiles, const int* inst_active,
                           RhsState* st, const double* dpart, T* Tm, const double* Nb,
                           const double* rvec, int B, int mode_iter, int do_d, hipStream_t s);
hipError_t launch_scalar_b(const InstDesc* insts, int* inst_active, int* inst_count,
                           RhsState* st, const double* cpart, const double* alpha,
                           const void* Tm, int t_is_double, double* gc, double* uc,
                           double* wc, const double* rvec, int B, int mode_iter,
                           double tol, int stall, int maxit_cap, hipStream_t s);
hipError_t launch_count(const int* inst_count, int B, int* out, hipStream_t s);
template <typename TS, typename TD, bool UPPER, bool ADD>
hipError_t launch_trisolve(const InstDesc* insts, const BlockDesc* blks, int nblk,
                           const int* inst_active, const RhsState* st, int need_active,
                           const double* R, const TS* src, int src_is_t, TD* dst,
                           int dst_is_t, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* p, int64_t count, T v, hipStream_t s);
hipError_t launch_alpha(const InstDesc* insts, int B, const double* Om, double* alpha,
                        float* Om32, double* deq, hipStream_t s);
hipError_t launch_state_init(const InstDesc* insts, int B, const int* rankflag,
                             int rank_extra_base, const int* rinst_index, RhsState* st,
                             int* inst_active, int* ost, hipStream_t s);
hipError_t launch_activate(const InstDesc* insts, int B, const RhsState* st, int* inst_active,
                           hipStream_t s);
template <typename T>
hipError_t launch_copy_tc(const InstDesc* insts, int B, const T* Tm, double* wc,
                          hipStream_t s);
hipError_t launch_outer_check(const InstDesc* insts, const BlockDesc* blks, const double* R,
                              int B, int* inst_active, RhsState* st,
                              int* ost, const double* rpart, const double* ypart,
                              const double* XtW, double xtw_sign, const double* h2,
                              const double* Rc,
                              const double* rvec, const double* beta, const double* wc,
                              double* rho0, double* rhoc, double tol, int step,
                              int last_step, hipStream_t s);
template <typename T>
hipError_t launch_update_u(const InstDesc* insts, const TileDesc* tiles, int ntiles,
                           const int* inst_active, const RhsState* st, const T* du,
                           double* u, hipStream_t s);
hipError_t launch_beta_to_t(const InstDesc* insts, int B, const double* beta, double* Tm,
                            hipStream_t s);
hipError_t launch_eye(const InstDesc* insts, int B, double* E, hipStream_t s);
hipError_t launch_select_inner(const InstDesc* insts, int B, RhsState* st, const int* ost,
                               int* inst_active, int want, hipStream_t s);
hipError_t launch_update_c(const InstDesc* insts, int B, const RhsState* st,
                           const double* dwc, double* wc64, hipStream_t s);
hipError_t launch_red_panel(const RedDesc* d, int B, int panel, int maxseg, int maxcols,
                           double* W, double* Tleaf, double* Stk, double* tau, double* T,
                           hipStream_t s);
hipError_t launch_red_q1_panel(const RedDesc* d, int B, int panel, int maxseg, int maxcols,
                              const double* W, const double* Tleaf, const double* Stk,
                              const double* T, double* Q1, hipStream_t s);
hipError_t launch_red_qinit(const RedDesc* d, int B, double* Q1, hipStream_t s);
hipError_t launch_red_extract(const RedDesc* d, int B, const double* W, const int* ex,
                             const int* sel, double* Xr, hipStream_t s);
hipError_t launch_red_equilibrate(const RedDesc* d, int B, int maxM, const double* X, int* ex,
                                  double* W, hipStream_t s);
hipError_t launch_red_gemm_tn(const RedDesc* d, const GemmTile* tiles, int ntiles,
                             const double* Q1, const double* Y, double* Yr, hipStream_t s);
hipError_t launch_red_ginv(const RedDesc* d, int B, const double* Om, double* A, double* Og,
                          int* sing, hipStream_t s);
hipError_t launch_red_u(const RedDesc* d, int B, int maxM, const InstDesc* sinst,
                       const BlockDesc* sblk, const int* sel, const double* X,
                       const double* beta,
                       const double* Y, const double* Og, double* U, hipStream_t s);
hipError_t launch_red_singular(const RedDesc* d, int B, int chunks, const GemmTile* tiles2,
                              int ntiles2, const int* sing, const double* Om, const double* Og,
                              const double* Q1, const double* Ur, double* D, double* U,
                              hipStream_t s);
hipError_t launch_red_grad(const RedDesc* d, int B, int maxM, const InstDesc* sinst,
                          const int* colblk, const double* L, const double* U,
                          const double* beta, const double* lb, double* part, double* dOm,
                          double* dX, hipStream_t s);
hipError_t launch_ne_oinv(const InstDesc* insts, int B, const double* Om, double* A,
                          double* Oinv, RhsState* st, int* inst_active, hipStream_t s);
hipError_t launch_ne_start(const InstDesc* insts, const BlockDesc* blks, int B, const double* R,
                           const double* Oinv, const double* Tm, double* x, double* r,
                           double* z, double* p, RhsState* st, int* inst_active, int* icount,
                           hipStream_t s);
hipError_t launch_ne_step(const InstDesc* insts, const BlockDesc* blks, int B, const double* R,
                          const double* Oinv, const double* Tm, double* x, double* r,
                          double* z, double* p, RhsState* st, int* inst_active, int* icount,
                          double tol, int maxit_user, hipStream_t s);
hipError_t launch_grad(const InstDesc* insts, const TileDesc* tiles, int ntiles, int B,
                       const int* colblk, const double* L, const double* U,
                       const double* beta, const double* lb, double* part, double* dOm,
                       double* dX, hipStream_t s);

// pass-kernel modes
enum : int { PASS_A_ITER = 0, PASS_A_RHS = 1 };
enum : int { PASS_B_ITER = 0, PASS_B_INIT = 1, PASS_B_EXPAND = 2 };

}  // namespace glm
