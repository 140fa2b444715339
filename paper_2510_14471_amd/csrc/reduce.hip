// SUR model reduction (the remark on reducing the SUR model in the SUR
// section): one Householder QR of W = [X_1 ... X_G] = Q [R; 0] per instance.
// Rotating every equation by Q^T keeps Sigma = Omega (x) I_M, and the rotated
// rows t >= n carry no information on beta, so the GLS of the first
// Mr = min(M, n + 1) rotated rows is the GLS of the full model.
//
// Factorization (once per W): panels of RED_PANEL columns, each factored
// TSQR-wise (independent row segments, then the stack of their R factors)
// and applied to the trailing columns of W; then the explicit first Mr
// columns of Q = Q_0 Q_1 ..., Q1 = Q [I; 0] (M x Mr), accumulated backwards.
//   k_tsqr_leaf, k_tsqr_tree       factor panel p (below)
//   k_leaf_apply_mf, k_tree_apply_mf   C <- Q_p^T C (trailing columns of W)
//                                      or C <- Q_p C (Q1), on the FP64
//                                      matrix cores
//   k_red_qinit       Q1 <- [I; 0]
//   k_red_extract     reduced regressors (the rows of R)
// Solve (per right-hand side block Y, M x G K):
//   k_red_gemm_tn     reduced responses Y_red = Q1^T Y
//   k_red_ginv        a generalized inverse Omega^g by pivoted Cholesky (the
//                     inverse for positive definite Omega) and its rank
//   k_red_u           U = (Y - [X_i beta_i]) Omega^g
//   k_red_delta       (singular Omega) D = U_red - U_red Omega Omega^g
//   k_red_gemm_nn     (singular Omega) U += Q1 D
// which is U = Q [U_red; (Q^T Y)_{t >= Mr} Omega^g]: with
// Q Q^T = Q1 Q1^T + Q2 Q2^T and Y_red = X_red beta + U_red Omega,
//   Q1 U_red + (I - Q1 Q1^T) Y Omega^g = (Y - W beta) Omega^g + Q1 U_red (I - Omega Omega^g).
// Reverse mode on a reduced handle reuses the same path for the adjoint and
//   k_red_grad_omega_part/_reduce, k_red_grad_x   dOmega and dX of the full model.
#include "glm.h"
#include "glm_internal.h"
#include "ginv.h"
#include "qr_panel.h"

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>

namespace glm {

namespace {

constexpr int RP = RED_PANEL;
constexpr int EQ_ROWS = 512;   // rows per workgroup of the column equilibration

// exponent of a column's scaling (INT_MIN marks a column of zeros: no scaling)
__device__ __forceinline__ int col_exp(int e) { return e == INT_MIN ? 0 : e; }

// V[r][j] of panel rows r (relative to the panel's first row): the unit
// diagonal and zeros above it are implicit in the stored factorization.
__device__ __forceinline__ double vpanel(const double* __restrict__ a0, int ld, int r, int j,
                                         int rows, int w) {
  if (j >= w || r >= rows) return 0.0;
  if (r == j) return 1.0;
  return r > j ? a0[(int64_t)r * ld + j] : 0.0;
}

// Panel factorization, TSQR form.  Panel p holds the columns [c0, c0 + w),
// c0 = 32 p, of the rows [c0, M).  Those rows are cut into segments of TS
// rows; every segment is factored on its own (leaf: A_s = Q_s [R_s; 0]) and
// the R_s, stacked 32 rows apart, are factored once more (tree:
// [R_0; R_1; ...] = Q_t [R; 0]).  The panel's orthogonal factor is
// Q_p = diag(Q_s) Q_t, with Q_t acting on the first rows of the segments, and
// R goes to the panel's first rows.  Each Q_s and Q_t is kept in compact WY
// form, I - V T V^T (T upper triangular): the leaves' V in place in W, the
// tree's V in the stack buffer.
//   k_tsqr_leaf        factor a segment in registers; V_s, T_s; R_s to the stack
//   k_tsqr_tree        factor the stack in place; T_t; R into W
//   k_leaf_apply_mf    C_s <- (I - V_s op(T_s) V_s^T) C_s, one pass over C
//   k_tree_apply_mf    the same with Q_t on the segments' first rows
constexpr int TS = RED_LEAF;      // rows per leaf segment
constexpr int TSJ = TS / 8;       // rows per thread in the leaf factorization (8 row slots)

// T of a block reflector (forward, columnwise): T[j][j] = tau_j,
// T[0:j, j] = -tau_j T[0:j, 0:j] S[0:j, j] with S = V^T V.  Column j needs the
// columns before it; within a column thread i forms entry i.  Called by every
// thread of the workgroup (NT >= 32).
template <int NT>
__device__ void form_t(const double (*S)[RP + 1], const double* tau, int w, double (*Tl)[RP]) {
  const int tid = threadIdx.x;
  for (int e = tid; e < RP * RP; e += NT) Tl[e / RP][e % RP] = 0.0;
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    if (tid < j) {
      double s = 0.0;
      for (int k = tid; k < j; ++k) s += Tl[tid][k] * S[k][j];
      Tl[tid][j] = -tau[j] * s;
    } else if (tid == j) {
      Tl[j][j] = tau[j];
    }
    __syncthreads();
  }
}

// Householder QR of a rows x w block (w <= 32) held in registers: thread
// (slot, c) = (tid / 32, tid % 32) holds column c of rows slot + SL j, j < TJ
// (SL = NT / 32 row slots), zero for rows past the block and columns past w.
// Reflector p: v = [1; x scale], H = I - tau v v^T, a_k -= tau v (pivrow_k +
// scale dsum_k); the sweep that applies reflector p also forms the pivot row
// and the dot products of reflector p + 1.  Every thread forms the
// reflector's scalars itself (the same arithmetic on the same shared values),
// so the two barriers of col_sum are the only ones per reflector: the sweep
// writes the other pivot-row buffer, and dsum and red are rewritten only
// after the next col_sum's first barrier, which every thread reaches after
// its reads of this reflector's values.  On return the registers hold R on
// and above the diagonal and the reflectors below it (LAPACK geqr2
// convention), tau_s the reflector scalars.  Called by every thread.
template <int NT, int TJ>
__device__ __forceinline__ void qr_regs(double (&a)[TJ], int rows, int w,
                                        double (*red)[NT / 64], double* dsum,
                                        double (*pivrow)[32], double* tau_s) {
  constexpr int SL = NT / 32;
  const int tid = threadIdx.x, c = tid & 31, slot = tid >> 5;
  const bool colok = c < w;
  const int ws = min(rows, w);
  if (tid < 32) tau_s[tid] = 0.0;
  double dot = 0.0;
#pragma unroll
  for (int j = 0; j < TJ; ++j) {
    const int r = slot + SL * j;
    const double ap = shfl_col(a[j], 0);
    if (r == 0 && colok) pivrow[0][c] = a[j];
    if (r > 0 && r < rows) dot += ap * a[j];
  }
  for (int p = 0; p < ws; ++p) {
    col_sum<NT>(dot, p, w, red, dsum);
    const double alpha = pivrow[p & 1][p];
    const double xnorm2 = dsum[p];
    double beta, tau, scale;
    if (!(xnorm2 > kQrTinyNorm2)) {
      beta = alpha;
      tau = 0.0;
      scale = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + xnorm2);
      beta = (alpha >= 0.0) ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    if (tid == 0) tau_s[p] = tau;
    const double wkc = (c > p && colok) ? pivrow[p & 1][c] + scale * dsum[c] : 0.0;
    const int q = p + 1;
    dot = 0.0;
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int r = slot + SL * j;
      const double ap = shfl_col(a[j], p);
      if (r >= p && r < rows) {
        const double vv = (r > p) ? ap * scale : 1.0;
        if (c > p) a[j] -= tau * vv * wkc;
        if (c == p) a[j] = (r == p) ? beta : vv;
      }
      const double aq = shfl_col(a[j], q & 31);
      if (r == q && colok) pivrow[q & 1][c] = a[j];
      if (r > q && r < rows && c >= q) dot += aq * a[j];
    }
  }
  __syncthreads();   // pivot rows and tau_s complete
}

// S = V^T V (V with the unit diagonal, w columns) from the registers of
// qr_regs, eight rows of S at a time; per-wave sums go through part (four
// waves at a time), the total into S.  Overwrites a with V.
template <int NT, int TJ>
__device__ __forceinline__ void vtv_regs(double (&a)[TJ], int rows, int w,
                                         double (*part)[RP][RP], double (*S)[RP + 1]) {
  constexpr int SL = NT / 32, NW = NT / 64;
  const int tid = threadIdx.x, c = tid & 31, slot = tid >> 5, wave = tid >> 6;
#pragma unroll
  for (int j = 0; j < TJ; ++j) {
    const int r = slot + SL * j;
    a[j] = (c < w && r < rows) ? (r > c ? a[j] : (r == c ? 1.0 : 0.0)) : 0.0;
  }
  for (int i0 = 0; i0 < RP; i0 += 8) {
    double acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0;
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[i] += shfl_col(a[j], i0 + i) * a[j];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] += __shfl_xor(acc[i], 32, 64);
    // waves 4g .. 4g + 3 add into part[0..3] in turn
    for (int g = 0; g < NW / 4; ++g) {
      if (wave / 4 == g && (tid & 63) < 32)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          if (g == 0) part[wave & 3][i0 + i][c] = acc[i];
          else part[wave & 3][i0 + i][c] += acc[i];
        }
      if (NW > 4) __syncthreads();
    }
  }
  __syncthreads();
  for (int e = tid; e < RP * RP; e += NT) {
    const int i = e / RP, jj = e % RP;
    S[i][jj] = part[0][i][jj] + part[1][i][jj] + part[2][i][jj] + part[3][i][jj];
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256, 3)
k_tsqr_leaf(const RedDesc* __restrict__ descs, int panel, double* __restrict__ W,
            double* __restrict__ Tleaf, double* __restrict__ Stk) {
  const RedDesc d = descs[blockIdx.x];
  const int c0 = panel * RP;
  if (c0 >= d.kr) return;
  const int w = min(RP, d.kr - c0), rows_all = d.M - c0, sg = blockIdx.y, r0 = sg * TS;
  if (r0 >= rows_all) return;
  const int rs = min(TS, rows_all - r0), ws = min(rs, w), ld = d.n;
  double* a0 = W + d.w_off + (int64_t)(c0 + r0) * ld + c0;
  const int tid = threadIdx.x, c = tid & 31, slot = tid >> 5;
  const bool colok = c < w;
  __shared__ double red[32][4];
  __shared__ double dsum[32], pivrow[2][32], tau_s[32];
  __shared__ double S[RP][RP + 1];
  __shared__ double part[4][RP][RP];
  double a[TSJ];
#pragma unroll
  for (int j = 0; j < TSJ; ++j) {
    const int r = slot + 8 * j;
    a[j] = (r < rs && colok) ? a0[(int64_t)r * ld + c] : 0.0;
  }
  qr_regs<256, TSJ>(a, rs, w, red, dsum, pivrow, tau_s);
  // reflectors below the diagonal, R_s on and above it
#pragma unroll
  for (int j = 0; j < TSJ; ++j) {
    const int r = slot + 8 * j;
    if (r < rs && colok) a0[(int64_t)r * ld + c] = a[j];
  }
  // R_s into the stack (32 rows per segment; rows at or past ws and the
  // entries below the diagonal are zero)
  double* stk = Stk + d.stk_off + ((int64_t)panel * d.nseg0 + sg) * RP * RP;
#pragma unroll
  for (int j = 0; j < TSJ; ++j) {
    const int r = slot + 8 * j;
    if (r < RP) stk[r * RP + c] = (r < ws && colok && c >= r) ? a[j] : 0.0;
  }
  // S = V^T V (V with the unit diagonal, ws columns)
  vtv_regs<256, TSJ>(a, rs, ws, part, S);
  double (*Tl)[RP] = part[0];
  form_t<256>(S, tau_s, ws, Tl);
  double* Tp = Tleaf + d.leaf_off + ((int64_t)panel * d.nseg0 + sg) * RP * RP;
  for (int e = tid; e < RP * RP; e += 256) Tp[e] = Tl[e / RP][e % RP];
}

// The tree: the stack (nseg x 32 rows, ld 32) factored in place by one
// workgroup; T_t to the panel's T slot, R into W's first panel rows.
constexpr int RPNT = 1024;
constexpr int RPU = 16;             // rows in flight per lane in the tree passes
constexpr int RPW = RPNT / 64;      // waves per tree workgroup

__global__ void __launch_bounds__(RPNT)
k_tsqr_tree(const RedDesc* __restrict__ descs, int panel, double* __restrict__ W,
            double* __restrict__ Stk, double* __restrict__ tau, double* __restrict__ T) {
  const RedDesc d = descs[blockIdx.x];
  const int c0 = panel * RP;
  if (c0 >= d.kr) return;
  const int w = min(RP, d.kr - c0), nseg = (d.M - c0 + TS - 1) / TS, rows = nseg * RP;
  double* a0 = Stk + d.stk_off + (int64_t)panel * d.nseg0 * RP * RP;
  __shared__ Qr32Shared<RPNT> sh;
  __shared__ double S[RP][RP + 1];
  __shared__ double part[4][RP][RP];
  qr32_factor<RPNT, RPU>(a0, rows, w, RP, sh);
  const int tid = threadIdx.x, c = tid & 31, slot = tid >> 5;
  if (tid < w) tau[d.tau_off + c0 + tid] = sh.tau_s[tid];
  double acc[RP];
#pragma unroll
  for (int i = 0; i < RP; ++i) acc[i] = 0.0;
  constexpr int SU = 4;
  for (int q0 = 0; q0 < rows; q0 += (RPNT / 32) * SU) {
    double v[SU];
#pragma unroll
    for (int q = 0; q < SU; ++q) v[q] = vpanel(a0, RP, q0 + slot + (RPNT / 32) * q, c, rows, w);
#pragma unroll
    for (int q = 0; q < SU; ++q)
#pragma unroll
      for (int i = 0; i < RP; ++i) acc[i] += shfl_col(v[q], i) * v[q];
  }
#pragma unroll
  for (int i = 0; i < RP; ++i) acc[i] += __shfl_xor(acc[i], 32, 64);
  const int wave = tid >> 6;
  for (int g = 0; g < RPW / 4; ++g) {
    if (wave / 4 == g && (tid & 63) < 32)
#pragma unroll
      for (int i = 0; i < RP; ++i) {
        if (g == 0) part[wave & 3][i][c] = acc[i];
        else part[wave & 3][i][c] += acc[i];
      }
    __syncthreads();
  }
  for (int e = tid; e < RP * RP; e += RPNT) {
    const int i = e / RP, j = e % RP;
    S[i][j] = part[0][i][j] + part[1][i][j] + part[2][i][j] + part[3][i][j];
  }
  __syncthreads();
  double (*Tl)[RP] = part[0];
  form_t<RPNT>(S, sh.tau_s, w, Tl);
  double* Tp = T + d.t_off + (int64_t)panel * RP * RP;
  for (int e = tid; e < RP * RP; e += RPNT) Tp[e] = Tl[e / RP][e % RP];
  // the panel's R (upper triangle of the first w rows) into W
  for (int e = tid; e < w * w; e += RPNT) {
    const int i = e / w, j = e % w;
    if (j >= i) W[d.w_off + (int64_t)(c0 + i) * d.n + c0 + j] = a0[i * RP + j];
  }
}

// The tree with the stack in registers (up to 32 TJ rows, TJ <= 24 doubles
// per thread within the 128 VGPRs of a 1024-thread workgroup): the
// arithmetic of k_tsqr_leaf
// on 32 row slots, so that the reflectors' sweeps never leave the
// workgroup.  Leaves the stack, tau, T_t and R as k_tsqr_tree does.
template <int TJ>
__global__ void __launch_bounds__(RPNT)
k_tsqr_tree_reg(const RedDesc* __restrict__ descs, int panel, double* __restrict__ W,
                double* __restrict__ Stk, double* __restrict__ tau, double* __restrict__ T) {
  const RedDesc d = descs[blockIdx.x];
  const int c0 = panel * RP;
  if (c0 >= d.kr) return;
  const int w = min(RP, d.kr - c0), nseg = (d.M - c0 + TS - 1) / TS, rows = nseg * RP;
  double* a0 = Stk + d.stk_off + (int64_t)panel * d.nseg0 * RP * RP;
  const int tid = threadIdx.x, c = tid & 31, slot = tid >> 5;
  __shared__ double red[32][RPW];
  __shared__ double dsum[32], pivrow[2][32], tau_s[32];
  __shared__ double S[RP][RP + 1];
  __shared__ double part[4][RP][RP];
  double a[TJ];
#pragma unroll
  for (int j = 0; j < TJ; ++j) {
    const int r = slot + 32 * j;
    a[j] = (r < rows && c < w) ? a0[r * RP + c] : 0.0;
  }
  qr_regs<RPNT, TJ>(a, rows, w, red, dsum, pivrow, tau_s);
#pragma unroll
  for (int j = 0; j < TJ; ++j) {
    const int r = slot + 32 * j;
    if (r < rows && c < w) a0[r * RP + c] = a[j];
  }
  // the panel's R (upper triangle of the first w rows, slot r, j = 0) into W
  if (slot < w && c < w && c >= slot) W[d.w_off + (int64_t)(c0 + slot) * d.n + c0 + c] = a[0];
  if (tid < w) tau[d.tau_off + c0 + tid] = tau_s[tid];
  vtv_regs<RPNT, TJ>(a, rows, w, part, S);
  double (*Tl)[RP] = part[0];
  form_t<RPNT>(S, tau_s, w, Tl);
  double* Tp = T + d.t_off + (int64_t)panel * RP * RP;
  for (int e = tid; e < RP * RP; e += RPNT) Tp[e] = Tl[e / RP][e % RP];
}

// Target of the applies: the trailing columns of W (TGT_W, op(T) = T^T:
// Q_p^T) or the columns c0.. of Q1 (TGT_Q1, op(T) = T: Q_p).
enum : int { TGT_W = 1, TGT_Q1 = 2 };

struct ApplyTarget {
  double* cb;   // row c0 of the target, first column
  int ncols, ld;
};

template <int TGT>
__device__ __forceinline__ ApplyTarget apply_target(const RedDesc& d, int c0, int w, double* C) {
  ApplyTarget a;
  if (TGT == TGT_W) {
    a.ncols = d.n - c0 - w;
    a.ld = d.n;
    a.cb = C + d.w_off + (int64_t)c0 * d.n + c0 + w;
  } else {
    a.ncols = d.Mr - c0;
    a.ld = d.Mr;
    a.cb = C + d.q1_off + (int64_t)c0 * d.Mr + c0;
  }
  return a;
}

// ---- leaf apply on the matrix cores ----------------------------------------
// C_s <- (I - V_s op(T_s) V_s^T) C_s with v_mfma_f64_16x16x4f64 (D = A B + D,
// A 16 x 4, B 4 x 16).  Lane l = 16 g + j supplies A[j][g] and B[g][j], and
// holds D[g + 4 r][j] in register r.  Workgroup (instance, 64 target
// columns, segment of TS rows); wave w owns 16 of the columns and keeps the
// whole TS x 16 block of C in registers, in the accumulator layout: row
// tile t, register r -> row 16 t + g + 4 r, column j.  The summation index
// of each product runs in the order that makes its B operand a register the
// lane already holds:
//   Z  = V^T C    (i x c):   k-step (t, r) takes row 16 t + g + 4 r, whose
//                            value is C's register r of tile t;
//   Z' = op(T) Z  (i x c):   k-step (it, r) takes i = 16 it + g + 4 r, Z's
//                            register r of tile it;
//   C -= V Z'     (row x c): k-step (mt, r) takes i = 16 mt + g + 4 r, Z''s
//                            register r of tile mt.
// V sits in LDS with row stride VLD = 36 doubles (the update's operand
// pattern, 16 rows by 4 consecutive columns, then touches every bank pair
// exactly twice per wave; the first product's, 4 rows by 16 columns, at most
// four times); op(T) comes straight from global memory (16 values per lane).
typedef double md4 __attribute__((ext_vector_type(4)));
constexpr int VLD = 36;
constexpr int TT = TS / 16;   // row tiles per segment

// rows h0 .. h0 + TS - 1 of a stored reflector block (unit diagonal and
// zeros above it implicit) into Vs, with row stride VLD
__device__ __forceinline__ void stage_v_mf(double (*Vs)[VLD], const double* __restrict__ a0,
                                           int ld, int h0, int rows, int w) {
  const int tid = threadIdx.x;
  for (int b = 0; b < TS * RP; b += 8 * 256) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = b + q * 256 + tid, r = h0 + e / RP, j = e % RP;
      v[q] = (j < w && r < rows && r > j) ? a0[(int64_t)r * ld + j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = b + q * 256 + tid, r = h0 + e / RP, j = e % RP;
      Vs[e / RP][j] = (j < w && r < rows && r == j) ? 1.0 : v[q];
    }
  }
}

template <int TGT>
__global__ void __launch_bounds__(256, 2)
k_leaf_apply_mf(const RedDesc* __restrict__ descs, int panel, const double* __restrict__ W,
                const double* __restrict__ Tleaf, double* __restrict__ C) {
  const RedDesc d = descs[blockIdx.x];
  const int c0 = panel * RP;
  if (c0 >= d.kr) return;
  const int w = min(RP, d.kr - c0), rows_all = d.M - c0, sg = blockIdx.z, r0 = sg * TS;
  if (r0 >= rows_all) return;
  const ApplyTarget a = apply_target<TGT>(d, c0, w, C);
  const int col0 = blockIdx.y * 64;
  if (col0 >= a.ncols) return;
  const int rs = min(TS, rows_all - r0), ws = min(rs, w);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, j = lane & 15, g = lane >> 4;
  const int col = col0 + wave * 16 + j;
  const bool ok = col < a.ncols;
  __shared__ __align__(16) double Vs[TS][VLD];
  // C block into registers (all loads in flight before the first use)
  double* cc = a.cb + (int64_t)r0 * a.ld + col;
  md4 c[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + g + 4 * r;
      c[t][r] = (ok && row < rs) ? cc[(int64_t)row * a.ld] : 0.0;
    }
  stage_v_mf(Vs, W + d.w_off + (int64_t)(c0 + r0) * d.n + c0, d.n, 0, rs, ws);
  __syncthreads();
  // Z = V^T C
  md4 z[2];
#pragma unroll
  for (int it = 0; it < 2; ++it) z[it] = md4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int it = 0; it < 2; ++it)
        z[it] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[16 * t + g + 4 * r][16 * it + j],
                                                     c[t][r], z[it], 0, 0, 0);
  // Z' = op(T) Z, negated for the update; A[m][k] = op(T)[16 mt + j][16 it + g + 4 r]
  const double* Tp = Tleaf + d.leaf_off + ((int64_t)panel * d.nseg0 + sg) * RP * RP;
  md4 zp[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    zp[mt] = md4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int it = 0; it < 2; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = 16 * mt + j, kk = 16 * it + g + 4 * r;
        const double ta = (TGT == TGT_W) ? Tp[kk * RP + ii] : Tp[ii * RP + kk];
        zp[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ta, z[it][r], zp[mt], 0, 0, 0);
      }
  }
  // C -= V Z'
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        c[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[16 * t + j][16 * mt + g + 4 * r],
                                                    zp[mt][r], c[t], 0, 0, 0);
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + g + 4 * r;
      if (ok && row < rs) cc[(int64_t)row * a.ld] = c[t][r];
    }
}

// Tree apply on the matrix cores, with the lane layout and summation orders
// of k_leaf_apply_mf.  Workgroup (instance, 64 target columns): the target
// rows are the segments' first rows (stack row h = 32 s + i is row 256 s + i
// of the panel, i < ws_s), taken TS stack rows at a time, twice: Z = V_t^T C
// over all of them, then C -= V_t Z' with Z' = op(T) Z.
template <int TGT>
__global__ void __launch_bounds__(256, 2)
k_tree_apply_mf(const RedDesc* __restrict__ descs, int panel, const double* __restrict__ Stk,
                const double* __restrict__ T, double* __restrict__ C) {
  const RedDesc d = descs[blockIdx.x];
  const int c0 = panel * RP;
  if (c0 >= d.kr) return;
  const int w = min(RP, d.kr - c0), rows_all = d.M - c0;
  const int nseg = (rows_all + TS - 1) / TS, H = nseg * RP;
  const ApplyTarget a = apply_target<TGT>(d, c0, w, C);
  const int col0 = blockIdx.y * 64;
  if (col0 >= a.ncols) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, j = lane & 15, g = lane >> 4;
  const int col = col0 + wave * 16 + j;
  const bool ok = col < a.ncols;
  const double* v0 = Stk + d.stk_off + (int64_t)panel * d.nseg0 * RP * RP;
  __shared__ __align__(16) double Vs[TS][VLD];
  // target row of stack row h, or -1 (zero rows of a short segment, or past H)
  auto trow = [&](int h) -> int {
    if (h >= H) return -1;
    const int sg = h / RP, i = h - sg * RP;
    const int rs = min(TS, rows_all - sg * TS);
    return i < min(rs, w) ? sg * TS + i : -1;
  };
  md4 z[2];
#pragma unroll
  for (int it = 0; it < 2; ++it) z[it] = md4{0.0, 0.0, 0.0, 0.0};
  for (int h0 = 0; h0 < H; h0 += TS) {
    md4 c[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tr = trow(h0 + 16 * t + g + 4 * r);
        c[t][r] = (ok && tr >= 0) ? a.cb[(int64_t)tr * a.ld + col] : 0.0;
      }
    __syncthreads();
    stage_v_mf(Vs, v0, RP, h0, H, w);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int it = 0; it < 2; ++it)
          z[it] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[16 * t + g + 4 * r][16 * it + j],
                                                       c[t][r], z[it], 0, 0, 0);
  }
  const double* Tp = T + d.t_off + (int64_t)panel * RP * RP;
  md4 zp[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    zp[mt] = md4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int it = 0; it < 2; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = 16 * mt + j, kk = 16 * it + g + 4 * r;
        const double ta = (TGT == TGT_W) ? Tp[kk * RP + ii] : Tp[ii * RP + kk];
        zp[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ta, z[it][r], zp[mt], 0, 0, 0);
      }
  }
  for (int h0 = 0; h0 < H; h0 += TS) {
    md4 c[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tr = trow(h0 + 16 * t + g + 4 * r);
        c[t][r] = (ok && tr >= 0) ? a.cb[(int64_t)tr * a.ld + col] : 0.0;
      }
    __syncthreads();
    stage_v_mf(Vs, v0, RP, h0, H, w);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TT; ++t)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          c[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[16 * t + j][16 * mt + g + 4 * r],
                                                      zp[mt][r], c[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < TT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tr = trow(h0 + 16 * t + g + 4 * r);
        if (ok && tr >= 0) a.cb[(int64_t)tr * a.ld + col] = c[t][r];
      }
  }
}

// Q1 <- [I; 0] (M x Mr per instance)
__global__ void __launch_bounds__(QNT)
k_red_qinit(const RedDesc* __restrict__ descs, double* __restrict__ Q1) {
  const RedDesc d = descs[blockIdx.x];
  const int64_t cnt = (int64_t)d.M * d.Mr;
  for (int64_t e = (int64_t)blockIdx.y * QNT + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.y * QNT) {
    const int64_t t = e / d.Mr;
    Q1[d.q1_off + e] = (t == e - t * d.Mr) ? 1.0 : 0.0;
  }
}

// Reduced regressors Xr[t][c] = R[t][c] (c >= t, t < kr; zero elsewhere).
// With common regressors (sel non-null) column c of the reduced regressors
// is column sel[c] of R (the equation's kept column of Z0).
__global__ void __launch_bounds__(QNT)
k_red_extract(const RedDesc* __restrict__ descs, const double* __restrict__ W,
              const int* __restrict__ ex, const int* __restrict__ sel,
              double* __restrict__ Xr) {
  const RedDesc d = descs[blockIdx.x];
  const int64_t cnt = (int64_t)d.Mr * d.nsub;
  for (int64_t e = threadIdx.x; e < cnt; e += QNT) {
    const int t = (int)(e / d.nsub), cs = (int)(e % d.nsub);
    const int c = sel ? sel[d.sel_off + cs] : cs;
    Xr[d.xr_off + e] = (t < d.kr && c >= t)
                           ? ldexp(W[d.w_off + (int64_t)t * d.n + c], col_exp(ex[d.tau_off + c]))
                           : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Column equilibration of W by powers of two.  Column c of an instance is
// multiplied by 2^-e_c, e_c the binary exponent of its largest magnitude
// (frexp convention).  The scaling is exact and the QR commutes with it: the
// reflectors, T factors and Q1 of the scaled W are those of W, while the rows
// of R come out with column c multiplied by 2^-e_c and are scaled back by
// k_red_extract.  With every column's largest entry in [1/2, 1) the norms of
// the factorization neither overflow nor underflow whatever the scale of the
// data.  Workgroup (instance, EQ_ROWS rows); the exponents are combined with
// integer atomic maxima (order independent) over an array preset to INT_MIN.
// ---------------------------------------------------------------------------
constexpr int EQ_NT = 256;

__global__ void __launch_bounds__(EQ_NT)
k_red_colexp(const RedDesc* __restrict__ descs, const double* __restrict__ X,
             int* __restrict__ ex) {
  const RedDesc d = descs[blockIdx.x];
  const int r0 = blockIdx.y * EQ_ROWS;
  if (r0 >= d.M) return;
  const int r1 = min(d.M, r0 + EQ_ROWS), n = d.n, tid = threadIdx.x;
  __shared__ int sh[NMAX_INST];
  for (int c = tid; c < n; c += EQ_NT) sh[c] = INT_MIN;
  __syncthreads();
  // lane -> (row slot, column): min(n, EQ_NT) columns per pass
  const int cw = n < EQ_NT ? n : EQ_NT, nrs = EQ_NT / cw;
  const int cl = tid % cw, rs = tid / cw;
  const double* __restrict__ x = X + d.w_off;
  if (rs < nrs)
    for (int c = cl; c < n; c += cw) {
      int e = INT_MIN;
      for (int t = r0 + rs; t < r1; t += nrs) {
        const double v = fabs(x[(int64_t)t * n + c]);
        if (v > 0.0 && v <= DBL_MAX) {
          int q;
          (void)frexp(v, &q);
          e = max(e, q);
        }
      }
      if (e != INT_MIN) atomicMax(&sh[c], e);
    }
  __syncthreads();
  for (int c = tid; c < n; c += EQ_NT)
    if (sh[c] != INT_MIN) atomicMax(&ex[d.tau_off + c], sh[c]);
}

__global__ void __launch_bounds__(EQ_NT)
k_red_scale_copy(const RedDesc* __restrict__ descs, const double* __restrict__ X,
                 const int* __restrict__ ex, double* __restrict__ W) {
  const RedDesc d = descs[blockIdx.x];
  const int r0 = blockIdx.y * EQ_ROWS;
  if (r0 >= d.M) return;
  const int r1 = min(d.M, r0 + EQ_ROWS), n = d.n;
  __shared__ int sh[NMAX_INST];
  for (int c = threadIdx.x; c < n; c += EQ_NT) sh[c] = -col_exp(ex[d.tau_off + c]);
  __syncthreads();
  const int64_t base = d.w_off + (int64_t)r0 * n, cnt = (int64_t)(r1 - r0) * n;
  for (int64_t e = threadIdx.x; e < cnt; e += EQ_NT)
    W[base + e] = ldexp(X[base + e], sh[(int)(e % n)]);
}

// ---------------------------------------------------------------------------
// Batched FP64 products with Q1, one 64 x 64 output tile per workgroup
// (tile table entries, XCD-grouped by the host), reduction chunks of 16
// staged through LDS (double-buffered), 4 x 4 outputs per thread.
// ---------------------------------------------------------------------------
constexpr int GT = 64;
constexpr int GKC = 16;

// Y_red = Q1^T Y: output Mr x P (P = G K), reduction over the M rows, on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64, lane l = 16 g + j supplying
// A[j][g] and B[g][j] and holding D[g + 4 r][j]): wave w owns output rows
// 16 w .. 16 w + 15 of the tile and its four 16-column blocks; k-step s of a
// chunk takes rows 4 s + g.  The chunks sit in LDS with row stride GTL = 80
// doubles, so that the four rows of one operand read touch every bank pair
// twice.
constexpr int GTL = GT + 16;

__global__ void __launch_bounds__(256)
k_red_gemm_tn(const RedDesc* __restrict__ descs, const GemmTile* __restrict__ tiles,
              const double* __restrict__ Q1, const double* __restrict__ Y,
              double* __restrict__ Yr) {
  const GemmTile tl = tiles[blockIdx.x];
  if (tl.inst < 0) return;
  const RedDesc d = descs[tl.inst];
  const int M = d.M, Mr = d.Mr, P = d.G * d.K;
  __shared__ __align__(16) double As[2][GKC][GTL];
  __shared__ __align__(16) double Bs[2][GKC][GTL];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, j = lane & 15, g = lane >> 4;
  const double* __restrict__ qb = Q1 + d.q1_off;
  const double* __restrict__ yb = Y + d.v_off;
  double ra[4], rb[4];
  auto load = [&](int t0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, kk = e >> 6, cc = e & 63, t = t0 + kk;
      const int i = tl.i0 + cc, jj = tl.j0 + cc;
      ra[q] = (t < M && i < Mr) ? qb[(int64_t)t * Mr + i] : 0.0;
      rb[q] = (t < M && jj < P) ? yb[(int64_t)t * P + jj] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, kk = e >> 6, cc = e & 63;
      As[buf][kk][cc] = ra[q];
      Bs[buf][kk][cc] = rb[q];
    }
  };
  md4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = md4{0.0, 0.0, 0.0, 0.0};
  const int nk = (M + GKC - 1) / GKC;
  load(0);
  store(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) load((kc + 1) * GKC);
#pragma unroll
    for (int st = 0; st < GKC / 4; ++st) {
      const double a = As[buf][4 * st + g][16 * wave + j];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[buf][4 * st + g][16 * c + j], acc[c],
                                                      0, 0, 0);
    }
    if (kc + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = tl.i0 + 16 * wave + g + 4 * r;
    if (i >= Mr) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int jj = tl.j0 + 16 * c + j;
      if (jj < P) Yr[d.vr_off + (int64_t)i * P + jj] = acc[c][r];
    }
  }
}

// U += Q1 D for the instances with a singular Omega: output M x P,
// reduction over the Mr columns of Q1.
__global__ void __launch_bounds__(256)
k_red_gemm_nn(const RedDesc* __restrict__ descs, const GemmTile* __restrict__ tiles,
              const int* __restrict__ sing, const double* __restrict__ Q1,
              const double* __restrict__ D, double* __restrict__ U) {
  const GemmTile tl = tiles[blockIdx.x];
  if (tl.inst < 0) return;
  const RedDesc d = descs[tl.inst];
  if (!sing[d.inst]) return;
  const int M = d.M, Mr = d.Mr, P = d.G * d.K;
  // A tile stored transposed (k, t), rows padded to keep the strided LDS
  // writes off one bank and the 16-byte reads aligned
  __shared__ __align__(16) double As[2][GKC][GT + 2];
  __shared__ __align__(16) double Bs[2][GKC][GT];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const double* __restrict__ qb = Q1 + d.q1_off;
  const double* __restrict__ db = D + d.vr_off;
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      {
        const int tt = e >> 4, kk = e & 15, t = tl.i0 + tt, k = k0 + kk;
        ra[q] = (t < M && k < Mr) ? qb[(int64_t)t * Mr + k] : 0.0;
      }
      {
        const int kk = e >> 6, cc = e & 63, k = k0 + kk, j = tl.j0 + cc;
        rb[q] = (k < Mr && j < P) ? db[(int64_t)k * P + j] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      As[buf][e & 15][e >> 4] = ra[q];
      Bs[buf][e >> 6][e & 63] = rb[q];
    }
  };
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  const int nk = (Mr + GKC - 1) / GKC;
  load(0);
  store(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) load((kc + 1) * GKC);
#pragma unroll 4
    for (int k = 0; k < GKC; ++k) {
      const double2 a01 = *reinterpret_cast<const double2*>(&As[buf][k][ty * 4]);
      const double2 a23 = *reinterpret_cast<const double2*>(&As[buf][k][ty * 4 + 2]);
      const double2 b01 = *reinterpret_cast<const double2*>(&Bs[buf][k][tx * 4]);
      const double2 b23 = *reinterpret_cast<const double2*>(&Bs[buf][k][tx * 4 + 2]);
      const double av[4] = {a01.x, a01.y, a23.x, a23.y};
      const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
    }
    if (kc + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int t = tl.i0 + ty * 4 + r;
    if (t >= M) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = tl.j0 + tx * 4 + c;
      if (j < P) U[d.v_off + (int64_t)t * P + j] += acc[r][c];
    }
  }
}

// Omega^g, a generalized inverse of the PSD Omega (Omega Omega^g Omega =
// Omega; the inverse when Omega is positive definite), one workgroup per
// instance (A: G x G work area).  sing[b] = 1 when Omega is singular.
__global__ void __launch_bounds__(GINV_NT)
k_red_ginv(const RedDesc* __restrict__ descs, const double* __restrict__ Om,
           double* __restrict__ A, double* __restrict__ Og, int* __restrict__ sing) {
  const RedDesc d = descs[blockIdx.x];
  const int r = psd_ginv(d.G, Om + d.om_off, A + d.om_off, Og + d.om_off);
  if (threadIdx.x == 0) sing[d.inst] = (r < d.G) ? 1 : 0;
}

// U = (Y - [X_i beta_i]) Omega^g.  Workgroup (instance, URC rows), taken in
// sub-chunks of ur rows whose X and Y rows are staged in LDS with coalesced
// loads; Omega^g sits in the same 40 KB of LDS first when G <= 32.  The
// plan guarantees that one row fits the rest (n + G K <= ULDS - G^2 when
// Omega^g is staged, else n + G K <= ULDS).  Y may be null (zero).  The
// blocks' columns come from the reduced problem's block table (the same
// blocks).
constexpr int RTR = 32;
constexpr int URC = 64;
constexpr int ULDS = RED_U_LDS;

// dst[e] = src[e] (src may be null: zeros) for e < count by the workgroup,
// eight loads in flight per thread
__device__ __forceinline__ void stage_rows(double* __restrict__ dst,
                                           const double* __restrict__ src, int count) {
  for (int base = 0; base < count; base += 8 * QNT) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = base + q * QNT + (int)threadIdx.x;
      v[q] = (src && e < count) ? src[e] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = base + q * QNT + (int)threadIdx.x;
      if (e < count) dst[e] = v[q];
    }
  }
}

__global__ void __launch_bounds__(QNT)
k_red_u(const RedDesc* __restrict__ descs, const InstDesc* __restrict__ sinst,
        const BlockDesc* __restrict__ sblk, const int* __restrict__ sel,
        const double* __restrict__ X,
        const double* __restrict__ beta, const double* __restrict__ Y,
        const double* __restrict__ Og, double* __restrict__ U) {
  const RedDesc d = descs[blockIdx.x];
  const int G = d.G, K = d.K, P = G * K, n = d.n, tid = threadIdx.x;
  const int tb = blockIdx.y * URC;
  if (tb >= d.M) return;
  const int te = min(d.M, tb + URC);
  __shared__ double sm[ULDS];
  __shared__ int s_col[256], s_ni[256];
  const BlockDesc* bd = sblk + sinst[d.inst].blk0;
  for (int g = tid; g < G; g += QNT) {
    s_col[g] = bd[g].col;
    s_ni[g] = bd[g].ni;
  }
  const double* og = Og + d.om_off;
  const bool og_lds = G <= 32;
  if (og_lds)
    for (int e = tid; e < G * G; e += QNT) sm[e] = og[e];
  const double* ogp = og_lds ? sm : og;
  const double* bb = beta + d.b_off;
  __syncthreads();   // s_col, s_ni
  // the first BREG coefficients of this thread's first (equation, rhs)
  // pair, which every sub-chunk uses again, stay in registers
  constexpr int BREG = 24;
  double breg[BREG];
  {
    const int g = tid < P ? tid / K : 0, k = tid - g * K;
    const int ni = tid < P ? s_ni[g] : 0;
    const double* br = bb + (int64_t)s_col[g] * K + k;
#pragma unroll
    for (int q = 0; q < BREG; ++q) breg[q] = q < ni ? br[(int64_t)q * K] : 0.0;
  }
  double* Xs = sm + (og_lds ? G * G : 0);
  const int cap = ULDS - (og_lds ? G * G : 0);
  const int ur = max(1, min(8, cap / (n + P)));
  double* Es = Xs + ur * n;
  for (int t0 = tb; t0 < te; t0 += ur) {
    const int nr = min(ur, te - t0);
    __syncthreads();
    stage_rows(Xs, X + d.w_off + (int64_t)t0 * n, nr * n);
    stage_rows(Es, Y ? Y + d.v_off + (int64_t)t0 * P : nullptr, nr * P);
    __syncthreads();
    // fitted values: a thread per (equation g, rhs k) pair over the
    // sub-chunk's rows, the block's beta column eight coefficients at a time
    // (the first pair's first BREG from registers, the rest from memory)
    for (int pq = tid; pq < P; pq += QNT) {
      const int g = pq / K, k = pq - g * K, col = s_col[g], ni = s_ni[g];
      const bool first = pq == tid;
      const double* br = bb + (int64_t)col * K + k;
      const int* xs = sel ? sel + d.sel_off + col : nullptr;   // X column of coefficient c
      double acc[8];
#pragma unroll
      for (int tt = 0; tt < 8; ++tt) acc[tt] = 0.0;
      auto mac = [&](const double (&bv)[8], int c0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (c0 + q >= ni) break;
#pragma unroll
          for (int tt = 0; tt < 8; ++tt)
            if (tt < nr) acc[tt] += Xs[tt * n + (xs ? xs[c0 + q] : col + c0 + q)] * bv[q];
        }
      };
#pragma unroll
      for (int c0 = 0; c0 < BREG; c0 += 8) {
        if (c0 < ni) {
          double bv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q)
            bv[q] = (c0 + q < ni) ? (first ? breg[c0 + q] : br[(int64_t)(c0 + q) * K]) : 0.0;
          mac(bv, c0);
        }
      }
      for (int c0 = BREG; c0 < ni; c0 += 8) {
        double bv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) bv[q] = (c0 + q < ni) ? br[(int64_t)(c0 + q) * K] : 0.0;
        mac(bv, c0);
      }
#pragma unroll
      for (int tt = 0; tt < 8; ++tt)
        if (tt < nr) Es[tt * P + pq] -= acc[tt];
    }
    __syncthreads();
    // u = e Omega^g, four partial sums over the equations
    for (int e = tid; e < nr * P; e += QNT) {
      const int tt = e / P, rem = e - tt * P, i = rem / K, k = rem - i * K;
      const double* er = Es + tt * P + k;
      const double* oc = ogp + i;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int g = 0;
      for (; g + 4 <= G; g += 4) {
        s0 += er[g * K] * oc[g * G];
        s1 += er[(g + 1) * K] * oc[(g + 1) * G];
        s2 += er[(g + 2) * K] * oc[(g + 2) * G];
        s3 += er[(g + 3) * K] * oc[(g + 3) * G];
      }
      for (; g < G; ++g) s0 += er[g * K] * oc[g * G];
      U[d.v_off + (int64_t)t0 * P + e] = (s0 + s1) + (s2 + s3);
    }
  }
}

// D = U_red - (U_red Omega) Omega^g on the Mr reduced rows (singular Omega only)
__global__ void __launch_bounds__(QNT)
k_red_delta(const RedDesc* __restrict__ descs, const int* __restrict__ sing,
            const double* __restrict__ Om, const double* __restrict__ Og,
            const double* __restrict__ Ur, double* __restrict__ D) {
  const RedDesc d = descs[blockIdx.x];
  if (!sing[d.inst]) return;
  const int G = d.G, K = d.K, P = G * K, tid = threadIdx.x;
  const int rows = max(1, min(RTR, 4096 / P));
  const int t0 = blockIdx.y * rows;
  if (t0 >= d.Mr) return;
  const int t1 = min(d.Mr, t0 + rows);
  __shared__ double Ws[4096];
  const double* om = Om + d.om_off;
  const double* og = Og + d.om_off;
  for (int e = tid; e < (t1 - t0) * P; e += QNT) {
    const int tt = e / P, rem = e - tt * P, i = rem / K, k = rem - i * K;
    const double* ur = Ur + d.vr_off + (int64_t)(t0 + tt) * P + k;
    double s = 0.0;
    for (int h = 0; h < G; ++h) s += ur[h * K] * om[h * G + i];
    Ws[e] = s;
  }
  __syncthreads();
  for (int e = tid; e < (t1 - t0) * P; e += QNT) {
    const int tt = e / P, rem = e - tt * P, i = rem / K, k = rem - i * K;
    const double* wr = Ws + tt * P + k;
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += wr[g * K] * og[g * G + i];
    const int64_t at = d.vr_off + (int64_t)(t0 + tt) * P + rem;
    D[at] = Ur[at] - s;
  }
}

// Reverse mode on a reduced handle, full model:
//   S_seg[i][j] = sum_{t in segment, k} L[t][i][k] U[t][j][k]  (partials),
//   dOmega = -sym(sum_seg S_seg),
//   dX[t][c] = -sum_k (L[t][i(c)][k] beta[c][k] + U[t][i(c)][k] lb[c][k]).
__global__ void __launch_bounds__(QNT)
k_red_grad_omega_part(const RedDesc* __restrict__ descs, const double* __restrict__ L,
                      const double* __restrict__ U, double* __restrict__ part) {
  const RedDesc d = descs[blockIdx.x];
  const int t0 = blockIdx.y * RED_SEG;
  if (t0 >= d.M) return;
  const int t1 = min(d.M, t0 + RED_SEG), G = d.G, K = d.K, P = G * K;
  for (int pr = threadIdx.x; pr < G * G; pr += QNT) {
    const int i = pr / G, j = pr % G;
    double s = 0.0;
    for (int t = t0; t < t1; ++t) {
      const double* lr = L + d.v_off + (int64_t)t * P + i * K;
      const double* ur = U + d.v_off + (int64_t)t * P + j * K;
      for (int k = 0; k < K; ++k) s += lr[k] * ur[k];
    }
    part[d.zp_off + (int64_t)blockIdx.y * G * G + pr] = s;
  }
}

__global__ void __launch_bounds__(QNT)
k_red_grad_omega_reduce(const RedDesc* __restrict__ descs, const double* __restrict__ part,
                        double* __restrict__ dOm) {
  const RedDesc d = descs[blockIdx.x];
  const int G = d.G, nseg = (d.M + RED_SEG - 1) / RED_SEG;
  for (int pr = threadIdx.x; pr < G * G; pr += QNT) {
    const int i = pr / G, j = pr % G;
    double sij = 0.0, sji = 0.0;
    for (int sg = 0; sg < nseg; ++sg) {
      sij += part[d.zp_off + (int64_t)sg * G * G + i * G + j];
      sji += part[d.zp_off + (int64_t)sg * G * G + j * G + i];
    }
    dOm[d.om_off + pr] = -0.5 * (sij + sji);
  }
}

__global__ void __launch_bounds__(QNT)
k_red_grad_x(const RedDesc* __restrict__ descs, const InstDesc* __restrict__ sinst,
             const int* __restrict__ colblk, const double* __restrict__ L,
             const double* __restrict__ U, const double* __restrict__ beta,
             const double* __restrict__ lb, double* __restrict__ dX) {
  const RedDesc d = descs[blockIdx.x];
  const int t0 = blockIdx.y * RTR;
  if (t0 >= d.M) return;
  const int t1 = min(d.M, t0 + RTR), G = d.G, K = d.K, n = d.n;
  const int* cb = colblk + sinst[d.inst].col_off;
  for (int e = threadIdx.x; e < (t1 - t0) * n; e += QNT) {
    const int t = t0 + e / n, c = e % n, i = cb[c];
    const int64_t vr = d.v_off + ((int64_t)t * G + i) * K;
    const int64_t br = d.b_off + (int64_t)c * K;
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += L[vr + k] * beta[br + k] + U[vr + k] * lb[br + k];
    dX[d.w_off + (int64_t)t * n + c] = -s;
  }
}

}  // namespace

hipError_t launch_red_panel(const RedDesc* d, int B, int panel, int maxseg, int maxcols,
                           double* W, double* Tleaf, double* Stk, double* tau, double* T,
                           hipStream_t s) {
  if (B <= 0 || maxseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tsqr_leaf, dim3(B, maxseg), dim3(256), 0, s, d, panel, W, Tleaf, Stk);
  if (hipError_t e = hipGetLastError()) return e;
  if (maxcols > 0)
    hipLaunchKernelGGL(k_leaf_apply_mf<TGT_W>, dim3(B, (maxcols + 63) / 64, maxseg), dim3(256), 0,
                       s, d, panel, (const double*)W, (const double*)Tleaf, W);
  if (hipError_t e = hipGetLastError()) return e;
  // the stack of every instance (maxseg x 32 rows at most) in registers when
  // it fits, else swept through memory
  if (maxseg <= 8)
    hipLaunchKernelGGL(k_tsqr_tree_reg<8>, dim3(B), dim3(RPNT), 0, s, d, panel, W, Stk, tau, T);
  else if (maxseg <= 16)
    hipLaunchKernelGGL(k_tsqr_tree_reg<16>, dim3(B), dim3(RPNT), 0, s, d, panel, W, Stk, tau, T);
  else if (maxseg <= 24)
    hipLaunchKernelGGL(k_tsqr_tree_reg<24>, dim3(B), dim3(RPNT), 0, s, d, panel, W, Stk, tau, T);
  else
    hipLaunchKernelGGL(k_tsqr_tree, dim3(B), dim3(RPNT), 0, s, d, panel, W, Stk, tau, T);
  if (hipError_t e = hipGetLastError()) return e;
  if (maxcols > 0)
    hipLaunchKernelGGL(k_tree_apply_mf<TGT_W>, dim3(B, (maxcols + 63) / 64), dim3(256), 0, s, d,
                       panel, (const double*)Stk, (const double*)T, W);
  return hipGetLastError();
}

hipError_t launch_red_q1_panel(const RedDesc* d, int B, int panel, int maxseg, int maxcols,
                              const double* W, const double* Tleaf, const double* Stk,
                              const double* T, double* Q1, hipStream_t s) {
  if (B <= 0 || maxseg <= 0 || maxcols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tree_apply_mf<TGT_Q1>, dim3(B, (maxcols + 63) / 64), dim3(256), 0, s, d,
                     panel, Stk, T, Q1);
  if (hipError_t e = hipGetLastError()) return e;
  hipLaunchKernelGGL(k_leaf_apply_mf<TGT_Q1>, dim3(B, (maxcols + 63) / 64, maxseg), dim3(256), 0,
                     s, d, panel, W, Tleaf, Q1);
  return hipGetLastError();
}

hipError_t launch_red_qinit(const RedDesc* d, int B, double* Q1, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_qinit, dim3(B, 64), dim3(QNT), 0, s, d, Q1);
  return hipGetLastError();
}

hipError_t launch_red_extract(const RedDesc* d, int B, const double* W, const int* ex,
                             const int* sel, double* Xr, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_extract, dim3(B), dim3(QNT), 0, s, d, W, ex, sel, Xr);
  return hipGetLastError();
}

// W = X with its columns equilibrated; ex (sum of n ints) receives the
// exponents and must hold INT_MIN on entry
hipError_t launch_red_equilibrate(const RedDesc* d, int B, int maxM, const double* X, int* ex,
                                  double* W, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  const dim3 grid(B, (maxM + EQ_ROWS - 1) / EQ_ROWS);
  hipLaunchKernelGGL(k_red_colexp, grid, dim3(EQ_NT), 0, s, d, X, ex);
  hipLaunchKernelGGL(k_red_scale_copy, grid, dim3(EQ_NT), 0, s, d, X, ex, W);
  return hipGetLastError();
}

hipError_t launch_red_gemm_tn(const RedDesc* d, const GemmTile* tiles, int ntiles,
                             const double* Q1, const double* Y, double* Yr, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_gemm_tn, dim3(ntiles), dim3(256), 0, s, d, tiles, Q1, Y, Yr);
  return hipGetLastError();
}

hipError_t launch_red_ginv(const RedDesc* d, int B, const double* Om, double* A, double* Og,
                          int* sing, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_ginv, dim3(B), dim3(GINV_NT), 0, s, d, Om, A, Og, sing);
  return hipGetLastError();
}

hipError_t launch_red_u(const RedDesc* d, int B, int maxM, const InstDesc* sinst,
                       const BlockDesc* sblk, const int* sel, const double* X,
                       const double* beta, const double* Y, const double* Og, double* U,
                       hipStream_t s) {
  if (B <= 0 || maxM <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_u, dim3(B, (maxM + URC - 1) / URC), dim3(QNT), 0, s, d, sinst, sblk,
                     sel, X, beta, Y, Og, U);
  return hipGetLastError();
}

hipError_t launch_red_singular(const RedDesc* d, int B, int chunks, const GemmTile* tiles2,
                              int ntiles2, const int* sing, const double* Om, const double* Og,
                              const double* Q1, const double* Ur, double* D, double* U,
                              hipStream_t s) {
  if (B <= 0 || chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_delta, dim3(B, chunks), dim3(QNT), 0, s, d, sing, Om, Og, Ur, D);
  if (hipError_t e = hipGetLastError()) return e;
  if (ntiles2 > 0)
    hipLaunchKernelGGL(k_red_gemm_nn, dim3(ntiles2), dim3(256), 0, s, d, tiles2, sing, Q1,
                       (const double*)D, U);
  return hipGetLastError();
}

hipError_t launch_red_grad(const RedDesc* d, int B, int maxM, const InstDesc* sinst,
                          const int* colblk, const double* L, const double* U,
                          const double* beta, const double* lb, double* part, double* dOm,
                          double* dX, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (dOm) {
    hipLaunchKernelGGL(k_red_grad_omega_part, dim3(B, (maxM + RED_SEG - 1) / RED_SEG),
                       dim3(QNT), 0, s, d, L, U, part);
    hipLaunchKernelGGL(k_red_grad_omega_reduce, dim3(B), dim3(QNT), 0, s, d,
                       (const double*)part, dOm);
  }
  if (dX)
    hipLaunchKernelGGL(k_red_grad_x, dim3(B, (maxM + RTR - 1) / RTR), dim3(QNT), 0, s, d,
                       sinst, colblk, L, U, beta, lb, dX);
  return hipGetLastError();
}

}  // namespace glm
