// SUR model reduction (the remark on reducing the SUR model in the SUR
// section): one Householder QR of W = [X_1 ... X_G] = Q [R; 0] per instance.
// Rotating every equation by Q^T keeps Sigma = Omega (x) I_M, and the rotated
// rows t >= n carry no information on beta, so the GLS of the first
// Mr = min(M, n + 1) rotated rows is the GLS of the full model.
//
// Factorization (once per W): Householder panels of RED_PANEL columns in
// compact WY form, B_p = I - V_p T_p V_p^T (T_p upper triangular), applied to
// the trailing columns of W; then the explicit first Mr columns of
// Q = B_0 B_1 ..., Q1 = Q [I; 0] (M x Mr), accumulated backwards.
//   k_red_panel       factor panel p in place, store tau and T_p
//   k_red_apply_z/_c  C <- B_p^T C (trailing columns of W) or C <- B_p C (Q1)
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
#include "qr_panel.h"

#include <cmath>

namespace glm {

namespace {

constexpr int RP = RED_PANEL;
constexpr int RCH = 128;  // rows of V staged in LDS per chunk

// V[r][j] of panel rows r (relative to the panel's first row): the unit
// diagonal and zeros above it are implicit in the stored factorization.
__device__ __forceinline__ double vpanel(const double* __restrict__ a0, int ld, int r, int j,
                                         int rows, int w) {
  if (j >= w || r >= rows) return 0.0;
  if (r == j) return 1.0;
  return r > j ? a0[(int64_t)r * ld + j] : 0.0;
}

// The panel kernel runs RPNT threads per instance: the panel passes are
// sequential over the rows, so the rows in flight per instance set its time.
constexpr int RPNT = 1024;
constexpr int RPU = 16;             // rows in flight per lane in the panel passes
constexpr int RPW = RPNT / 64;      // waves per panel workgroup

__global__ void __launch_bounds__(RPNT)
k_red_panel(const RedDesc* __restrict__ descs, int panel, double* __restrict__ W,
            double* __restrict__ tau, double* __restrict__ T) {
  const RedDesc d = descs[blockIdx.x];
  const int c0 = panel * RP;
  if (c0 >= d.kr) return;
  const int w = min(RP, d.kr - c0), rows = d.M - c0, ld = d.n;
  double* a0 = W + d.w_off + (int64_t)c0 * ld + c0;
  __shared__ Qr32Shared<RPNT> sh;
  __shared__ double S[RP][RP + 1];
  __shared__ double part[4][RP][RP];
  qr32_factor<RPNT, RPU>(a0, rows, w, ld, sh);
  const int tid = threadIdx.x, c = tid & 31, slot = tid >> 5;
  if (tid < w) tau[d.tau_off + c0 + tid] = sh.tau_s[tid];
  // S = V^T V: lane c accumulates S[i][c] for every i over its rows
  double acc[RP];
#pragma unroll
  for (int i = 0; i < RP; ++i) acc[i] = 0.0;
  // rows r0 + slot + (RPNT / 32) q: the same half-wave that factored them
  constexpr int SU = 4;
  for (int r0 = 0; r0 < rows; r0 += (RPNT / 32) * SU) {
    double v[SU];
#pragma unroll
    for (int q = 0; q < SU; ++q) v[q] = vpanel(a0, ld, r0 + slot + (RPNT / 32) * q, c, rows, w);
#pragma unroll
    for (int q = 0; q < SU; ++q)
#pragma unroll
      for (int i = 0; i < RP; ++i) acc[i] += shfl_col(v[q], i) * v[q];
  }
#pragma unroll
  for (int i = 0; i < RP; ++i) acc[i] += __shfl_xor(acc[i], 32, 64);
  // wave partials summed in four slots, four waves at a time in wave order
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
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) s += part[q][i][j];
    S[i][j] = s;
  }
  __syncthreads();
  // T (forward, columnwise): T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] S[0:j, j];
  // built in LDS (the partial sums are no longer needed) by one thread
  double (*Tl)[RP] = part[0];
  for (int e = tid; e < RP * RP; e += RPNT) Tl[e / RP][e % RP] = 0.0;
  __syncthreads();
  if (tid == 0)
    for (int j = 0; j < w; ++j) {
      const double tj = sh.tau_s[j];
      for (int i = 0; i < j; ++i) {
        double s = 0.0;
        for (int k = i; k < j; ++k) s += Tl[i][k] * S[k][j];
        Tl[i][j] = -tj * s;
      }
      Tl[j][j] = tj;
    }
  __syncthreads();
  double* Tp = T + d.t_off + (int64_t)panel * RP * RP;
  for (int e = tid; e < RP * RP; e += RPNT) Tp[e] = Tl[e / RP][e % RP];
}

// C <- (I - V op(T) V^T) C on rows [c0, M) of one instance, op(T) = T^T when
// trans (B_p^T) else T (B_p).  Target: the trailing columns of W (TGT_W) or
// the columns c0.. of Q1 (TGT_Q1).  The rows are cut into segments of
// RED_SEG, so that a tall instance spreads over as many workgroups as a short
// one has rows to spare; workgroup (instance, chunk of QNT columns, segment),
// lane per column:
//   k_red_apply_z   partial z_s = V_s^T c_s of the segment
//   k_red_apply_c   z = sum of the partials (fixed order), z' = op(T) z,
//                   c_s -= V_s z'
// V is staged in LDS RCH rows at a time, unpadded: every lane reads the same
// V entry (a broadcast), so rows 16-byte aligned give two entries per read;
// RU rows of c are loaded before they are used.
constexpr int RU = 32;
static_assert(RED_SEG % RCH == 0 && RCH % RU == 0, "segment, chunk and batch sizes nest");
enum : int { TGT_W = 1, TGT_Q1 = 2 };

struct ApplyTarget {
  const double* a0;  // panel block of the reflectors (row c0, column c0)
  double* cb;        // row c0 of the target
  int w, rows, ncols, ld, seg_rows, r_seg;
};

// the apply's target for this workgroup, or false when it has nothing to do
template <int TGT>
__device__ __forceinline__ bool apply_target(const RedDesc& d, int panel, const double* W,
                                             double* C, ApplyTarget& a) {
  const int c0 = panel * RP;
  if (c0 >= d.kr) return false;
  a.w = min(RP, d.kr - c0);
  a.rows = d.M - c0;
  a.a0 = W + d.w_off + (int64_t)c0 * d.n + c0;
  if (TGT == TGT_W) {
    a.ncols = d.n - c0 - a.w;
    a.ld = d.n;
    a.cb = C + d.w_off + (int64_t)c0 * d.n + c0 + a.w;
  } else {
    a.ncols = d.Mr - c0;
    a.ld = d.Mr;
    a.cb = C + d.q1_off + (int64_t)c0 * d.Mr + c0;
  }
  if ((int)blockIdx.y * QNT >= a.ncols) return false;
  a.r_seg = blockIdx.z * RED_SEG;
  if (a.r_seg >= a.rows) return false;
  a.seg_rows = min(RED_SEG, a.rows - a.r_seg);
  return true;
}

__device__ __forceinline__ void stage_v(double (*Vs)[RP], const ApplyTarget& a, int ldw,
                                        int r0) {
  for (int e = threadIdx.x; e < RCH * RP; e += QNT) {
    const int r = e / RP, j = e % RP;
    Vs[r][j] = vpanel(a.a0, ldw, r0 + r, j, a.rows, a.w);
  }
}

template <int TGT>
__global__ void __launch_bounds__(QNT)
k_red_apply_z(const RedDesc* __restrict__ descs, int panel, const double* __restrict__ W,
              double* __restrict__ C, double* __restrict__ Zp) {
  const RedDesc d = descs[blockIdx.x];
  ApplyTarget a;
  if (!apply_target<TGT>(d, panel, W, C, a)) return;
  __shared__ __align__(16) double Vs[RCH][RP];
  const int col = blockIdx.y * QNT + threadIdx.x;
  const bool ok = col < a.ncols;
  const double* cc = a.cb + col;
  double z[RP];
#pragma unroll
  for (int j = 0; j < RP; ++j) z[j] = 0.0;
  for (int r0 = a.r_seg; r0 < a.r_seg + a.seg_rows; r0 += RCH) {
    __syncthreads();
    stage_v(Vs, a, d.n, r0);
    __syncthreads();
    const int nr = min(RCH, a.r_seg + a.seg_rows - r0);
    for (int r = 0; r < nr; r += RU) {
      double x[RU];
#pragma unroll
      for (int q = 0; q < RU; ++q)
        x[q] = (ok && r + q < nr) ? cc[(int64_t)(r0 + r + q) * a.ld] : 0.0;
#pragma unroll
      for (int q = 0; q < RU; ++q)
#pragma unroll
        for (int j = 0; j < RP; ++j) z[j] += Vs[r + q][j] * x[q];
    }
  }
  if (ok) {
    double* zp = Zp + d.zp_off + (int64_t)blockIdx.z * RP * a.ncols + col;
#pragma unroll
    for (int j = 0; j < RP; ++j) zp[(int64_t)j * a.ncols] = z[j];
  }
}

template <int TGT>
__global__ void __launch_bounds__(QNT)
k_red_apply_c(const RedDesc* __restrict__ descs, int panel, const double* __restrict__ W,
              const double* __restrict__ T, double* __restrict__ C,
              const double* __restrict__ Zp, int trans) {
  const RedDesc d = descs[blockIdx.x];
  ApplyTarget a;
  if (!apply_target<TGT>(d, panel, W, C, a)) return;
  __shared__ double Ts[RP][RP + 1];
  __shared__ __align__(16) double Vs[RCH][RP];
  const int tid = threadIdx.x;
  {
    const double* Tp = T + d.t_off + (int64_t)panel * RP * RP;
    for (int e = tid; e < RP * RP; e += QNT) {
      const int i = e / RP, j = e % RP;
      Ts[i][j] = trans ? Tp[j * RP + i] : Tp[i * RP + j];
    }
  }
  const int col = blockIdx.y * QNT + tid;
  const bool ok = col < a.ncols;
  double* cc = a.cb + col;
  double z[RP];
#pragma unroll
  for (int j = 0; j < RP; ++j) z[j] = 0.0;
  if (ok) {
    const int nseg = (a.rows + RED_SEG - 1) / RED_SEG;
    const double* zp = Zp + d.zp_off + col;
    for (int s = 0; s < nseg; ++s)
#pragma unroll
      for (int j = 0; j < RP; ++j) z[j] += zp[((int64_t)s * RP + j) * a.ncols];
  }
  __syncthreads();  // Ts
  double zz[RP];
#pragma unroll
  for (int i = 0; i < RP; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < RP; ++j) s += Ts[i][j] * z[j];
    zz[i] = s;
  }
  for (int r0 = a.r_seg; r0 < a.r_seg + a.seg_rows; r0 += RCH) {
    __syncthreads();
    stage_v(Vs, a, d.n, r0);
    __syncthreads();
    const int nr = min(RCH, a.r_seg + a.seg_rows - r0);
    if (ok)
      for (int r = 0; r < nr; r += RU) {
        double x[RU];
#pragma unroll
        for (int q = 0; q < RU; ++q)
          x[q] = (r + q < nr) ? cc[(int64_t)(r0 + r + q) * a.ld] : 0.0;
#pragma unroll
        for (int q = 0; q < RU; ++q) {
          double v = x[q];
#pragma unroll
          for (int j = 0; j < RP; ++j) v -= Vs[r + q][j] * zz[j];
          if (r + q < nr) cc[(int64_t)(r0 + r + q) * a.ld] = v;
        }
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
__global__ void __launch_bounds__(QNT)
k_red_extract(const RedDesc* __restrict__ descs, const double* __restrict__ W,
              double* __restrict__ Xr) {
  const RedDesc d = descs[blockIdx.x];
  const int64_t cnt = (int64_t)d.Mr * d.n;
  for (int64_t e = threadIdx.x; e < cnt; e += QNT) {
    const int t = (int)(e / d.n), c = (int)(e % d.n);
    Xr[d.xr_off + e] = (t < d.kr && c >= t) ? W[d.w_off + e] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Batched FP64 products with Q1, one 64 x 64 output tile per workgroup
// (tile table entries, XCD-grouped by the host), reduction chunks of 16
// staged through LDS (double-buffered), 4 x 4 outputs per thread.
// ---------------------------------------------------------------------------
constexpr int GT = 64;
constexpr int GKC = 16;

// Y_red = Q1^T Y: output Mr x P (P = G K), reduction over the M rows.
__global__ void __launch_bounds__(256)
k_red_gemm_tn(const RedDesc* __restrict__ descs, const GemmTile* __restrict__ tiles,
              const double* __restrict__ Q1, const double* __restrict__ Y,
              double* __restrict__ Yr) {
  const GemmTile tl = tiles[blockIdx.x];
  if (tl.inst < 0) return;
  const RedDesc d = descs[tl.inst];
  const int M = d.M, Mr = d.Mr, P = d.G * d.K;
  __shared__ __align__(16) double As[2][GKC][GT];
  __shared__ __align__(16) double Bs[2][GKC][GT];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const double* __restrict__ qb = Q1 + d.q1_off;
  const double* __restrict__ yb = Y + d.v_off;
  double ra[4], rb[4];
  auto load = [&](int t0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, kk = e >> 6, cc = e & 63, t = t0 + kk;
      const int i = tl.i0 + cc, j = tl.j0 + cc;
      ra[q] = (t < M && i < Mr) ? qb[(int64_t)t * Mr + i] : 0.0;
      rb[q] = (t < M && j < P) ? yb[(int64_t)t * P + j] : 0.0;
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
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  const int nk = (M + GKC - 1) / GKC;
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
    const int i = tl.i0 + ty * 4 + r;
    if (i >= Mr) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = tl.j0 + tx * 4 + c;
      if (j < P) Yr[d.vr_off + (int64_t)i * P + j] = acc[r][c];
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

// ---------------------------------------------------------------------------
// Omega^g: a generalized inverse of the PSD Omega (Omega Omega^g Omega = Omega)
// by Cholesky with diagonal pivoting, stopped when the largest remaining
// diagonal is at most 16 G eps trace(Omega) (the rank r); with L the r x r
// factor and Pm the pivoting, Omega^g = Pm [L^-T L^-1, 0; 0, 0] Pm^T, the
// inverse when r = G.  One workgroup per instance, in global memory
// (A: G x G work area).  sing[b] = 1 when r < G.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_red_ginv(const RedDesc* __restrict__ descs, const double* __restrict__ Om,
           double* __restrict__ A, double* __restrict__ Og, int* __restrict__ sing) {
  const RedDesc d = descs[blockIdx.x];
  const int G = d.G, tid = threadIdx.x;
  double* a = A + d.om_off;
  const double* o = Om + d.om_off;
  double* og = Og + d.om_off;
  __shared__ int perm[256];
  __shared__ double dinv[256];
  __shared__ double s_piv, s_tol;
  __shared__ int s_j;
  for (int e = tid; e < G * G; e += 256) a[e] = o[e];
  for (int i = tid; i < G; i += 256) perm[i] = i;
  if (tid < 64) {
    double tr = 0.0;
    for (int i = tid; i < G; i += 64) tr += fabs(o[(int64_t)i * G + i]);
    tr = wave_sum(tr);
    if (tid == 0) s_tol = 16.0 * G * 2.220446049250313e-16 * tr;
  }
  __syncthreads();
  int r = G;
  for (int k = 0; k < G; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bj = k;
      for (int j = k + tid; j < G; j += 64) {
        const double v = a[(int64_t)j * G + j];
        if (v > best) {
          best = v;
          bj = j;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oj = __shfl_xor(bj, off, 64);
        if (ob > best || (ob == best && oj < bj)) {
          best = ob;
          bj = oj;
        }
      }
      if (tid == 0) {
        s_piv = best;
        s_j = bj;
      }
    }
    __syncthreads();
    if (!(s_piv > s_tol)) {
      r = k;
      break;
    }
    const int j = s_j;
    if (j != k) {
      for (int c = tid; c < G; c += 256) {
        const double t0 = a[(int64_t)k * G + c];
        a[(int64_t)k * G + c] = a[(int64_t)j * G + c];
        a[(int64_t)j * G + c] = t0;
      }
      __syncthreads();
      for (int rr = k + tid; rr < G; rr += 256) {
        const double t0 = a[(int64_t)rr * G + k];
        a[(int64_t)rr * G + k] = a[(int64_t)rr * G + j];
        a[(int64_t)rr * G + j] = t0;
      }
      if (tid == 0) {
        const int pk = perm[k];
        perm[k] = perm[j];
        perm[j] = pk;
      }
      __syncthreads();
    }
    const double lkk = sqrt(a[(int64_t)k * G + k]);
    __syncthreads();
    for (int i = k + 1 + tid; i < G; i += 256) a[(int64_t)i * G + k] /= lkk;
    if (tid == 0) {
      a[(int64_t)k * G + k] = lkk;
      dinv[k] = 1.0 / lkk;
    }
    __syncthreads();
    const int w = G - k - 1;
    for (int e = tid; e < w * w; e += 256) {
      const int i = k + 1 + e / w, c = k + 1 + e % w;
      a[(int64_t)i * G + c] -= a[(int64_t)i * G + k] * a[(int64_t)c * G + k];
    }
    __syncthreads();
  }
  // column c of L^-1 (rows i > c) into the upper triangle: a[c][i] = (L^-1)[i][c]
  for (int c = tid; c < r; c += 256) {
    for (int i = c + 1; i < r; ++i) {
      double s = a[(int64_t)i * G + c] * dinv[c];
      for (int kk = c + 1; kk < i; ++kk) s += a[(int64_t)i * G + kk] * a[(int64_t)c * G + kk];
      a[(int64_t)c * G + i] = -s * dinv[i];
    }
  }
  __syncthreads();
  for (int e = tid; e < G * G; e += 256) {
    const int p = e / G, q = e % G;
    double s = 0.0;
    if (p < r && q < r) {
      const int lo = p > q ? p : q;
      for (int kk = lo; kk < r; ++kk) {
        const double lp = (kk == p) ? dinv[p] : a[(int64_t)p * G + kk];
        const double lq = (kk == q) ? dinv[q] : a[(int64_t)q * G + kk];
        s += lp * lq;
      }
    }
    og[(int64_t)perm[p] * G + perm[q]] = s;
  }
  if (tid == 0) sing[d.inst] = (r < G) ? 1 : 0;
}

// U = (Y - [X_i beta_i]) Omega^g.  Workgroup (instance, URC rows), taken in
// sub-chunks of ur rows whose X and Y rows are staged in LDS with coalesced
// loads; Omega^g sits in the same 64 KB of LDS first when G <= 64.  The
// shape limits keep one row within the rest: G <= 64 has G K <= 1024 and
// n <= 2048; G > 64 has n + G K <= 1024 + 4096.  Y may be null (zero).  The
// blocks' columns come from the reduced problem's block table (the same
// blocks).
constexpr int RTR = 32;
constexpr int URC = 64;
constexpr int ULDS = 8192;     // doubles of LDS: Omega^g (G <= 64), then X and Y rows

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
        const BlockDesc* __restrict__ sblk, const double* __restrict__ X,
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
  const bool og_lds = G <= 64;
  if (og_lds)
    for (int e = tid; e < G * G; e += QNT) sm[e] = og[e];
  const double* ogp = og_lds ? sm : og;
  const double* bb = beta + d.b_off;
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
    // sub-chunk's rows, the block's beta column eight loads at a time
    for (int pq = tid; pq < P; pq += QNT) {
      const int g = pq / K, k = pq - g * K, col = s_col[g], ni = s_ni[g];
      const double* br = bb + (int64_t)col * K + k;
      double acc[8];
#pragma unroll
      for (int tt = 0; tt < 8; ++tt) acc[tt] = 0.0;
      for (int c0 = 0; c0 < ni; c0 += 8) {
        double bv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) bv[q] = (c0 + q < ni) ? br[(int64_t)(c0 + q) * K] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (c0 + q >= ni) break;
#pragma unroll
          for (int tt = 0; tt < 8; ++tt)
            if (tt < nr) acc[tt] += Xs[tt * n + col + c0 + q] * bv[q];
        }
      }
#pragma unroll
      for (int tt = 0; tt < 8; ++tt)
        if (tt < nr) Es[tt * P + pq] -= acc[tt];
    }
    __syncthreads();
    for (int e = tid; e < nr * P; e += QNT) {
      const int tt = e / P, rem = e - tt * P, i = rem / K, k = rem - i * K;
      const double* er = Es + tt * P + k;
      double s = 0.0;
      for (int g = 0; g < G; ++g) s += er[g * K] * ogp[g * G + i];
      U[d.v_off + (int64_t)t0 * P + e] = s;
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

hipError_t launch_red_panel(const RedDesc* d, int B, int panel, double* W, double* tau,
                           double* T, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_panel, dim3(B), dim3(RPNT), 0, s, d, panel, W, tau, T);
  return hipGetLastError();
}

hipError_t launch_red_apply(const RedDesc* d, int B, int panel, const double* W,
                           const double* T, double* C, double* Zp, int target_q1, int trans,
                           int maxcols, int maxrows, hipStream_t s) {
  if (B <= 0 || maxcols <= 0 || maxrows <= 0) return hipSuccess;
  const dim3 grid(B, (maxcols + QNT - 1) / QNT, (maxrows + RED_SEG - 1) / RED_SEG);
  if (target_q1)
    hipLaunchKernelGGL(k_red_apply_z<TGT_Q1>, grid, dim3(QNT), 0, s, d, panel, W, C, Zp);
  else
    hipLaunchKernelGGL(k_red_apply_z<TGT_W>, grid, dim3(QNT), 0, s, d, panel, W, C, Zp);
  if (hipError_t e = hipGetLastError()) return e;
  if (target_q1)
    hipLaunchKernelGGL(k_red_apply_c<TGT_Q1>, grid, dim3(QNT), 0, s, d, panel, W, T, C,
                       (const double*)Zp, trans);
  else
    hipLaunchKernelGGL(k_red_apply_c<TGT_W>, grid, dim3(QNT), 0, s, d, panel, W, T, C,
                       (const double*)Zp, trans);
  return hipGetLastError();
}

hipError_t launch_red_qinit(const RedDesc* d, int B, double* Q1, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_qinit, dim3(B, 64), dim3(QNT), 0, s, d, Q1);
  return hipGetLastError();
}

hipError_t launch_red_extract(const RedDesc* d, int B, const double* W, double* Xr,
                             hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_extract, dim3(B), dim3(QNT), 0, s, d, W, Xr);
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
  hipLaunchKernelGGL(k_red_ginv, dim3(B), dim3(256), 0, s, d, Om, A, Og, sing);
  return hipGetLastError();
}

hipError_t launch_red_u(const RedDesc* d, int B, int maxM, const InstDesc* sinst,
                       const BlockDesc* sblk, const double* X, const double* beta,
                       const double* Y, const double* Og, double* U, hipStream_t s) {
  if (B <= 0 || maxM <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_u, dim3(B, (maxM + URC - 1) / URC), dim3(QNT), 0, s, d, sinst, sblk,
                     X, beta, Y, Og, U);
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
