// SUR model reduction (the remark on reducing the SUR model in the SUR
// section): one Householder QR of W = [X_1 ... X_G] = Q [R; 0] per instance.
// Rotating every equation by Q^T keeps Sigma = Omega (x) I_M, and the rotated
// rows t >= n carry no information on beta, so the GLS of the first
// Mr = min(M, n + 1) rotated rows is the GLS of the full model.  The full
// residual-like vector is U = Q [U_red ; (Q^T Y)_{t >= Mr} Omega^-1].
//
// Q is kept as Householder panels of RED_PANEL columns in compact WY form,
// Q = B_0 B_1 ... with B_p = I - V_p T_p V_p^T (T_p upper triangular):
//   k_red_panel    factor panel p in place (reflectors below the diagonal),
//                  store tau and T_p
//   k_red_apply_z/_c  C <- B_p^T C (the trailing columns of W while factoring,
//                  and Y for Q^T Y) or C <- B_p C (Q Z for the residual)
//   k_red_extract  reduced regressors (R rows) and reduced responses
//   k_red_oinv     Omega^-1 per instance
//   k_red_tail     U rows: the reduced solve's rows, then (Q^T Y) Omega^-1
// One workgroup per instance, or per (instance, chunk of columns or rows).
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
// trans (B_p^T) else T (B_p).  Target: the trailing columns of W (target_w)
// or the M x (G K) vector array C.  The rows are cut into segments of
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

struct ApplyTarget {
  const double* a0;  // panel block of the reflectors (row c0, column c0)
  double* cb;        // row c0 of the target
  int w, rows, ncols, ld, seg_rows, r_seg;
};

// the apply's target for this workgroup, or false when it has nothing to do
template <bool TW>
__device__ __forceinline__ bool apply_target(const RedDesc& d, int panel, const double* W,
                                             double* C, ApplyTarget& a) {
  const int c0 = panel * RP;
  if (c0 >= d.kr) return false;
  a.w = min(RP, d.kr - c0);
  a.rows = d.M - c0;
  a.a0 = W + d.w_off + (int64_t)c0 * d.n + c0;
  if (TW) {
    a.ncols = d.n - c0 - a.w;
    a.ld = d.n;
    a.cb = C + d.w_off + (int64_t)c0 * d.n + c0 + a.w;
  } else {
    a.ncols = d.G * d.K;
    a.ld = a.ncols;
    a.cb = C + d.v_off + (int64_t)c0 * a.ld;
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

template <bool TW>
__global__ void __launch_bounds__(QNT)
k_red_apply_z(const RedDesc* __restrict__ descs, int panel, const double* __restrict__ W,
              double* __restrict__ C, double* __restrict__ Zp) {
  const RedDesc d = descs[blockIdx.x];
  ApplyTarget a;
  if (!apply_target<TW>(d, panel, W, C, a)) return;
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

template <bool TW>
__global__ void __launch_bounds__(QNT)
k_red_apply_c(const RedDesc* __restrict__ descs, int panel, const double* __restrict__ W,
              const double* __restrict__ T, double* __restrict__ C,
              const double* __restrict__ Zp, int trans) {
  const RedDesc d = descs[blockIdx.x];
  ApplyTarget a;
  if (!apply_target<TW>(d, panel, W, C, a)) return;
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

// Reduced regressors Xr[t][c] = R[t][c] (c >= t, t < kr; zero elsewhere) and
// reduced responses yr = (Q^T Y) rows t < Mr.  Either output may be null.
__global__ void __launch_bounds__(QNT)
k_red_extract(const RedDesc* __restrict__ descs, const double* __restrict__ W,
              const double* __restrict__ Yt, double* __restrict__ Xr, double* __restrict__ yr) {
  const RedDesc d = descs[blockIdx.x];
  if (Xr) {
    const int64_t cnt = (int64_t)d.Mr * d.n;
    for (int64_t e = threadIdx.x; e < cnt; e += QNT) {
      const int t = (int)(e / d.n), c = (int)(e % d.n);
      Xr[d.xr_off + e] = (t < d.kr && c >= t) ? W[d.w_off + e] : 0.0;
    }
  }
  if (yr) {
    const int64_t cnt = (int64_t)d.Mr * d.G * d.K;
    for (int64_t e = threadIdx.x; e < cnt; e += QNT) yr[d.vr_off + e] = Yt[d.v_off + e];
  }
}

// Omega^-1 of every instance by Gauss-Jordan elimination without pivoting
// (Omega symmetric positive definite); a non-positive pivot marks every rhs of
// the instance as a breakdown and leaves a zero inverse.
__global__ void __launch_bounds__(QNT)
k_red_oinv(const RedDesc* __restrict__ descs, const double* __restrict__ Om,
           double* __restrict__ Oinv, int32_t* __restrict__ info) {
  const RedDesc d = descs[blockIdx.x];
  const int G = d.G, tid = threadIdx.x;
  __shared__ double A[64][129];   // [Omega | I] -> [I | Omega^-1], G <= 64
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  for (int e = tid; e < G * 2 * G; e += QNT) {
    const int i = e / (2 * G), j = e % (2 * G);
    A[i][j] = (j < G) ? Om[d.om_off + (int64_t)i * G + j] : (j - G == i ? 1.0 : 0.0);
  }
  __syncthreads();
  double scale = 0.0;
  for (int i = 0; i < G; ++i) scale = fmax(scale, fabs(A[i][i]));
  for (int p = 0; p < G; ++p) {
    const double piv = A[p][p];
    __syncthreads();
    if (!(piv > 1e-14 * scale)) {
      if (tid == 0) s_bad = 1;
      break;
    }
    // row p scaled, then eliminated from every other row; column p is left
    // alone here (it is the multiplier every update reads)
    for (int j = tid; j < 2 * G; j += QNT) A[p][j] /= piv;
    __syncthreads();
    for (int e = tid; e < G * 2 * G; e += QNT) {
      const int i = e / (2 * G), j = e % (2 * G);
      if (i != p && j != p) A[i][j] -= A[i][p] * A[p][j];
    }
    __syncthreads();
    for (int i = tid; i < G; i += QNT)
      if (i != p) A[i][p] = 0.0;
    __syncthreads();
  }
  __syncthreads();
  const bool bad = s_bad != 0;
  if (bad && info && tid < d.K) info[d.rhs0 + tid] = GLM_INFO_BREAKDOWN;
  for (int e = tid; e < G * G; e += QNT)
    Oinv[d.om_off + e] = bad ? 0.0 : A[e / G][G + e % G];
}

// U before the final rotation, RTR rows per workgroup (instance, chunk):
// rows t < Mr from the reduced solve, rows t >= Mr = (Q^T Y)[t] Omega^-1.
constexpr int RTR = 64;

__global__ void __launch_bounds__(QNT)
k_red_tail(const RedDesc* __restrict__ descs, const double* __restrict__ Oinv,
           const double* __restrict__ Yt, const double* __restrict__ ur,
           double* __restrict__ u) {
  const RedDesc d = descs[blockIdx.x];
  const int t0 = blockIdx.y * RTR;
  if (t0 >= d.M) return;
  const int G = d.G, K = d.K, P = G * K, tid = threadIdx.x;
  const int t1 = min(d.M, t0 + RTR);
  __shared__ double Oi[64 * 64];
  if (t1 > d.Mr)
    for (int e = tid; e < G * G; e += QNT) Oi[e] = Oinv[d.om_off + e];
  __syncthreads();
  for (int64_t e = (int64_t)t0 * P + tid; e < (int64_t)t1 * P; e += QNT) {
    const int64_t t = e / P;
    if (t < d.Mr) {
      u[d.v_off + e] = ur[d.vr_off + e];
    } else {
      const int rem = (int)(e - t * P), j = rem / K, k = rem - (rem / K) * K;
      const double* yrow = Yt + d.v_off + t * P + k;
      double s = 0.0;
      for (int i = 0; i < G; ++i) s += yrow[(int64_t)i * K] * Oi[i * G + j];
      u[d.v_off + e] = s;
    }
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
                           const double* T, double* C, double* Zp, int target_w, int trans,
                           int maxcols, int maxrows, hipStream_t s) {
  if (B <= 0 || maxcols <= 0 || maxrows <= 0) return hipSuccess;
  const dim3 grid(B, (maxcols + QNT - 1) / QNT, (maxrows + RED_SEG - 1) / RED_SEG);
  // separate instantiations for W and for the vectors: their shapes differ,
  // and so do their durations in a kernel trace
  if (target_w)
    hipLaunchKernelGGL(k_red_apply_z<true>, grid, dim3(QNT), 0, s, d, panel, W, C, Zp);
  else
    hipLaunchKernelGGL(k_red_apply_z<false>, grid, dim3(QNT), 0, s, d, panel, W, C, Zp);
  if (hipError_t e = hipGetLastError()) return e;
  if (target_w)
    hipLaunchKernelGGL(k_red_apply_c<true>, grid, dim3(QNT), 0, s, d, panel, W, T, C,
                       (const double*)Zp, trans);
  else
    hipLaunchKernelGGL(k_red_apply_c<false>, grid, dim3(QNT), 0, s, d, panel, W, T, C,
                       (const double*)Zp, trans);
  return hipGetLastError();
}

hipError_t launch_red_extract(const RedDesc* d, int B, const double* W, const double* Yt,
                             double* Xr, double* yr, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_extract, dim3(B), dim3(QNT), 0, s, d, W, Yt, Xr, yr);
  return hipGetLastError();
}

hipError_t launch_red_tail(const RedDesc* d, int B, int maxM, const double* Om, double* Oinv,
                          const double* Yt, const double* ur, double* u, int32_t* info,
                          hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_oinv, dim3(B), dim3(QNT), 0, s, d, Om, Oinv, info);
  if (hipError_t e = hipGetLastError()) return e;
  const int chunks = (maxM + RTR - 1) / RTR;
  hipLaunchKernelGGL(k_red_tail, dim3(B, chunks), dim3(QNT), 0, s, d, Oinv, Yt, ur, u);
  return hipGetLastError();
}

}  // namespace glm
