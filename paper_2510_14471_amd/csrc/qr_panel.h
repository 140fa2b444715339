// Householder factorization of narrow blocks (at most 32 columns) by one
// workgroup: shared by the per-block QR of the SUR regressors and the panel
// steps of the model-reduction QR.
#pragma once

#include "glm_internal.h"

#include <cmath>

namespace glm {
namespace {

constexpr int QNT = 256;            // threads per QR workgroup
// A subcolumn whose squared norm is below this is taken as exactly zero
// (H = I).  Exact linear dependencies among the columns (the intercept of
// every equation in W = [X_1 ... X_G]) leave subcolumns that shrink by about
// eps per dependent column; squaring entries below ~1e-154 underflows and
// would give a norm inconsistent with the stored reflector.
constexpr double kQrTinyNorm2 = 1e-250;
constexpr int QW = QNT / 64;        // waves per QR workgroup

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Factorization of blocks of at most 32 columns with the data mapping turned
// around against the row-per-lane form: lane l owns column l % 32, and the row slot
// 2 w + l / 32 of wave w takes rows slot, slot + NT / 32, ...  A row segment is
// then one coalesced access, U rows per lane are in flight at once, the dot
// products are one register per lane, and the pivot-column entry of a row
// comes from its lane by a shuffle.  Arithmetic and order of the updates
// follow k_qr; only the summation order of the dot products differs.  NT is
// the workgroup size (a multiple of 64).

// value of column col in the row this lane's half-wave holds
__device__ __forceinline__ double shfl_col(double v, int col) {
  return __shfl(v, (int)(threadIdx.x & 32) | col, 64);
}

// dsum[k] = sum of dot over the workgroup's lanes of column k, k in [lo, cols)
template <int NT>
__device__ __forceinline__ void col_sum(double dot, int lo, int cols, double (*red)[NT / 64],
                                        double* dsum) {
  const int tid = threadIdx.x;
  dot += __shfl_xor(dot, 32, 64);
  if ((tid & 63) < 32) red[tid & 31][tid >> 6] = dot;
  __syncthreads();
  if (tid >= lo && tid < cols) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) s += red[tid][q];
    dsum[tid] = s;
  }
  __syncthreads();
}

// Householder factorization of a rows x cols block (cols <= 32) at a0 with
// row stride ld, in place (R on and above the diagonal, the reflectors below,
// LAPACK geqr2 convention); tau_s receives the reflector scalars.  Called by
// every thread of the workgroup.
template <int NT>
struct Qr32Shared {
  double red[32][NT / 64];
  double dsum[32];
  double pivrow[2][32];   // the pivot rows of consecutive reflectors, alternating
  double tau_s[32];
};

template <int NT, int U>
__device__ void qr32_factor(double* __restrict__ a0, int rows, int cols, int ld,
                            Qr32Shared<NT>& sh) {
  constexpr int SLOTS = NT / 32;   // row slots per workgroup
  static_assert(NT % 64 == 0 && ((SLOTS * U) & (SLOTS * U - 1)) == 0,
                "whole waves; rows per sweep step a power of two");
  double (*red)[NT / 64] = sh.red;
  double* dsum = sh.dsum;
  double* tau_s = sh.tau_s;
  const int tid = threadIdx.x, c = tid & 31, slot = tid >> 5;
  const bool colok = c < cols;
  // Every thread forms each reflector's scalars itself (the same arithmetic
  // on the same shared values), so the two barriers of col_sum are the only
  // ones per reflector: the sweep writes the other pivot-row buffer, a row
  // is loaded and stored by the same half-wave in every sweep, and dsum and
  // red are rewritten only after the next col_sum's first barrier.
  double beta_j = 0.0, tau_j = 0.0, scale_j = 0.0;
  for (int p = 0; p <= cols; ++p) {
    const int j = p - 1;
    // v^T a_c of reflector j (v = [1; x scale]) from its pivot row and dot
    // products; each lane forms its own column's
    const double wkc =
        (p > 0 && c > j && colok) ? sh.pivrow[j & 1][c] + scale_j * dsum[c] : 0.0;
    const int lo = (j > 0) ? j : 0;
    double dot = 0.0;
    // the sweep starts at a multiple of SLOTS * U, so that a row is
    // loaded and stored by the same half-wave in every pass
    for (int t0 = lo & ~(SLOTS * U - 1); t0 < rows; t0 += SLOTS * U) {
      double a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + slot + SLOTS * u;
        a[u] = (t < rows && t >= lo && colok && c >= lo) ? a0[(int64_t)t * ld + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + slot + SLOTS * u;
        const bool rok = t < rows && t >= lo;
        double x = a[u];
        if (p > 0) {
          const double aj = shfl_col(x, j);
          const double vv = (t > j) ? aj * scale_j : 1.0;   // reflector j at row t
          if (c > j) x -= tau_j * vv * wkc;
          if (c == j) x = (t == j) ? beta_j : vv;
          if (rok && colok && c >= j) a0[(int64_t)t * ld + c] = x;
        }
        if (p < cols) {
          if (rok && t == p && colok && c >= p) sh.pivrow[p & 1][c] = x;
          // dot products of the subcolumn below the pivot with every column
          const double ap = shfl_col(x, p);
          if (rok && t > p && c >= p) dot += ap * x;
        }
      }
    }
    if (p == cols) break;
    col_sum<NT>(dot, p, cols, red, dsum);
    const double alpha = sh.pivrow[p & 1][p];
    const double xnorm2 = dsum[p];            // squared norm below the pivot
    if (!(xnorm2 > kQrTinyNorm2)) {
      beta_j = alpha;  // H = I (LAPACK: tau = 0 when the subcolumn is zero)
      tau_j = 0.0;
      scale_j = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + xnorm2);
      beta_j = (alpha >= 0.0) ? -nrm : nrm;
      tau_j = (beta_j - alpha) / beta_j;
      scale_j = 1.0 / (alpha - beta_j);
    }
    if (tid == 0) tau_s[p] = tau_j;
  }
  __syncthreads();
}

}  // namespace
}  // namespace glm
