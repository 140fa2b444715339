// Batched Householder QR of tall, uneven blocks (double precision), run once
// per problem.  The SUR section factors every X_i once (X_i = Q_i R_i) so that
// each PCG step only needs products with Q_i and triangular solves with R_i.
//
// One workgroup factors one block in place (Householder reflectors in the
// LAPACK geqr2 convention), copies R out, then overwrites the reflectors with
// the explicit thin Q (LAPACK org2r order).  Every pass over the block is
// fused: the update by reflector j-1 and the dot products that define
// reflector j happen in the same sweep over the rows, so the factorization
// costs one read+write of the trailing block per column and forming Q costs
// the same again.  A row's trailing segment lives in registers (NMAX wide).
#include "glm_internal.h"
#include "qr_panel.h"

#include <cfloat>
#include <climits>
#include <cmath>

namespace glm {

namespace {

// Sum dots[k] (k in [lo, cols)) over the workgroup; result in out[k].
template <int NMAX>
__device__ void block_sum(double (&dots)[NMAX], int lo, int cols,
                          double (*red)[QW], double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    if (k >= lo && k < cols) {
      double s = wave_sum(dots[k]);
      if (lane == 0) red[k][wv] = s;
    }
  }
  __syncthreads();
  for (int k = lo + (int)threadIdx.x; k < cols; k += QNT) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < QW; ++q) s += red[k][q];
    out[k] = s;
  }
  __syncthreads();
}

// Column equilibration by powers of two.  Column c of the rows x cols block
// (cols <= 64) is multiplied by 2^-ex[c], ex[c] the binary exponent of its
// largest magnitude (frexp convention; 0 for a column of zeros).  The
// scaling is exact and Householder QR commutes with it: the reflectors and
// Q of the scaled block are those of the block itself, and R's column c
// comes out multiplied by 2^-ex[c].  With every column's largest entry in
// [1/2, 1) the norms of the factorization neither overflow nor underflow,
// whatever the scale of the data, and the zero-subcolumn threshold of the
// reflectors acts relative to the column's magnitude.
__device__ void equilibrate_cols(double* __restrict__ a0, int rows, int cols, int ld,
                                 int* __restrict__ ex, int (*part)[QW]) {
  const int tid = threadIdx.x, c = tid & 63, rg = tid >> 6;
  int e = INT_MIN;
  if (c < cols)
    for (int t = rg; t < rows; t += QW) {
      const double v = fabs(a0[(int64_t)t * ld + c]);
      if (v > 0.0 && v <= DBL_MAX) {
        int q;
        (void)frexp(v, &q);
        e = max(e, q);
      }
    }
  part[c][rg] = e;
  __syncthreads();
  if (tid < cols) {
    int m = INT_MIN;
#pragma unroll
    for (int q = 0; q < QW; ++q) m = max(m, part[tid][q]);
    ex[tid] = (m == INT_MIN) ? 0 : m;
  }
  __syncthreads();
  if (c < cols && ex[c] != 0)
    for (int t = rg; t < rows; t += QW)
      a0[(int64_t)t * ld + c] = ldexp(a0[(int64_t)t * ld + c], -ex[c]);
  __syncthreads();
}

// R (upper triangle of the first cols rows of the factored, equilibrated
// block) out with the column scaling undone, and the rank check on the
// equilibrated factor: a diagonal entry at most eps max(rows, cols) ||R||_F
// flags the block.  Column scaling does not change the column space, so the
// check is made where every column has unit scale.
__device__ void r_out_and_rank(const QRJob& job, const double* __restrict__ a0, int rows,
                               int cols, int ld, const int* __restrict__ ex,
                               double* __restrict__ Rout, int* __restrict__ flags,
                               double* fro2) {
  const int tid = threadIdx.x;
  if (tid == 0) *fro2 = 0.0;
  __syncthreads();
  double loc = 0.0;
  for (int e = tid; e < cols * cols; e += QNT) {
    const int r = e / cols, cc = e % cols;
    const double v = (cc >= r) ? a0[(int64_t)r * ld + cc] : 0.0;
    if (job.r_off >= 0) Rout[job.r_off + e] = ldexp(v, ex[cc]);
    loc += v * v;
  }
  loc = wave_sum(loc);
  if ((tid & 63) == 0) atomicAdd(fro2, loc);
  __syncthreads();
  if (tid == 0) {
    const double tolr = 2.220446049250313e-16 * (double)(rows > cols ? rows : cols) *
                        sqrt(*fro2);
    int bad = 0;
    for (int r = 0; r < cols; ++r)
      if (!(fabs(a0[(int64_t)r * ld + r]) > tolr)) bad = 1;
    if (job.flag >= 0) flags[job.flag] = bad;
  }
  __syncthreads();
}

template <int NMAX>
__global__ void __launch_bounds__(QNT)
k_qr(const QRJob* __restrict__ jobs, double* __restrict__ A,
     double* __restrict__ Rout, int* __restrict__ flags) {
  const QRJob job = jobs[blockIdx.x];
  const int rows = job.rows, cols = job.cols, ld = job.ld;
  double* __restrict__ a0 = A + job.a_off;

  __shared__ double red[NMAX][QW];
  __shared__ double dsum[NMAX];
  __shared__ double pivrow[NMAX];
  __shared__ double wk[NMAX];
  __shared__ double tau_s[NMAX];
  __shared__ double par[3];          // beta, tau, scale of the current reflector
  __shared__ double fro2;

  __shared__ int ex[NMAX];
  __shared__ int part[64][QW];
  const int tid = threadIdx.x;
  double dots[NMAX];
  equilibrate_cols(a0, rows, cols, ld, ex, part);

  // ---- factorization: pass p applies reflector p-1 and builds reflector p --
  for (int p = 0; p <= cols; ++p) {
    const int j = p - 1;
    const double beta_j = (p > 0) ? par[0] : 0.0;
    const double tau_j = (p > 0) ? par[1] : 0.0;
    const double scale_j = (p > 0) ? par[2] : 0.0;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) dots[k] = 0.0;
    const int lo = (j > 0) ? j : 0;
    for (int t = lo + tid; t < rows; t += QNT) {
      double a[NMAX];
      double* rowp = a0 + (int64_t)t * ld;
#pragma unroll
      for (int k = 0; k < NMAX; ++k)
        if (k >= lo && k < cols) a[k] = rowp[k];
      if (p > 0) {
        double vv = 1.0;   // reflector j at row t (v[j] = 1, scaled below)
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k == j && t > j) vv = a[k] * scale_j;
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k > j && k < cols) a[k] -= tau_j * vv * wk[k];
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k == j) a[k] = (t == j) ? beta_j : vv;
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k >= j && k < cols) rowp[k] = a[k];
      }
      if (p < cols && t == p) {
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k >= p && k < cols) pivrow[k] = a[k];
      }
      if (p < cols && t > p) {
        // dot products of the subcolumn below the pivot with every column
        double ap = 0.0;
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k == p) ap = a[k];
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k >= p && k < cols) dots[k] += ap * a[k];
      }
    }
    if (p == cols) break;
    __syncthreads();  // pivrow visible, all rows written
    block_sum<NMAX>(dots, p, cols, red, dsum);
    if (tid == 0) {
      const double alpha = pivrow[p];
      const double xnorm2 = dsum[p];            // squared norm below the pivot
      const double nrm2 = alpha * alpha + xnorm2;
      double beta, tau, scale;
      if (!(xnorm2 > kQrTinyNorm2)) {
        beta = alpha;  // H = I (LAPACK: tau = 0 when the subcolumn is zero)
        tau = 0.0;
        scale = 0.0;
      } else {
        const double nrm = sqrt(nrm2);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      par[0] = beta;
      par[1] = tau;
      par[2] = scale;
      tau_s[p] = tau;
      for (int k = p + 1; k < cols; ++k)
        wk[k] = pivrow[k] + scale * dsum[k];    // v^T a_k with v = [1; x * scale]
    }
    __syncthreads();
  }
  __syncthreads();

  // ---- R out (upper triangle of the first cols rows), rank check ---------
  r_out_and_rank(job, a0, rows, cols, ld, ex, Rout, flags, &fro2);

  // ---- explicit thin Q, backward accumulation of the reflectors ---------
  // pass j: apply H(j) (w from the previous pass) to columns > j, finalize
  // column j, then the dot products of H(j-1) with columns >= j.
  for (int j = cols - 1; j >= 0; --j) {
    const double tau_j = tau_s[j];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) dots[k] = 0.0;
    const int lo = (j > 0) ? j - 1 : 0;
    // rows above lo: column j becomes zero (row j-1 is handled in the sweep)
    for (int t = tid; t < lo && t < rows; t += QNT) a0[(int64_t)t * ld + j] = 0.0;
    for (int t = lo + tid; t < rows; t += QNT) {
      double a[NMAX];
      double* rowp = a0 + (int64_t)t * ld;
#pragma unroll
      for (int k = 0; k < NMAX; ++k)
        if (k >= lo && k < cols) a[k] = rowp[k];
      if (t >= j) {
        double vj = 1.0;
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k == j && t > j) vj = a[k];
        if (j < cols - 1) {
#pragma unroll
          for (int k = 0; k < NMAX; ++k)
            if (k > j && k < cols) a[k] -= tau_j * vj * wk[k];
        }
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k == j) a[k] = (t > j) ? -tau_j * vj : 1.0 - tau_j;
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k >= j && k < cols) rowp[k] = a[k];
      } else {
        // t == j - 1: above the diagonal of column j
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k == j) a[k] = 0.0;
        rowp[j] = 0.0;
      }
      if (j >= 1) {
        // reflector j-1: v[j-1] = 1, v[t] = a[j-1] below
        double vjm = 0.0;
        if (t == j - 1) {
          vjm = 1.0;
        } else {
#pragma unroll
          for (int k = 0; k < NMAX; ++k)
            if (k == j - 1) vjm = a[k];
        }
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k >= j && k < cols) dots[k] += vjm * a[k];
      }
    }
    __syncthreads();
    if (j >= 1) {
      block_sum<NMAX>(dots, j, cols, red, dsum);
      for (int k = j + (int)tid; k < cols; k += QNT) wk[k] = dsum[k];
      __syncthreads();
    }
  }
}

// rows in flight per lane in the per-block factorization and Q formation
constexpr int K32_U = 8;
constexpr int K32_SLOTS = QNT / 32;

__global__ void __launch_bounds__(QNT)
k_qr32(const QRJob* __restrict__ jobs, double* __restrict__ A, double* __restrict__ Rout,
       int* __restrict__ flags) {
  const QRJob job = jobs[blockIdx.x];
  const int rows = job.rows, cols = job.cols, ld = job.ld;
  double* __restrict__ a0 = A + job.a_off;

  __shared__ Qr32Shared<QNT> sh;
  __shared__ double fro2;
  __shared__ double wk[32];   // the Q formation's v^T a_c of the next reflector
  double (*red)[QW] = sh.red;
  double* dsum = sh.dsum;
  const double* tau_s = sh.tau_s;

  __shared__ int ex[32];
  __shared__ int part[64][QW];
  const int tid = threadIdx.x, c = tid & 31, slot = tid >> 5;
  const bool colok = c < cols;

  equilibrate_cols(a0, rows, cols, ld, ex, part);
  qr32_factor<QNT, K32_U>(a0, rows, cols, ld, sh);

  // ---- R out (upper triangle of the first cols rows), rank check ---------
  r_out_and_rank(job, a0, rows, cols, ld, ex, Rout, flags, &fro2);

  // ---- explicit thin Q, backward accumulation of the reflectors ---------
  for (int j = cols - 1; j >= 0; --j) {
    const double tau_j = tau_s[j];
    const double wkc = (j < cols - 1 && c > j && colok) ? wk[c] : 0.0;
    const int lo = (j > 0) ? j - 1 : 0;
    double dot = 0.0;
    // rows above lo: column j becomes zero (row j-1 is handled in the sweep)
    for (int t = tid; t < lo && t < rows; t += QNT) a0[(int64_t)t * ld + j] = 0.0;
    // the sweep starts at a multiple of K32_SLOTS * K32_U, so that a row is
    // loaded and stored by the same half-wave in every pass
    for (int t0 = lo & ~(K32_SLOTS * K32_U - 1); t0 < rows; t0 += K32_SLOTS * K32_U) {
      double a[K32_U];
#pragma unroll
      for (int u = 0; u < K32_U; ++u) {
        const int t = t0 + slot + K32_SLOTS * u;
        a[u] = (t < rows && t >= lo && colok && c >= lo) ? a0[(int64_t)t * ld + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < K32_U; ++u) {
        const int t = t0 + slot + K32_SLOTS * u;
        const bool rok = t < rows && t >= lo;
        double x = a[u];
        // columns j and j-1 of this row as loaded (this pass changes columns >= j)
        const double xj = shfl_col(x, j);
        const double xjm = shfl_col(x, j >= 1 ? j - 1 : 0);
        if (t >= j) {
          const double vj = (t > j) ? xj : 1.0;
          if (c > j) x -= tau_j * vj * wkc;
          if (c == j) x = (t > j) ? -tau_j * vj : 1.0 - tau_j;
          if (rok && colok && c >= j) a0[(int64_t)t * ld + c] = x;
        } else {
          // t == j - 1: above the diagonal of column j
          if (c == j) x = 0.0;
          if (rok && c == j) a0[(int64_t)t * ld + j] = 0.0;
        }
        if (j >= 1) {
          // reflector j-1: v[j-1] = 1, v[t] = a[j-1] below
          const double vjm = (t == j - 1) ? 1.0 : xjm;
          if (rok && c >= j) dot += vjm * x;
        }
      }
    }
    __syncthreads();
    if (j >= 1) {
      col_sum<QNT>(dot, j, cols, red, dsum);
      if (tid >= j && tid < cols) wk[tid] = dsum[tid];
      __syncthreads();
    }
  }
}

__global__ void k_to_float(const double* __restrict__ src, float* __restrict__ dst,
                           int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

// M0 = [ -R^-T R_c^T ; I_k ] for one restricted instance per workgroup, stored
// row-major ((n + k) x k) at nb_off; its orthonormalised columns span the null
// space of [R; R_c]^T (R = direct sum of the R_i).
__global__ void k_nullbasis_input(const InstDesc* __restrict__ insts,
                                  const int* __restrict__ rinst,
                                  const BlockDesc* __restrict__ blks,
                                  const double* __restrict__ R,
                                  const double* __restrict__ Rc,
                                  double* __restrict__ Nb) {
  const InstDesc in = insts[rinst[blockIdx.x]];
  const int n = in.n, kc = in.kc;
  double* nb = Nb + in.nb_off;
  const double* rc = Rc + in.rc_off;
  // one thread per (block i, restriction row q): forward substitution R_i^T z = rc_i
  for (int job = threadIdx.x; job < in.G * kc; job += blockDim.x) {
    const int i = job / kc, q = job % kc;
    const BlockDesc bd = blks[in.blk0 + i];
    const double* Ri = R + bd.r_off;
    for (int a = 0; a < bd.ni; ++a) {
      double s = rc[(int64_t)q * n + bd.col + a];
      for (int b = 0; b < a; ++b) s -= Ri[b * bd.ni + a] * nb[(int64_t)(bd.col + b) * kc + q];
      nb[(int64_t)(bd.col + a) * kc + q] = s / Ri[a * bd.ni + a];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * kc; e += blockDim.x) nb[e] = -nb[e];
  for (int e = threadIdx.x; e < kc * kc; e += blockDim.x)
    nb[(int64_t)n * kc + e] = ((e / kc) == (e % kc)) ? 1.0 : 0.0;
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

hipError_t launch_qr(const QRJob* d_jobs, int njobs, int nmax, double* A,
                     double* R, int* flags, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (nmax <= 32)
    hipLaunchKernelGGL(k_qr32, dim3(njobs), dim3(QNT), 0, s, d_jobs, A, R, flags);
  else
    hipLaunchKernelGGL(k_qr<64>, dim3(njobs), dim3(QNT), 0, s, d_jobs, A, R, flags);
  return hipGetLastError();
}

hipError_t launch_to_float(const double* src, float* dst, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_to_float, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_nullbasis_input(const InstDesc* insts, const int* rinst, int nr,
                                  const BlockDesc* blks, const double* R,
                                  const double* Rc, double* Nb, hipStream_t s) {
  if (nr <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nullbasis_input, dim3(nr), dim3(256), 0, s, insts, rinst, blks,
                     R, Rc, Nb);
  return hipGetLastError();
}

}  // namespace glm
