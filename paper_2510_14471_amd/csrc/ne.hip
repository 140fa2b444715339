// Conjugate gradients on the normal equations of the GLS problem (PCG-NE,
// the comparator of PCG-Aug in the section on the statistical properties of
// the PCG-Aug estimator):
//
//     (X^T Sigma^-1 X) beta = X^T Sigma^-1 y,   Sigma^-1 = Omega^-1 (x) I_M,
//
// with the block-Jacobi preconditioner made of the diagonal blocks
// w^ii X_i^T X_i = w^ii R_i^T R_i of the normal matrix ([w^ij] = Omega^-1),
// one pair of triangular solves per equation.  The normal matrix is never
// formed: X^T Sigma^-1 X p is one expansion w = X p and one projection
// X^T (w Omega^-1), done by the projection-pass kernels with X in place of Q
// and Omega^-1 in place of Omega; the projection returns the negated product.
//
//   k_ne_oinv   Omega^-1 per instance (pivoted Cholesky; instances whose
//               Omega is numerically singular stop with a breakdown)
//   k_ne_start  r = b, z = M^-1 r, p = z, rho = r^T z from T = -b
//   k_ne_step   alpha = rho / p^T A p, beta += alpha p, r -= alpha A p, the
//               stopping test ||r|| <= tol ||b||, z = M^-1 r, p = z + (rho'/rho) p
//
// One workgroup per instance for the scalar kernels; lane (k, cg) =
// (tid % 16, tid / 16) walks the entries (c, k) of the n x K vectors with
// c = cg, cg + 16, ... and the per-rhs sums are reduced over the 16 groups.
#include "glm.h"
#include "ginv.h"
#include "glm_internal.h"

#include <cmath>

namespace glm {
namespace {

constexpr int NE_NT = 256;
constexpr int NE_CG = NE_NT / KMAX;   // column groups per workgroup

static_assert(NE_NT == GINV_NT, "one workgroup size for both scalar kernels");

// per-rhs sum of v over the workgroup (lane k = tid % KMAX); the result is
// valid in out[k] after the call
__device__ __forceinline__ void ne_sum(double v, double (*red)[NE_CG], double* out) {
  const int tid = threadIdx.x;
  red[tid % KMAX][tid / KMAX] = v;
  __syncthreads();
  if (tid < KMAX) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NE_CG; ++q) s += red[tid][q];
    out[tid] = s;
  }
  __syncthreads();
}

// z = M^-1 r for every (block, rhs) pair of the instance whose rhs is
// active: R_i^T y = r_i, then R_i z_i = y / w^ii, in place in z.
__device__ void ne_precond(const InstDesc& in, const BlockDesc* __restrict__ blks,
                           const double* __restrict__ R, const double* __restrict__ Oinv,
                           const double* __restrict__ r, double* __restrict__ z,
                           const int* act) {
  const int K = in.K;
  for (int q = threadIdx.x; q < in.G * K; q += NE_NT) {
    const int i = q / K, k = q - (q / K) * K;
    if (!act[k]) continue;
    const BlockDesc bd = blks[in.blk0 + i];
    const double* Ri = R + bd.r_off;
    const int ni = bd.ni;
    const int64_t o = in.t_off + (int64_t)bd.col * K + k;
    for (int a = 0; a < ni; ++a) {
      double s = r[o + (int64_t)a * K];
      for (int c = 0; c < a; ++c) s -= Ri[c * ni + a] * z[o + (int64_t)c * K];
      z[o + (int64_t)a * K] = s / Ri[a * ni + a];
    }
    const double wii = Oinv[in.om_off + (int64_t)i * in.G + i];
    for (int a = ni - 1; a >= 0; --a) {
      double s = z[o + (int64_t)a * K] / wii;
      for (int c = a + 1; c < ni; ++c) s -= Ri[a * ni + c] * z[o + (int64_t)c * K];
      z[o + (int64_t)a * K] = s / Ri[a * ni + a];
    }
  }
  __syncthreads();
}

// per-instance activity for the pass kernels and the host poll
__device__ __forceinline__ void ne_publish(int b, int K, const int* act, int* inst_active,
                                           int* icount) {
  if (threadIdx.x == 0) {
    int c = 0;
    for (int k = 0; k < K; ++k) c += act[k];
    icount[b] = c;
    inst_active[b] = c > 0;
  }
}

__global__ void __launch_bounds__(NE_NT)
k_ne_oinv(const InstDesc* __restrict__ insts, const double* __restrict__ Om,
          double* __restrict__ A, double* __restrict__ Oinv, RhsState* __restrict__ st,
          int* __restrict__ inst_active) {
  const int b = blockIdx.x;
  const InstDesc in = insts[b];
  const int r = psd_ginv(in.G, Om + in.om_off, A + in.om_off, Oinv + in.om_off);
  if (r < in.G) {
    if ((int)threadIdx.x < in.K && st[in.rhs0 + threadIdx.x].status == ST_ACTIVE)
      st[in.rhs0 + threadIdx.x].status = ST_BREAKDOWN;
    if (threadIdx.x == 0) inst_active[b] = 0;
  }
}

__global__ void __launch_bounds__(NE_NT)
k_ne_start(const InstDesc* __restrict__ insts, const BlockDesc* __restrict__ blks,
           const double* __restrict__ R, const double* __restrict__ Oinv,
           const double* __restrict__ Tm, double* __restrict__ x, double* __restrict__ r,
           double* __restrict__ z, double* __restrict__ p, RhsState* __restrict__ st,
           int* __restrict__ inst_active, int* __restrict__ icount) {
  const int b = blockIdx.x;
  const InstDesc in = insts[b];
  const int K = in.K, n = in.n, tid = threadIdx.x, kk = tid % KMAX, cg = tid / KMAX;
  __shared__ double red[KMAX][NE_CG];
  __shared__ double s_bn2[KMAX], s_rz[KMAX];
  __shared__ int s_act[KMAX];
  // the estimate starts at zero (and stays there for instances not solved)
  if (kk < K)
    for (int c = cg; c < n; c += NE_CG) x[in.b_off + (int64_t)c * K + kk] = 0.0;
  if (tid < KMAX) s_act[tid] = inst_active[b] && tid < K && st[in.rhs0 + tid].status == ST_ACTIVE;
  __syncthreads();
  if (!inst_active[b]) {
    if (tid == 0) icount[b] = 0;
    return;
  }
  double acc = 0.0;
  if (kk < K)
    for (int c = cg; c < n; c += NE_CG) {
      const int64_t e = in.t_off + (int64_t)c * K + kk;
      const double v = -Tm[e];
      r[e] = v;
      acc += v * v;
    }
  ne_sum(acc, red, s_bn2);
  ne_precond(in, blks, R, Oinv, r, z, s_act);
  acc = 0.0;
  if (kk < K && s_act[kk])
    for (int c = cg; c < n; c += NE_CG) {
      const int64_t e = in.t_off + (int64_t)c * K + kk;
      const double zv = z[e];
      p[e] = zv;
      acc += r[e] * zv;
    }
  ne_sum(acc, red, s_rz);
  if (tid < K) {
    RhsState s = st[in.rhs0 + tid];
    s.ynorm2 = s_bn2[tid];
    s.rnorm2 = s_bn2[tid];
    s.c = s_rz[tid];
    s.iters = s.total_iters = 0;
    if (s_act[tid] && !(s_bn2[tid] > 0.0)) {   // b = 0: beta = 0 solves it
      s.status = ST_CONVERGED;
      s_act[tid] = 0;
    }
    st[in.rhs0 + tid] = s;
  }
  __syncthreads();
  ne_publish(b, K, s_act, inst_active, icount);
}

__global__ void __launch_bounds__(NE_NT)
k_ne_step(const InstDesc* __restrict__ insts, const BlockDesc* __restrict__ blks,
          const double* __restrict__ R, const double* __restrict__ Oinv,
          const double* __restrict__ Tm, double* __restrict__ x, double* __restrict__ r,
          double* __restrict__ z, double* __restrict__ p, RhsState* __restrict__ st,
          int* __restrict__ inst_active, int* __restrict__ icount, double tol, int maxit_user) {
  const int b = blockIdx.x;
  if (!inst_active[b]) return;
  const InstDesc in = insts[b];
  const int K = in.K, n = in.n, tid = threadIdx.x, kk = tid % KMAX, cg = tid / KMAX;
  const int maxit = maxit_user > 0 ? maxit_user : n;
  __shared__ double red[KMAX][NE_CG];
  __shared__ double s_pap[KMAX], s_rn2[KMAX], s_rz[KMAX], s_alpha[KMAX];
  __shared__ int s_act[KMAX];
  if (tid < KMAX) s_act[tid] = tid < K && st[in.rhs0 + tid].status == ST_ACTIVE;
  __syncthreads();
  const bool mine = kk < K && s_act[kk];
  // Tm holds -A p
  double acc = 0.0;
  if (mine)
    for (int c = cg; c < n; c += NE_CG) {
      const int64_t e = in.t_off + (int64_t)c * K + kk;
      acc -= p[e] * Tm[e];
    }
  ne_sum(acc, red, s_pap);
  if (tid < K && s_act[tid]) {
    const double pap = s_pap[tid];
    if (!(pap > 0.0) || !std::isfinite(pap)) {
      st[in.rhs0 + tid].status = ST_BREAKDOWN;
      s_act[tid] = 0;
      s_alpha[tid] = 0.0;
    } else {
      s_alpha[tid] = st[in.rhs0 + tid].c / pap;
    }
  }
  __syncthreads();
  acc = 0.0;
  if (kk < K && s_act[kk]) {
    const double al = s_alpha[kk];
    for (int c = cg; c < n; c += NE_CG) {
      const int64_t e = in.t_off + (int64_t)c * K + kk;
      const int64_t xe = in.b_off + (int64_t)c * K + kk;
      x[xe] += al * p[e];
      const double rv = r[e] + al * Tm[e];
      r[e] = rv;
      acc += rv * rv;
    }
  }
  ne_sum(acc, red, s_rn2);
  if (tid < K && s_act[tid]) {
    RhsState s = st[in.rhs0 + tid];
    s.rnorm2 = s_rn2[tid];
    s.iters += 1;
    s.total_iters += 1;
    if (sqrt(s_rn2[tid]) <= tol * sqrt(s.ynorm2)) {
      s.status = ST_CONVERGED;
      s_act[tid] = 0;
    } else if (!std::isfinite(s_rn2[tid])) {
      s.status = ST_BREAKDOWN;
      s_act[tid] = 0;
    } else if (s.iters >= maxit) {
      s.status = ST_MAXITER;
      s_act[tid] = 0;
    }
    st[in.rhs0 + tid] = s;
  }
  __syncthreads();
  ne_precond(in, blks, R, Oinv, r, z, s_act);
  acc = 0.0;
  if (kk < K && s_act[kk])
    for (int c = cg; c < n; c += NE_CG) {
      const int64_t e = in.t_off + (int64_t)c * K + kk;
      acc += r[e] * z[e];
    }
  ne_sum(acc, red, s_rz);
  if (kk < K && s_act[kk]) {
    const double bt = s_rz[kk] / st[in.rhs0 + kk].c;
    for (int c = cg; c < n; c += NE_CG) {
      const int64_t e = in.t_off + (int64_t)c * K + kk;
      p[e] = z[e] + bt * p[e];
    }
  }
  __syncthreads();   // every lane has read the old rho before it is replaced
  if (tid < K && s_act[tid]) st[in.rhs0 + tid].c = s_rz[tid];
  ne_publish(b, K, s_act, inst_active, icount);
}

}  // namespace

hipError_t launch_ne_oinv(const InstDesc* insts, int B, const double* Om, double* A,
                          double* Oinv, RhsState* st, int* inst_active, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ne_oinv, dim3(B), dim3(NE_NT), 0, s, insts, Om, A, Oinv, st,
                     inst_active);
  return hipGetLastError();
}

hipError_t launch_ne_start(const InstDesc* insts, const BlockDesc* blks, int B, const double* R,
                           const double* Oinv, const double* Tm, double* x, double* r,
                           double* z, double* p, RhsState* st, int* inst_active, int* icount,
                           hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ne_start, dim3(B), dim3(NE_NT), 0, s, insts, blks, R, Oinv, Tm, x, r, z,
                     p, st, inst_active, icount);
  return hipGetLastError();
}

hipError_t launch_ne_step(const InstDesc* insts, const BlockDesc* blks, int B, const double* R,
                          const double* Oinv, const double* Tm, double* x, double* r,
                          double* z, double* p, RhsState* st, int* inst_active, int* icount,
                          double tol, int maxit_user, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ne_step, dim3(B), dim3(NE_NT), 0, s, insts, blks, R, Oinv, Tm, x, r, z,
                     p, st, inst_active, icount, tol, maxit_user);
  return hipGetLastError();
}

}  // namespace glm
