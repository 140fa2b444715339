// A generalized inverse of a symmetric positive semi-definite G x G matrix by
// one workgroup: shared by the model reduction (Omega^g of the full model's
// u) and the normal-equations solver (Omega^-1 of Sigma^-1 = Omega^-1 (x) I_M).
#pragma once

#include "glm_internal.h"

#include <cmath>

namespace glm {
namespace {

constexpr int GINV_NT = 256;   // workgroup size of psd_ginv's callers

// Cholesky with diagonal pivoting of the PSD matrix o (row-major G x G,
// G <= 256), stopped when the largest remaining diagonal is at most
// 16 G eps trace(o) (the numerical rank r).  With L the r x r factor and Pm
// the pivoting, og = Pm [L^-T L^-1, 0; 0, 0] Pm^T satisfies o og o = o and is
// the inverse when r = G.  a is a G x G work area in global memory.  Called
// by every thread of a GINV_NT-thread workgroup; returns r to every thread.
__device__ int psd_ginv(int G, const double* __restrict__ o, double* __restrict__ a,
                        double* __restrict__ og) {
  const int tid = threadIdx.x;
  __shared__ int perm[256];
  __shared__ double dinv[256];
  __shared__ double s_piv, s_tol;
  __shared__ int s_j;
  for (int e = tid; e < G * G; e += GINV_NT) a[e] = o[e];
  for (int i = tid; i < G; i += GINV_NT) perm[i] = i;
  if (tid < 64) {
    double tr = 0.0;
    for (int i = tid; i < G; i += 64) tr += fabs(o[(int64_t)i * G + i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
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
      for (int c = tid; c < G; c += GINV_NT) {
        const double t0 = a[(int64_t)k * G + c];
        a[(int64_t)k * G + c] = a[(int64_t)j * G + c];
        a[(int64_t)j * G + c] = t0;
      }
      __syncthreads();
      for (int rr = k + tid; rr < G; rr += GINV_NT) {
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
    for (int i = k + 1 + tid; i < G; i += GINV_NT) a[(int64_t)i * G + k] /= lkk;
    if (tid == 0) {
      a[(int64_t)k * G + k] = lkk;
      dinv[k] = 1.0 / lkk;
    }
    __syncthreads();
    const int w = G - k - 1;
    for (int e = tid; e < w * w; e += GINV_NT) {
      const int i = k + 1 + e / w, c = k + 1 + e % w;
      a[(int64_t)i * G + c] -= a[(int64_t)i * G + k] * a[(int64_t)c * G + k];
    }
    __syncthreads();
  }
  // column c of L^-1 (rows i > c) into the upper triangle: a[c][i] = (L^-1)[i][c]
  for (int c = tid; c < r; c += GINV_NT) {
    for (int i = c + 1; i < r; ++i) {
      double s = a[(int64_t)i * G + c] * dinv[c];
      for (int kk = c + 1; kk < i; ++kk) s += a[(int64_t)i * G + kk] * a[(int64_t)c * G + kk];
      a[(int64_t)c * G + i] = -s * dinv[i];
    }
  }
  __syncthreads();
  for (int e = tid; e < G * G; e += GINV_NT) {
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
  __syncthreads();
  return r;
}

}  // namespace
}  // namespace glm
