// Setup, iterative-refinement and gradient kernels around the PCG-Aug core.
//
//  * refinement (mixed precision): from the double-precision residual of the
//    augmented system  rho = [y - Sigma u - X beta ; h2 - X^T u]  (formed by
//    the FP64 projection passes with X, not the single-precision Q, in place
//    of Q), per (instance, rhs) the stopping test, the choice of the inner
//    precision and the right-hand sides of the next inner solve;
//  * gradients: dOmega = -sym(sum_t L_t U_t^T) (Kronecker-reduced outer
//    products of the adjoint and primal u blocks) and dX_i = -(l_u,i beta_i^T
//    + u_i l_beta,i^T), from the reverse rule of the augmented system.
#include "glm_internal.h"

#include <cmath>

namespace glm {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t count, T v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

// alpha_b = max_i omega_ii (D = alpha I); when requested, the per-equation
// scalars d_i = omega_ii of D = diag(d) (x) I_M (alpha for an equation with
// omega_ii = 0 and for every equation of a restricted instance, which keeps
// D = alpha I), and a single-precision Omega.
__global__ void k_alpha(const InstDesc* __restrict__ insts, int B,
                        const double* __restrict__ Om, double* __restrict__ alpha,
                        float* __restrict__ Om32, double* __restrict__ deq) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const InstDesc in = insts[b];
  const double* o = Om + in.om_off;
  double a = 0.0;
  for (int i = 0; i < in.G; ++i) a = fmax(a, o[i * in.G + i]);
  a = (a > 0.0) ? a : 1.0;
  if (threadIdx.x == 0) alpha[b] = a;
  if (deq)
    for (int i = threadIdx.x; i < in.G; i += blockDim.x) {
      const double di = o[i * in.G + i];
      deq[in.blk0 + i] = (in.kc == 0 && di > 1e-300 * a) ? di : a;
    }
  if (Om32)
    for (int e = threadIdx.x; e < in.G * in.G; e += blockDim.x) Om32[in.om_off + e] = (float)o[e];
}

// Fresh per-(instance, rhs) state; instances with a rank-deficient block are
// marked and excluded.  `status0` is ST_ACTIVE or ST_IDLE.
__global__ void k_state_init(const InstDesc* __restrict__ insts, int B,
                             const int* __restrict__ rankflag, int rank_extra_base,
                             const int* __restrict__ rinst_index,
                             RhsState* __restrict__ st, int* __restrict__ inst_active,
                             int* __restrict__ ost, int maxit_user) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const InstDesc in = insts[b];
  __shared__ int bad;
  if (threadIdx.x == 0) {
    int r = 0;
    for (int i = 0; i < in.G; ++i) r |= rankflag[in.blk0 + i];
    if (in.kc > 0 && rinst_index[b] >= 0) r |= rankflag[rank_extra_base + rinst_index[b]];
    bad = r;
    inst_active[b] = !r;
  }
  __syncthreads();
  if ((int)threadIdx.x < in.K) {
    RhsState s;
    s.c = s.c1 = s.d = s.lam = s.mu = s.cmin = 0.0;
    s.rnorm2 = s.ynorm2 = 0.0;
    s.status = bad ? ST_RANK : ST_ACTIVE;
    s.iters = s.since = s.total_iters = 0;
    s.itol = 0.0;
    s.esc = s.pad = 0;
    st[in.rhs0 + threadIdx.x] = s;
    if (ost) ost[in.rhs0 + threadIdx.x] = bad ? ST_RANK : ST_ACTIVE;
  }
  (void)maxit_user;
}

// Before a final projection: every instance with a solved rhs takes part.
__global__ void k_activate(const InstDesc* __restrict__ insts, int B,
                           const RhsState* __restrict__ st, int* __restrict__ inst_active) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const InstDesc in = insts[b];
  int any = 0;
  for (int k = 0; k < in.K; ++k) {
    const int s = st[in.rhs0 + k].status;
    any |= (s != ST_IDLE && s != ST_RANK);
  }
  inst_active[b] = any;
}

// restriction rows of X* h2 (bottom of the projected start) -> wc
template <typename T>
__global__ void k_copy_tc(const InstDesc* __restrict__ insts, int B, const T* __restrict__ Tm,
                          double* __restrict__ wc) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const InstDesc in = insts[b];
  for (int e = threadIdx.x; e < in.kc * in.K; e += blockDim.x)
    wc[in.c_off + e] = (double)Tm[in.t_off + (int64_t)in.n * in.K + e];
}

// Per instance: rho_0 = h2 - X^T w - R_c^T wc, rho_c = r - R_c beta, the norms
// and the outer stopping test.  Rhs that still need work become ST_ACTIVE for
// the next inner solve, the others ST_IDLE; ost keeps the outer outcome.
__global__ void __launch_bounds__(NT)
k_outer_check(const InstDesc* __restrict__ insts, const BlockDesc* __restrict__ blks,
              const double* __restrict__ R, int* __restrict__ inst_active,
              RhsState* __restrict__ st, int* __restrict__ ost,
              const double* __restrict__ rpart, const double* __restrict__ ypart,
              const double* __restrict__ XtW, double xtw_sign, const double* __restrict__ h2,
              const double* __restrict__ Rc, const double* __restrict__ rvec,
              const double* __restrict__ beta, const double* __restrict__ wc,
              double* __restrict__ rho0, double* __restrict__ rhoc, double tol,
              int step, int last_step) {
  const int b = blockIdx.x;
  const InstDesc in = insts[b];
  const int K = in.K, n = in.n, kc = in.kc;
  __shared__ int s_any;
  __shared__ double rr[NT / 64], yy[NT / 64];
  __shared__ double lo_r[KMAX], lo_y[KMAX];
  if (threadIdx.x == 0) s_any = 0;
  if ((int)threadIdx.x < KMAX) lo_r[threadIdx.x] = lo_y[threadIdx.x] = 0.0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // rho0 of every refining rhs
  for (int e = threadIdx.x; e < n * K; e += NT) {
    const int c = e / K, k = e - c * K;
    if (ost[in.rhs0 + k] != ST_ACTIVE) continue;
    const int64_t bi = in.b_off + e;
    double v = (h2 ? h2[bi] : 0.0) - xtw_sign * XtW[in.t_off + e];
    for (int q = 0; q < kc; ++q)
      v -= Rc[in.rc_off + (int64_t)q * n + c] * wc[in.c_off + (int64_t)q * K + k];
    rho0[bi] = v;
  }
  __syncthreads();
  // The lower block is measured in the coordinates of the orthonormal
  // factor: with X_i = Q_i R_i, X_i^T u = h_i is R_i^T (Q_i^T u) = h_i, so its
  // residual is R_i^-T rho0_i (for h2 = 0: Q^T u), which does not change when
  // the columns of X are scaled.  One (block, rhs) pair per thread.
  for (int e = threadIdx.x; e < in.G * K; e += NT) {
    const int i = e / K, k = e - i * K;
    if (ost[in.rhs0 + k] != ST_ACTIVE) continue;
    const BlockDesc bd = blks[in.blk0 + i];
    const double* Ri = R + bd.r_off;
    const int ni = bd.ni;
    const int64_t o = in.b_off + (int64_t)bd.col * K + k;
    double zr[QR_NMAX], zh[QR_NMAX];
    double ar = 0.0, ay = 0.0;
    for (int a = 0; a < ni; ++a) {
      double sr = rho0[o + (int64_t)a * K];
      double sh = h2 ? h2[o + (int64_t)a * K] : 0.0;
      for (int c = 0; c < a; ++c) {
        sr -= Ri[c * ni + a] * zr[c];
        sh -= Ri[c * ni + a] * zh[c];
      }
      zr[a] = sr / Ri[a * ni + a];
      zh[a] = sh / Ri[a * ni + a];
      ar += zr[a] * zr[a];
      ay += zh[a] * zh[a];
    }
    atomicAdd(&lo_r[k], ar);
    atomicAdd(&lo_y[k], ay);
  }
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    const int s_idx = in.rhs0 + k;
    const int o = ost[s_idx];
    if (o != ST_ACTIVE) continue;   // uniform across the workgroup
    double acc_r = 0.0, acc_y = 0.0;
    for (int q = wv; q < kc; q += NT / 64) {
      double s = 0.0;
      for (int c = lane; c < n; c += 64)
        s += Rc[in.rc_off + (int64_t)q * n + c] * beta[in.b_off + (int64_t)c * K + k];
      s = wave_sum(s);
      if (lane == 0) {
        const int64_t ci = in.c_off + (int64_t)q * K + k;
        const double rv = rvec ? rvec[ci] : 0.0;
        rhoc[ci] = rv - s;
      }
    }
    __syncthreads();
    // restriction contributions (few rows): one thread
    double extra_r = 0.0, extra_y = 0.0;
    if (threadIdx.x == 0) {
      extra_r = lo_r[k];
      extra_y = lo_y[k];
      for (int q = 0; q < kc; ++q) {
        const int64_t ci = in.c_off + (int64_t)q * K + k;
        const double rv = rvec ? rvec[ci] : 0.0;
        extra_r += rhoc[ci] * rhoc[ci];
        extra_y += rv * rv;
      }
      for (int p = 0; p < in.ntiles; ++p) {
        extra_r += rpart[(int64_t)(in.tile0 + p) * KMAX + k];
        extra_y += ypart[(int64_t)(in.tile0 + p) * KMAX + k];
      }
    }
    acc_r += extra_r;
    acc_y += extra_y;
    acc_r = wave_sum(acc_r);
    acc_y = wave_sum(acc_y);
    if (lane == 0) {
      rr[wv] = acc_r;
      yy[wv] = acc_y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double R2 = 0.0, Y2 = 0.0;
      for (int q = 0; q < NT / 64; ++q) {
        R2 += rr[q];
        Y2 += yy[q];
      }
      RhsState& s = st[s_idx];
      const double prev = s.rnorm2;   // residual of the previous refinement step
      s.rnorm2 = R2;
      s.ynorm2 = Y2;
      // A healthy FP32 inner solve cuts the residual by about its tolerance;
      // one that gains less than a factor 10 in norm no longer resolves the
      // remaining error (FP32 rounding of Q and Omega), and the refinement
      // continues with FP64 inner solves.  Once those stop halving the norm,
      // refinement has reached what the arithmetic allows.
      const bool weak = step > 0 && !(R2 < 1e-2 * prev);
      const bool stalled = step > 0 && !(R2 < 0.25 * prev);
      if (!(R2 > tol * tol * Y2)) {
        ost[s_idx] = ST_CONVERGED;
        s.status = ST_IDLE;
      } else if (!s.esc && weak && !last_step && isfinite(R2)) {
        s.esc = 1;
        s.status = ST_ACTIVE;
        s_any = 1;
      } else if (stalled) {
        // the last correction is kept
        ost[s_idx] = ST_STAGNATED;
        s.status = ST_IDLE;
      } else if (last_step || !isfinite(R2)) {
        ost[s_idx] = ST_MAXITER;
        s.status = ST_IDLE;
      } else {
        s.status = ST_ACTIVE;
        s_any = 1;
      }
      // an FP64 continuation solve aims a little below the outer target
      if (s.status == ST_ACTIVE && s.esc)
        s.itol = fmin(1e-3, fmax(1e-15, 0.1 * tol * sqrt(Y2 / R2)));
    }
    __syncthreads();
  }
  __syncthreads();
  if (threadIdx.x == 0) inst_active[b] = s_any;
  for (int k = threadIdx.x; k < K; k += NT) {
    if (ost[in.rhs0 + k] != ST_ACTIVE && st[in.rhs0 + k].status == ST_ACTIVE)
      st[in.rhs0 + k].status = ST_IDLE;
  }
}

// u += du for the rhs of the inner solve (FP32 or FP64 correction), over one tile.
template <typename T>
__global__ void __launch_bounds__(NT)
k_update_u(const InstDesc* __restrict__ insts, const TileDesc* __restrict__ tiles,
           const int* __restrict__ inst_active, const RhsState* __restrict__ st,
           const T* __restrict__ du, double* __restrict__ u) {
  const TileDesc tile = tiles[blockIdx.x];
  if (!inst_active[tile.inst]) return;
  const InstDesc in = insts[tile.inst];
  __shared__ int s_on[KMAX];
  if ((int)threadIdx.x < in.K) {
    const int s = st[in.rhs0 + threadIdx.x].status;
    s_on[threadIdx.x] = (s != ST_IDLE && s != ST_RANK);
  }
  __syncthreads();
  const int64_t base = in.v_off + (int64_t)tile.row0 * in.G * in.K;
  const int cnt = tile.rows * in.G * in.K;
  for (int e = threadIdx.x; e < cnt; e += NT)
    if (s_on[e % in.K]) u[base + e] += (double)du[base + e];
}

__global__ void k_update_c(const InstDesc* __restrict__ insts, int B,
                           const RhsState* __restrict__ st, const double* __restrict__ dwc,
                           double* __restrict__ wc64) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const InstDesc in = insts[b];
  for (int e = threadIdx.x; e < in.kc * in.K; e += blockDim.x) {
    const int k = e % in.K;
    const int s = st[in.rhs0 + k].status;
    if (s != ST_IDLE && s != ST_RANK) wc64[in.c_off + e] += dwc[in.c_off + e];
  }
}

// ---------------------------------------------------------------------------
// gradients
// ---------------------------------------------------------------------------

// per tile: S[i][j] = sum_{t in tile, k} L[t][i][k] U[t][j][k]  (G x G partial)
__global__ void __launch_bounds__(NT)
k_grad_omega_part(const InstDesc* __restrict__ insts, const TileDesc* __restrict__ tiles,
                  const double* __restrict__ L, const double* __restrict__ U,
                  double* __restrict__ part) {
  const TileDesc tile = tiles[blockIdx.x];
  const InstDesc in = insts[tile.inst];
  const int G = in.G, K = in.K;
  const int64_t base = in.v_off + (int64_t)tile.row0 * G * K;
  double* out = part + tile.tp_off;
  for (int pr = threadIdx.x; pr < G * G; pr += NT) {
    const int i = pr / G, j = pr % G;
    double s = 0.0;
    for (int t = 0; t < tile.rows; ++t) {
      const double* lr = L + base + ((int64_t)t * G + i) * K;
      const double* ur = U + base + ((int64_t)t * G + j) * K;
      for (int k = 0; k < K; ++k) s += lr[k] * ur[k];
    }
    out[pr] = s;
  }
}

__global__ void __launch_bounds__(NT)
k_grad_omega_reduce(const InstDesc* __restrict__ insts, const TileDesc* __restrict__ tiles,
                    const double* __restrict__ part, double* __restrict__ dOm) {
  const InstDesc in = insts[blockIdx.x];
  const int G = in.G;
  const int64_t base = tiles[in.tile0].tp_off;
  for (int pr = threadIdx.x; pr < G * G; pr += NT) {
    const int i = pr / G, j = pr % G;
    double sij = 0.0, sji = 0.0;
    for (int p = 0; p < in.ntiles; ++p) {
      sij += part[base + (int64_t)p * in.tp_stride + i * G + j];
      sji += part[base + (int64_t)p * in.tp_stride + j * G + i];
    }
    dOm[in.om_off + pr] = -0.5 * (sij + sji);
  }
}

// dX[t][c] = -sum_k ( L[t][i(c)][k] beta[c][k] + U[t][i(c)][k] lb[c][k] )
__global__ void __launch_bounds__(NT)
k_grad_x(const InstDesc* __restrict__ insts, const TileDesc* __restrict__ tiles,
         const int* __restrict__ colblk, const double* __restrict__ L,
         const double* __restrict__ U, const double* __restrict__ beta,
         const double* __restrict__ lb, double* __restrict__ dX) {
  const TileDesc tile = tiles[blockIdx.x];
  const InstDesc in = insts[tile.inst];
  const int G = in.G, K = in.K, n = in.n;
  const int* cb = colblk + in.col_off;
  for (int e = threadIdx.x; e < tile.rows * n; e += NT) {
    const int t = e / n, c = e % n;
    const int i = cb[c];
    const int64_t vr = in.v_off + ((int64_t)(tile.row0 + t) * G + i) * K;
    const int64_t br = in.b_off + (int64_t)c * K;
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += L[vr + k] * beta[br + k] + U[vr + k] * lb[br + k];
    dX[in.q_off + (int64_t)(tile.row0 + t) * n + c] = -s;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

static unsigned grid_for(int64_t count) {
  int64_t b = (count + 255) / 256;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

template <typename T>
hipError_t launch_fill(T* p, int64_t count, T v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(count)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}
template hipError_t launch_fill<double>(double*, int64_t, double, hipStream_t);
template hipError_t launch_fill<float>(float*, int64_t, float, hipStream_t);
template hipError_t launch_fill<int>(int*, int64_t, int, hipStream_t);

hipError_t launch_alpha(const InstDesc* insts, int B, const double* Om, double* alpha,
                        float* Om32, double* deq, hipStream_t s) {
  hipLaunchKernelGGL(k_alpha, dim3(B), dim3(256), 0, s, insts, B, Om, alpha, Om32, deq);
  return hipGetLastError();
}

hipError_t launch_state_init(const InstDesc* insts, int B, const int* rankflag,
                             int rank_extra_base, const int* rinst_index, RhsState* st,
                             int* inst_active, int* ost, hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(B), dim3(64), 0, s, insts, B, rankflag,
                     rank_extra_base, rinst_index, st, inst_active, ost, 0);
  return hipGetLastError();
}

hipError_t launch_activate(const InstDesc* insts, int B, const RhsState* st, int* inst_active,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_activate, dim3((B + 255) / 256), dim3(256), 0, s, insts, B, st,
                     inst_active);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy_tc(const InstDesc* insts, int B, const T* Tm, double* wc,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_copy_tc<T>, dim3(B), dim3(64), 0, s, insts, B, Tm, wc);
  return hipGetLastError();
}
template hipError_t launch_copy_tc<double>(const InstDesc*, int, const double*, double*,
                                           hipStream_t);
template hipError_t launch_copy_tc<float>(const InstDesc*, int, const float*, double*,
                                          hipStream_t);

hipError_t launch_outer_check(const InstDesc* insts, const BlockDesc* blks, const double* R,
                              int B, int* inst_active, RhsState* st,
                              int* ost, const double* rpart, const double* ypart,
                              const double* XtW, double xtw_sign, const double* h2,
                              const double* Rc,
                              const double* rvec, const double* beta, const double* wc,
                              double* rho0, double* rhoc, double tol, int step,
                              int last_step, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_check, dim3(B), dim3(NT), 0, s, insts, blks, R, inst_active, st,
                     ost,
                     rpart, ypart, XtW, xtw_sign, h2, Rc, rvec, beta, wc, rho0, rhoc, tol, step,
                     last_step);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_update_u(const InstDesc* insts, const TileDesc* tiles, int ntiles,
                           const int* inst_active, const RhsState* st, const T* du,
                           double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_update_u<T>, dim3(ntiles), dim3(NT), 0, s, insts, tiles, inst_active,
                     st, du, u);
  return hipGetLastError();
}
template hipError_t launch_update_u<float>(const InstDesc*, const TileDesc*, int, const int*,
                                           const RhsState*, const float*, double*, hipStream_t);
template hipError_t launch_update_u<double>(const InstDesc*, const TileDesc*, int, const int*,
                                            const RhsState*, const double*, double*,
                                            hipStream_t);

// beta (n x K per instance) into the projection layout ((n + k) x K per
// instance), so that the expansion half of a pass forms X beta.
__global__ void k_beta_to_t(const InstDesc* __restrict__ insts, int B,
                            const double* __restrict__ beta, double* __restrict__ Tm) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const InstDesc in = insts[b];
  for (int e = threadIdx.x; e < in.n * in.K; e += blockDim.x)
    Tm[in.t_off + e] = beta[in.b_off + e];
}

hipError_t launch_beta_to_t(const InstDesc* insts, int B, const double* beta, double* Tm,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_beta_to_t, dim3(B), dim3(NT), 0, s, insts, B, beta, Tm);
  return hipGetLastError();
}

// G x G identity per instance (the Omega of a pass that must not weight W).
__global__ void k_eye(const InstDesc* __restrict__ insts, int B, double* __restrict__ E) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const InstDesc in = insts[b];
  for (int e = threadIdx.x; e < in.G * in.G; e += blockDim.x)
    E[in.om_off + e] = (e / in.G == e % in.G) ? 1.0 : 0.0;
}

hipError_t launch_eye(const InstDesc* insts, int B, double* E, hipStream_t s) {
  hipLaunchKernelGGL(k_eye, dim3(B), dim3(NT), 0, s, insts, B, E);
  return hipGetLastError();
}

// Mixed path: the rhs whose refinement continues take part in the next inner
// solve of precision `want` (0 = FP32, 1 = FP64); -2 selects all of them (the
// refinement residual), -1 only sets the instance activity.
__global__ void k_select_inner(const InstDesc* __restrict__ insts, int B,
                               RhsState* __restrict__ st, const int* __restrict__ ost,
                               int* __restrict__ inst_active, int want) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const InstDesc in = insts[b];
  int any = 0;
  for (int k = 0; k < in.K; ++k) {
    RhsState& s = st[in.rhs0 + k];
    const bool on = ost[in.rhs0 + k] == ST_ACTIVE && (want < 0 || s.esc == want);
    if (want != -1 && s.status != ST_RANK) s.status = on ? ST_ACTIVE : ST_IDLE;
    any |= on;
  }
  inst_active[b] = any;
}

hipError_t launch_select_inner(const InstDesc* insts, int B, RhsState* st, const int* ost,
                               int* inst_active, int want, hipStream_t s) {
  hipLaunchKernelGGL(k_select_inner, dim3((B + 63) / 64), dim3(64), 0, s, insts, B, st, ost,
                     inst_active, want);
  return hipGetLastError();
}

hipError_t launch_update_c(const InstDesc* insts, int B, const RhsState* st,
                           const double* dwc, double* wc64, hipStream_t s) {
  hipLaunchKernelGGL(k_update_c, dim3(B), dim3(64), 0, s, insts, B, st, dwc, wc64);
  return hipGetLastError();
}

hipError_t launch_grad(const InstDesc* insts, const TileDesc* tiles, int ntiles, int B,
                       const int* colblk, const double* L, const double* U,
                       const double* beta, const double* lb, double* part, double* dOm,
                       double* dX, hipStream_t s) {
  if (dOm) {
    hipLaunchKernelGGL(k_grad_omega_part, dim3(ntiles), dim3(NT), 0, s, insts, tiles, L, U,
                       part);
    hipLaunchKernelGGL(k_grad_omega_reduce, dim3(B), dim3(NT), 0, s, insts, tiles, part, dOm);
  }
  if (dX)
    hipLaunchKernelGGL(k_grad_x, dim3(ntiles), dim3(NT), 0, s, insts, tiles, colblk, L, U,
                       beta, lb, dX);
  return hipGetLastError();
}

}  // namespace glm
