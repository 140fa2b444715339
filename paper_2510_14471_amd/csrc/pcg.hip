// PCG-Aug iteration kernels for batched SUR GLS (gfx950).
//
// The iteration is Algorithm "The PCG-Aug method" with D = alpha I, carrying
// g_i = Pi r_i (Pi X = 0 removes the X v_i term from its update and
// Pi D Pi = Pi gives c_i = alpha ||g_i||^2):
//
//   u   <- g + mu u                          (u_{i+1} = Pi r_{i+1} + mu_i u_i)
//   B   <- U Omega                           (Sigma u = vec(U Omega), SUR section)
//   d   <- u . B ;  T_i <- Q_i^T B_i          projection pass A (reduction over rows)
//   lambda = c / d
//   g   <- g - (lambda/alpha)(B_i - Q_i T_i) projection pass B (OLS residual)
//   w   <- w - lambda u
//   c'  <- alpha ||g||^2 ; mu = c'/c
//
// Work decomposition: every instance is cut into row tiles; one workgroup
// streams one tile in LDS-staged sub-tiles of `rs` rows.  A tile's vector
// slab is contiguous (rows x G x K, K innermost) and so is its Q slab
// (rows x n), so every global access is a contiguous sweep.  Cross-tile sums
// (Q^T B, d, c) are written as per-tile partials and reduced by small
// follow-up kernels: no atomics, deterministic results.
#include "glm_internal.h"

#include <cmath>

namespace glm {

namespace {

enum : int { A_ITER = 0, A_RHS = 1 };
enum : int { B_ITER = 0, B_INIT = 1, B_EXPAND = 2 };

template <typename T>
struct VecArgs {
  const InstDesc* __restrict__ insts;
  const TileDesc* __restrict__ tiles;
  const BlockDesc* __restrict__ blks;
  const int* __restrict__ colblk;
  const int* __restrict__ inst_active;
  const T* __restrict__ Q;        // Q (or X) of the precision of the pass
  const T* __restrict__ Om;       // Omega of the precision of the pass
  const double* __restrict__ alpha;
  const double* __restrict__ deq;  // per-block D scalars, or null (D = alpha I)
  const RhsState* __restrict__ st;
  const T* __restrict__ y;        // right-hand side (A_RHS, B_INIT)
  T* w;
  T* g;
  T* u;
  const T* __restrict__ Tm;       // reduced projections (pass B)
  T* Tpart;                       // per-tile projection partials (pass A)
  double* dpart;                  // per-tile d partials   [tile][KMAX]
  double* cpart;                  // per-tile c partials   [tile][KMAX]
  unsigned long long* bytes;      // algorithmic byte counter or nullptr
  int w_nonzero;                  // w holds a nonzero start (A_RHS, B_INIT)
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Reduce acc[k] (k < KC) over the workgroup and write the sums to out[k] for k < K.
template <int KC>
__device__ void wg_reduce_store(double (&acc)[KC], int K, double* out, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    double s = wave_sum(acc[k]);
    if (lane == 0) red[k * (NT / 64) + wv] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < K) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) s += red[threadIdx.x * (NT / 64) + q];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Bs[t][j][k] = sum_i Us[t][i][k] Omega[i][j], units (t, j).  FORM: OM_PLAIN,
// OM_DOT (also accumulates the d partials u . B), OM_RHS (Bs = y - U Omega).
enum : int { OM_PLAIN = 0, OM_DOT = 1, OM_RHS = 2 };
template <typename T, int KC, int FORM>
__device__ void omega_apply(const T* __restrict__ Us, T* __restrict__ Bs,
                            const T* __restrict__ Om, int nr, int G, int K,
                            bool have_u, const T* __restrict__ ysrc,
                            double (&dacc)[KC]) {
  for (int unit = threadIdx.x; unit < nr * G; unit += NT) {
    const int t = unit / G, j = unit - t * G;
    T acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = T(0);
    if (have_u) {
      const T* urow = Us + (size_t)t * G * K;
      for (int i = 0; i < G; ++i) {
        const T om = Om[i * G + j];
#pragma unroll
        for (int k = 0; k < KC; ++k)
          if (k < K) acc[k] += urow[i * K + k] * om;
      }
    }
    T* brow = Bs + ((size_t)t * G + j) * K;
    if (FORM == OM_RHS) {
      if (ysrc) {
        const T* yrow = ysrc + ((size_t)t * G + j) * K;
#pragma unroll
        for (int k = 0; k < KC; ++k)
          if (k < K) brow[k] = yrow[k] - acc[k];
      } else {
#pragma unroll
        for (int k = 0; k < KC; ++k)
          if (k < K) brow[k] = -acc[k];
      }
    } else if (FORM == OM_DOT) {
      const T* urow = Us + ((size_t)t * G + j) * K;
#pragma unroll
      for (int k = 0; k < KC; ++k)
        if (k < K) {
          brow[k] = acc[k];
          dacc[k] += (double)urow[k] * (double)acc[k];
        }
    } else {
#pragma unroll
      for (int k = 0; k < KC; ++k)
        if (k < K) brow[k] = acc[k];
    }
  }
}


// sums[k] = sum over the instance's tiles of part[tile][k] (k < K), computed by
// all NT threads of the workgroup: 16 lanes per k, a strided loop over tiles
// and an LDS tree over the 16 lanes.  Called by every thread.
__device__ void sum_tile_partials(const double* __restrict__ part, int tile0, int ntiles,
                                  int K, double* __restrict__ red, double* __restrict__ sums) {
  const int k = threadIdx.x % KMAX, g = threadIdx.x / KMAX;   // 16 groups of 16
  double s = 0.0;
  if (k < K)
    for (int p = g; p < ntiles; p += NT / KMAX) s += part[(int64_t)(tile0 + p) * KMAX + k];
  red[threadIdx.x] = s;
  __syncthreads();
  if ((int)threadIdx.x < K) {
    double t = 0.0;
    for (int q = 0; q < NT / KMAX; ++q) t += red[q * KMAX + threadIdx.x];
    sums[threadIdx.x] = t;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// projection pass A: T partials of Q^T B (ITER: B = Sigma u after u <- g + mu u;
// RHS: B = y - Sigma w) and the d partials.
// ---------------------------------------------------------------------------
template <typename T, int KC, int SL, int MODE>
__global__ void __launch_bounds__(NT)
k_pass_a(VecArgs<T> a) {
  const TileDesc tile = a.tiles[blockIdx.x];
  if (!a.inst_active[tile.inst]) return;
  const InstDesc in = a.insts[tile.inst];
  const int G = in.G, K = in.K, n = in.n, rs = rows_of<T>(in);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Us = reinterpret_cast<T*>(smem_raw);
  T* Bs = Us + (size_t)rs * G * K;
  __shared__ double s_mu[KMAX];
  __shared__ int s_act[KMAX], s_first[KMAX];
  __shared__ double red[KC * (NT / 64)];
  if ((int)threadIdx.x < K) {
    const RhsState s = a.st[in.rhs0 + threadIdx.x];
    s_act[threadIdx.x] = (s.status == ST_ACTIVE);
    s_first[threadIdx.x] = (s.iters == 0);
    s_mu[threadIdx.x] = s.mu;
  }
  __syncthreads();
  const T* __restrict__ Om = a.Om + in.om_off;
  const T* __restrict__ Qb = a.Q + in.q_off;
  const int* __restrict__ cb = a.colblk + in.col_off;

  T tacc[SL][KC];
#pragma unroll
  for (int s = 0; s < SL; ++s)
#pragma unroll
    for (int k = 0; k < KC; ++k) tacc[s][k] = T(0);
  double dacc[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) dacc[k] = 0.0;
  int kact = 0;
  for (int k = 0; k < K; ++k) kact += s_act[k];

  for (int sub = 0; sub < tile.rows; sub += rs) {
    const int nr = min(rs, tile.rows - sub);
    const int row = tile.row0 + sub;
    const int64_t base = in.v_off + (int64_t)row * G * K;
    const int cnt = nr * G * K;
    // step 1: stage u (ITER: u <- g + mu u) or w (RHS)
    if (MODE == A_ITER) {
      for (int e = threadIdx.x; e < cnt; e += NT) {
        const int k = e % K;
        const T uo = a.u[base + e];
        T nu = uo;
        if (s_act[k]) {
          const T gg = a.g[base + e];
          nu = s_first[k] ? gg : gg + (T)s_mu[k] * uo;
          a.u[base + e] = nu;
        }
        Us[e] = nu;
      }
    } else if (a.w_nonzero) {
      for (int e = threadIdx.x; e < cnt; e += NT) Us[e] = a.w[base + e];
    }
    __syncthreads();
    // step 2: B = U Omega (ITER, with the d partials) or y - W Omega (RHS)
    if (MODE == A_ITER)
      omega_apply<T, KC, OM_DOT>(Us, Bs, Om, nr, G, K, true, nullptr, dacc);
    else
      omega_apply<T, KC, OM_RHS>(Us, Bs, Om, nr, G, K, a.w_nonzero != 0,
                                 a.y ? a.y + base : nullptr, dacc);
    __syncthreads();
    // step 3: column-wise Q^T B partial sums (thread c owns columns c + s*NT)
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int c = threadIdx.x + s * NT;
      if (c < n) {
        const int bi = cb[c];
        const T* qcol = Qb + (int64_t)row * n + c;
        for (int t = 0; t < nr; ++t) {
          const T q = qcol[(int64_t)t * n];
          const T* brow = Bs + ((size_t)t * G + bi) * K;
#pragma unroll
          for (int k = 0; k < KC; ++k)
            if (k < K) tacc[s][k] += q * brow[k];
        }
      }
    }
    __syncthreads();
  }
  // flush the tile's partials
  T* tp = a.Tpart + tile.tp_off;
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    const int c = threadIdx.x + s * NT;
    if (c < n) {
#pragma unroll
      for (int k = 0; k < KC; ++k)
        if (k < K) tp[(int64_t)c * K + k] = tacc[s][k];
    }
  }
  if (MODE == A_ITER) wg_reduce_store<KC>(dacc, K, a.dpart + (int64_t)blockIdx.x * KMAX, red);
  if (a.bytes && threadIdx.x == 0) {
    const unsigned long long bq = (unsigned long long)tile.rows * n * sizeof(T);
    const unsigned long long bv = 3ull * tile.rows * G * kact * sizeof(T);
    atomicAdd(a.bytes, bq + bv);
  }
}

// ---------------------------------------------------------------------------
// projection pass B: OLS residual B_i - Q_i T_i and the vector updates.
// ---------------------------------------------------------------------------
template <typename T, int KC, int MODE>
__global__ void __launch_bounds__(NT)
k_pass_b(VecArgs<T> a) {
  const TileDesc tile = a.tiles[blockIdx.x];
  if (!a.inst_active[tile.inst]) return;
  const InstDesc in = a.insts[tile.inst];
  const int G = in.G, K = in.K, n = in.n, rs = rows_of<T>(in);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Us = reinterpret_cast<T*>(smem_raw);
  T* Bs = Us + (size_t)rs * G * K;
  __shared__ double s_lam[KMAX];
  __shared__ int s_act[KMAX];
  __shared__ double red[KC * (NT / 64)];
  __shared__ double s_ialpha;
  if ((int)threadIdx.x < K) {
    const RhsState s = a.st[in.rhs0 + threadIdx.x];
    s_act[threadIdx.x] = (s.status == ST_ACTIVE);
    s_lam[threadIdx.x] = s.lam;
  }
  if (threadIdx.x == 0) s_ialpha = 1.0 / a.alpha[tile.inst];
  __syncthreads();
  const T* __restrict__ Om = a.Om + in.om_off;
  const T* __restrict__ Qb = a.Q + in.q_off;
  const T* __restrict__ Tb = a.Tm + in.t_off;
  const BlockDesc* __restrict__ bd = a.blks + in.blk0;
  const T ialpha = (T)s_ialpha;
  double cacc[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) cacc[k] = 0.0;
  int kact = 0;
  for (int k = 0; k < K; ++k) kact += s_act[k];

  for (int sub = 0; sub < tile.rows; sub += rs) {
    const int nr = min(rs, tile.rows - sub);
    const int row = tile.row0 + sub;
    const int64_t base = in.v_off + (int64_t)row * G * K;
    const int cnt = nr * G * K;
    if (MODE != B_EXPAND) {
      if (MODE == B_ITER) {
        for (int e = threadIdx.x; e < cnt; e += NT) Us[e] = a.u[base + e];
      } else if (a.w_nonzero) {
        for (int e = threadIdx.x; e < cnt; e += NT) Us[e] = a.w[base + e];
      }
      __syncthreads();
      if (MODE == B_ITER)
        omega_apply<T, KC, OM_PLAIN>(Us, Bs, Om, nr, G, K, true, nullptr, cacc);
      else
        omega_apply<T, KC, OM_RHS>(Us, Bs, Om, nr, G, K, a.w_nonzero != 0,
                                   a.y ? a.y + base : nullptr, cacc);
      __syncthreads();
    }
    // units (t, i): the block-i row of Q T, then the elementwise update
    for (int unit = threadIdx.x; unit < nr * G; unit += NT) {
      const int t = unit / G, i = unit - t * G;
      const BlockDesc b = bd[i];
      T qt[KC];
#pragma unroll
      for (int k = 0; k < KC; ++k) qt[k] = T(0);
      const T* qrow = Qb + (int64_t)(row + t) * n + b.col;
      const T* trow = Tb + (int64_t)b.col * K;
      for (int c = 0; c < b.ni; ++c) {
        const T q = qrow[c];
#pragma unroll
        for (int k = 0; k < KC; ++k)
          if (k < K) qt[k] += q * trow[c * K + k];
      }
      const int64_t e0 = base + ((int64_t)t * G + i) * K;
      const int l0 = (t * G + i) * K;
      // D = diag(d) (x) I_M: Pi_i = P_i / d_i, and c = sum_i d_i ||g_i||^2 is
      // accumulated as alpha * sum_i (d_i / alpha) ||g_i||^2
      T ia = ialpha;
      double wgt = 1.0;
      if (a.deq) {
        const double di = a.deq[in.blk0 + i];
        ia = (T)(1.0 / di);
        wgt = di * s_ialpha;
      }
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        if (k < K && s_act[k]) {
          if (MODE == B_ITER) {
            const T lam = (T)s_lam[k];
            const T gg = a.g[e0 + k] - lam * ia * (Bs[l0 + k] - qt[k]);
            a.g[e0 + k] = gg;
            a.w[e0 + k] = a.w[e0 + k] - lam * Us[l0 + k];
            cacc[k] += wgt * (double)gg * (double)gg;
          } else if (MODE == B_INIT) {
            const T gg = -(Bs[l0 + k] - qt[k]) * ia;
            a.g[e0 + k] = gg;
            cacc[k] += wgt * (double)gg * (double)gg;
          } else {
            a.w[e0 + k] = qt[k];
          }
        }
      }
    }
    __syncthreads();
  }
  if (MODE != B_EXPAND)
    wg_reduce_store<KC>(cacc, K, a.cpart + (int64_t)blockIdx.x * KMAX, red);
  if (MODE == B_ITER && a.bytes && threadIdx.x == 0) {
    const unsigned long long bq = (unsigned long long)tile.rows * n * sizeof(T);
    const unsigned long long bv = 3ull * tile.rows * G * kact * sizeof(T);  // Q + read w, write g, w
    atomicAdd(a.bytes, bq + bv);
  }
}

// ---------------------------------------------------------------------------
// reductions and scalar steps
// ---------------------------------------------------------------------------

// T[c][k] = sum over the instance's tiles of the partials (n x K each).
template <typename T>
__global__ void __launch_bounds__(NT)
k_reduce_t(const InstDesc* __restrict__ insts, const TileDesc* __restrict__ tiles,
           const int* __restrict__ inst_active, const RedChunk* __restrict__ chunks,
           const T* __restrict__ Tpart, T* __restrict__ Tm, int use_rpar) {
  const RedChunk ch = chunks[blockIdx.x];
  if (!inst_active[ch.inst]) return;
  const InstDesc in = insts[ch.inst];
  const int nk = in.n * in.K;
  const int pr = ch.p0 + threadIdx.x;
  if (pr >= nk) return;
  const int64_t base = tiles[in.tile0].tp_off;
  const int slots = use_rpar ? tps_of<T>(in) : 1;    // row-group partials inside a tile
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const int64_t st4 = in.tp_stride;
  for (int r = 0; r < slots; ++r) {
    const T* src = Tpart + base + (int64_t)r * nk + pr;
    int p = 0;
    for (; p + 4 <= in.ntiles; p += 4) {
      s0 += (double)src[(int64_t)p * st4];
      s1 += (double)src[(int64_t)(p + 1) * st4];
      s2 += (double)src[(int64_t)(p + 2) * st4];
      s3 += (double)src[(int64_t)(p + 3) * st4];
    }
    for (; p < in.ntiles; ++p) s0 += (double)src[(int64_t)p * st4];
  }
  Tm[in.t_off + pr] = (T)((s0 + s1) + (s2 + s3));
}

// Per instance: d (ITER) -> lambda and breakdown; restriction rows of the
// projection (0 in ITER, the restriction right-hand side in RHS mode) and the
// rank-k correction  T <- T - N (N^T T)  that turns the blockwise projection
// into the projection onto the range of [X; R_c] (eq. rglm1m).
template <typename T>
__global__ void __launch_bounds__(NT)
k_scalar_a(const InstDesc* __restrict__ insts, const TileDesc* __restrict__ tiles,
           const int* __restrict__ inst_active, RhsState* __restrict__ st,
           const double* __restrict__ dpart, T* __restrict__ Tm,
           const double* __restrict__ Nb, const double* __restrict__ rvec,
           int mode_iter, int do_d) {
  const int b = blockIdx.x;
  if (!inst_active[b]) return;
  const InstDesc in = insts[b];
  const int K = in.K;
  __shared__ double red_s[NT];
  __shared__ double dsum[KMAX];
  if (do_d) sum_tile_partials(dpart, in.tile0, in.ntiles, K, red_s, dsum);
  if (do_d && (int)threadIdx.x < K) {
    const int k = threadIdx.x;
    RhsState& s = st[in.rhs0 + k];
    if (s.status == ST_ACTIVE) {
      const double d = dsum[k];
      s.d = d;
      if (!(d > 0.0) || !isfinite(d) || !isfinite(s.c)) {
        s.status = ST_BREAKDOWN;
        s.lam = 0.0;
      } else {
        s.lam = s.c / d;
      }
    }
  }
  const int kc = in.kc;
  if (kc == 0) return;
  const int n = in.n, nn = n + kc;
  T* Tb = Tm + in.t_off;
  // restriction rows of the projected vector
  for (int e = threadIdx.x; e < kc * K; e += NT) {
    const int q = e / K, k = e % K;
    Tb[(int64_t)(n + q) * K + k] = mode_iter ? T(0) : (rvec ? (T)rvec[in.c_off + e] : T(0));
  }
  __syncthreads();
  const double* N = Nb + in.nb_off;
  __shared__ double P[64 * KMAX];     // N^T T (kc <= 64)
  for (int e = threadIdx.x; e < kc * K; e += NT) P[e] = 0.0;
  __syncthreads();
  // each wave takes (q, k) pairs: P[q][k] = sum_r N[r][q] T[r][k]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int e = wv; e < kc * K; e += NT / 64) {
    const int q = e / K, k = e % K;
    double s = 0.0;
    for (int r = lane; r < nn; r += 64) s += N[(int64_t)r * kc + q] * (double)Tb[(int64_t)r * K + k];
    s = wave_sum(s);
    if (lane == 0) P[e] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nn * K; e += NT) {
    const int r = e / K, k = e % K;
    double s = 0.0;
    for (int q = 0; q < kc; ++q) s += N[(int64_t)r * kc + q] * P[q * K + k];
    Tb[e] = (T)((double)Tb[e] - s);
  }
}

// Per instance (one wave): c' from the partials, the restriction rows of g, u, w,
// stopping tests, mu; instance activity and active count for host polling.
__global__ void k_scalar_b(const InstDesc* __restrict__ insts, int* __restrict__ inst_active,
                           int* __restrict__ inst_count, RhsState* __restrict__ st,
                           const double* __restrict__ cpart, const double* __restrict__ alpha,
                           const void* __restrict__ Tm_raw, int t_is_double,
                           double* __restrict__ gc, double* __restrict__ uc,
                           double* __restrict__ wc, const double* __restrict__ rvec,
                           int mode_iter, double tol, int stall, int maxit_cap) {
  const int b = blockIdx.x;
  if (!inst_active[b]) {
    if (threadIdx.x == 0) inst_count[b] = 0;
    return;
  }
  const InstDesc in = insts[b];
  const int K = in.K, kc = in.kc, n = in.n;
  const double al = alpha[b];
  const int maxit = (maxit_cap > 0 && maxit_cap < in.maxit) ? maxit_cap : in.maxit;
  __shared__ double red_s[NT];
  __shared__ double csum[KMAX];
  __shared__ int s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  sum_tile_partials(cpart, in.tile0, in.ntiles, K, red_s, csum);
  int act = 0;
  if ((int)threadIdx.x < K) {
    const int k = threadIdx.x;
    RhsState& s = st[in.rhs0 + k];
    if (s.status == ST_ACTIVE) {
      double cp = csum[k];
      for (int q = 0; q < kc; ++q) {
        const int64_t ti = in.t_off + (int64_t)(n + q) * K + k;
        const double tq = t_is_double ? ((const double*)Tm_raw)[ti]
                                      : (double)((const float*)Tm_raw)[ti];
        const int64_t ci = in.c_off + (int64_t)q * K + k;
        double gq;
        if (mode_iter) {
          gq = gc[ci] + s.lam / al * tq;
          wc[ci] -= s.lam * uc[ci];
        } else {
          const double vq = rvec ? rvec[ci] : 0.0;
          gq = -(vq - tq) / al;
        }
        gc[ci] = gq;
        cp += gq * gq;
      }
      const double cn = al * cp;
      if (mode_iter) {
        s.iters += 1;
        s.total_iters += 1;
        if (!isfinite(cn)) {
          s.status = ST_BREAKDOWN;
        } else if (sqrt(cn / s.c1) <= (s.itol > 0.0 ? s.itol : tol)) {
          s.status = ST_CONVERGED;
        } else {
          // progress = c at least halves relative to the reference value;
          // `stall` iterations without progress end the solve (stagnation)
          if (cn < 0.5 * s.cmin) {
            s.cmin = cn;
            s.since = 0;
          } else if (++s.since >= stall) {
            s.status = ST_STAGNATED;
          }
          if (s.status == ST_ACTIVE && s.iters >= maxit) s.status = ST_MAXITER;
        }
        s.mu = cn / s.c;
        s.c = cn;
        if (s.status == ST_ACTIVE)
          for (int q = 0; q < kc; ++q) {
            const int64_t ci = in.c_off + (int64_t)q * K + k;
            uc[ci] = gc[ci] + s.mu * uc[ci];
          }
      } else {
        s.c = cn;
        s.c1 = cn;
        s.cmin = cn;
        s.mu = 0.0;
        s.since = 0;
        s.iters = 0;
        for (int q = 0; q < kc; ++q) {
          const int64_t ci = in.c_off + (int64_t)q * K + k;
          uc[ci] = gc[ci];
        }
        if (!(cn > 0.0)) s.status = (cn == 0.0) ? ST_CONVERGED : ST_BREAKDOWN;
        if (s.status == ST_ACTIVE && maxit <= 0) s.status = ST_MAXITER;
      }
    }
    act = (s.status == ST_ACTIVE);
  }
  if (act) atomicAdd(&s_cnt, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    inst_active[b] = s_cnt > 0;
    inst_count[b] = s_cnt;
  }
}

__global__ void k_count(const int* __restrict__ inst_count, int B, int* __restrict__ out) {
  __shared__ int part[NT];
  int s = 0;
  for (int b = threadIdx.x; b < B; b += NT) s += inst_count[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

// Triangular solves per (block, rhs).  UPPER: x = R^-1 t (beta from the
// projection); LOWER: x = R^-T h (the start w_1 = X* h of a nonzero lower
// right-hand side).  ADD accumulates into a double destination.
template <typename TS, typename TD, bool UPPER, bool ADD>
__global__ void k_trisolve(const InstDesc* __restrict__ insts,
                           const BlockDesc* __restrict__ blks, int nblk,
                           const int* __restrict__ inst_active,
                           const RhsState* __restrict__ st, int need_active,
                           const double* __restrict__ R, const TS* __restrict__ src,
                           int src_is_t, TD* __restrict__ dst, int dst_is_t) {
  const int job = blockIdx.x * blockDim.x + threadIdx.x;
  if (job >= nblk * KMAX) return;
  const int bi = job / KMAX, k = job % KMAX;
  const BlockDesc bd = blks[bi];
  const InstDesc in = insts[bd.inst];
  if (k >= in.K) return;
  if (need_active) {
    if (!inst_active[bd.inst]) return;
    const int s = st[in.rhs0 + k].status;
    if (s == ST_IDLE || s == ST_RANK) return;
  }
  const double* Ri = R + bd.r_off;
  const int ni = bd.ni, K = in.K;
  const int64_t so = (src_is_t ? in.t_off : in.b_off) + (int64_t)bd.col * K + k;
  const int64_t dofs = (dst_is_t ? in.t_off : in.b_off) + (int64_t)bd.col * K + k;
  double x[QR_NMAX];
  if (UPPER) {
    for (int a = ni - 1; a >= 0; --a) {
      double s = (double)src[so + (int64_t)a * K];
      for (int c = a + 1; c < ni; ++c) s -= Ri[a * ni + c] * x[c];
      x[a] = s / Ri[a * ni + a];
    }
  } else {
    for (int a = 0; a < ni; ++a) {
      double s = (double)src[so + (int64_t)a * K];
      for (int c = 0; c < a; ++c) s -= Ri[c * ni + a] * x[c];
      x[a] = s / Ri[a * ni + a];
    }
  }
  for (int a = 0; a < ni; ++a) {
    if (ADD)
      dst[dofs + (int64_t)a * K] = (TD)((double)dst[dofs + (int64_t)a * K] + x[a]);
    else
      dst[dofs + (int64_t)a * K] = (TD)x[a];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <typename T>
static VecArgs<T> to_args(const PassLaunch<T>& p) {
  VecArgs<T> a;
  a.insts = p.insts;
  a.tiles = p.tiles;
  a.blks = p.blks;
  a.colblk = p.colblk;
  a.inst_active = p.inst_active;
  a.Q = p.Q;
  a.Om = p.Om;
  a.alpha = p.alpha;
  a.deq = p.deq;
  a.st = p.st;
  a.y = p.y;
  a.w = p.w;
  a.g = p.g;
  a.u = p.u;
  a.Tm = p.Tm;
  a.Tpart = p.Tpart;
  a.dpart = p.dpart;
  a.cpart = p.cpart;
  a.bytes = p.bytes;
  a.w_nonzero = p.w_nonzero;
  return a;
}

#define GLM_LAUNCH_A(KCV, SLV)                                                          \
  if (p.kc_t == KCV && p.sl == SLV) {                                                   \
    if (mode == A_ITER)                                                                 \
      hipLaunchKernelGGL((k_pass_a<T, KCV, SLV, A_ITER>), dim3(p.ntiles), dim3(NT),     \
                         p.lds, s, a);                                                  \
    else                                                                                \
      hipLaunchKernelGGL((k_pass_a<T, KCV, SLV, A_RHS>), dim3(p.ntiles), dim3(NT),      \
                         p.lds, s, a);                                                  \
    return hipGetLastError();                                                           \
  }

template <typename T>
hipError_t launch_pass_a(const PassLaunch<T>& p, int mode, hipStream_t s) {
  VecArgs<T> a = to_args(p);
  GLM_LAUNCH_A(1, 1) GLM_LAUNCH_A(1, 2) GLM_LAUNCH_A(1, 3) GLM_LAUNCH_A(1, 4) GLM_LAUNCH_A(1, 8)
  GLM_LAUNCH_A(2, 1) GLM_LAUNCH_A(2, 2) GLM_LAUNCH_A(2, 3) GLM_LAUNCH_A(2, 4) GLM_LAUNCH_A(2, 8)
  GLM_LAUNCH_A(4, 1) GLM_LAUNCH_A(4, 2) GLM_LAUNCH_A(4, 3) GLM_LAUNCH_A(4, 4) GLM_LAUNCH_A(4, 8)
  GLM_LAUNCH_A(8, 1) GLM_LAUNCH_A(8, 2) GLM_LAUNCH_A(8, 3) GLM_LAUNCH_A(8, 4)
  GLM_LAUNCH_A(16, 1) GLM_LAUNCH_A(16, 2) GLM_LAUNCH_A(16, 3) GLM_LAUNCH_A(16, 4)
  return hipErrorInvalidValue;
}

#define GLM_LAUNCH_B(KCV)                                                                \
  if (p.kc_t == KCV) {                                                                   \
    if (mode == B_ITER)                                                                  \
      hipLaunchKernelGGL((k_pass_b<T, KCV, B_ITER>), dim3(p.ntiles), dim3(NT), p.lds, s, a); \
    else if (mode == B_INIT)                                                             \
      hipLaunchKernelGGL((k_pass_b<T, KCV, B_INIT>), dim3(p.ntiles), dim3(NT), p.lds, s, a); \
    else                                                                                 \
      hipLaunchKernelGGL((k_pass_b<T, KCV, B_EXPAND>), dim3(p.ntiles), dim3(NT), 0, s, a);   \
    return hipGetLastError();                                                            \
  }

template <typename T>
hipError_t launch_pass_b(const PassLaunch<T>& p, int mode, hipStream_t s) {
  VecArgs<T> a = to_args(p);
  GLM_LAUNCH_B(1) GLM_LAUNCH_B(2) GLM_LAUNCH_B(4) GLM_LAUNCH_B(8) GLM_LAUNCH_B(16)
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_reduce_t(const InstDesc* insts, const TileDesc* tiles, const int* inst_active,
                           const void* chunks, int nchunks, const T* Tpart, T* Tm,
                           int use_rpar, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_t<T>, dim3(nchunks), dim3(NT), 0, s, insts, tiles, inst_active,
                     (const RedChunk*)chunks, Tpart, Tm, use_rpar);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scalar_a(const InstDesc* insts, const TileDesc* tiles, const int* inst_active,
                           RhsState* st, const double* dpart, T* Tm, const double* Nb,
                           const double* rvec, int B, int mode_iter, int do_d,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_scalar_a<T>, dim3(B), dim3(NT), 0, s, insts, tiles, inst_active, st,
                     dpart, Tm, Nb, rvec, mode_iter, do_d);
  return hipGetLastError();
}

hipError_t launch_scalar_b(const InstDesc* insts, int* inst_active, int* inst_count,
                           RhsState* st, const double* cpart, const double* alpha,
                           const void* Tm, int t_is_double, double* gc, double* uc,
                           double* wc, const double* rvec, int B, int mode_iter,
                           double tol, int stall, int maxit_cap, hipStream_t s) {
  hipLaunchKernelGGL(k_scalar_b, dim3(B), dim3(NT), 0, s, insts, inst_active, inst_count, st,
                     cpart, alpha, Tm, t_is_double, gc, uc, wc, rvec, mode_iter, tol, stall,
                     maxit_cap);
  return hipGetLastError();
}

hipError_t launch_count(const int* inst_count, int B, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3(1), dim3(NT), 0, s, inst_count, B, out);
  return hipGetLastError();
}

template <typename TS, typename TD, bool UPPER, bool ADD>
hipError_t launch_trisolve(const InstDesc* insts, const BlockDesc* blks, int nblk,
                           const int* inst_active, const RhsState* st, int need_active,
                           const double* R, const TS* src, int src_is_t, TD* dst,
                           int dst_is_t, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  const int threads = 128;
  const int grid = (nblk * KMAX + threads - 1) / threads;
  hipLaunchKernelGGL((k_trisolve<TS, TD, UPPER, ADD>), dim3(grid), dim3(threads), 0, s, insts,
                     blks, nblk, inst_active, st, need_active, R, src, src_is_t, dst, dst_is_t);
  return hipGetLastError();
}

// explicit instantiations used by the host orchestration
template hipError_t launch_pass_a<double>(const PassLaunch<double>&, int, hipStream_t);
template hipError_t launch_pass_a<float>(const PassLaunch<float>&, int, hipStream_t);
template hipError_t launch_pass_b<double>(const PassLaunch<double>&, int, hipStream_t);
template hipError_t launch_pass_b<float>(const PassLaunch<float>&, int, hipStream_t);
template hipError_t launch_reduce_t<double>(const InstDesc*, const TileDesc*, const int*,
                                            const void*, int, const double*, double*, int,
                                            hipStream_t);
template hipError_t launch_reduce_t<float>(const InstDesc*, const TileDesc*, const int*,
                                           const void*, int, const float*, float*, int,
                                           hipStream_t);
template hipError_t launch_scalar_a<double>(const InstDesc*, const TileDesc*, const int*,
                                            RhsState*, const double*, double*, const double*,
                                            const double*, int, int, int, hipStream_t);
template hipError_t launch_scalar_a<float>(const InstDesc*, const TileDesc*, const int*,
                                           RhsState*, const double*, float*, const double*,
                                           const double*, int, int, int, hipStream_t);
template hipError_t launch_trisolve<double, double, true, false>(
    const InstDesc*, const BlockDesc*, int, const int*, const RhsState*, int, const double*,
    const double*, int, double*, int, hipStream_t);
template hipError_t launch_trisolve<double, double, true, true>(
    const InstDesc*, const BlockDesc*, int, const int*, const RhsState*, int, const double*,
    const double*, int, double*, int, hipStream_t);
template hipError_t launch_trisolve<float, double, true, true>(
    const InstDesc*, const BlockDesc*, int, const int*, const RhsState*, int, const double*,
    const float*, int, double*, int, hipStream_t);
template hipError_t launch_trisolve<double, double, false, false>(
    const InstDesc*, const BlockDesc*, int, const int*, const RhsState*, int, const double*,
    const double*, int, double*, int, hipStream_t);
template hipError_t launch_trisolve<double, float, false, false>(
    const InstDesc*, const BlockDesc*, int, const int*, const RhsState*, int, const double*,
    const double*, int, float*, int, hipStream_t);

}  // namespace glm
