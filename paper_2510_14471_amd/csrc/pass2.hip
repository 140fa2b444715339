// Projection passes of the PCG-Aug iteration, lane-per-(equation, rhs) form.
//
// A workgroup streams one row tile of one instance.  Each lane owns one
// (equation i, right-hand side k) pair (and with few pairs per row, one of
// `rpar` row groups), so for every row t it produces exactly the element
// (t, i, k) of the vectors: the lanes of a row cover its contiguous
// G x K slab and every global access is coalesced.  Per lane, in registers:
//   * column i of Omega  (B[t][i][k] = sum_j U[t][j][k] Omega[j][i]),
//   * the lane's slice T_i[., k] of the projection (pass A accumulates
//     Q_i^T B_i over the tile's rows; pass B holds the reduced T_i).
// Only the U slab of a sub-tile is staged in LDS, because B[t][i][k] needs
// the whole row U[t][., k].
//
//   pass A  ITER : u <- g + mu u ;  B = U Omega ;  d += u.B ;  T_i += Q_i^T B_i
//           RHS  : B = y - W Omega ;  T_i += Q_i^T B_i
//   pass B  ITER : g <- g - (lambda/alpha)(B_i - Q_i T_i) ;  w <- w - lambda u ;  c += g.g
//           INIT : g <- -(y - W Omega - Q T)/alpha ;  c += g.g
//           EXPAND: w <- Q T
#include "glm_internal.h"

#include <cmath>

namespace glm {

namespace {

enum : int { A_ITER = 0, A_RHS = 1 };
enum : int { B_ITER = 0, B_INIT = 1, B_EXPAND = 2 };

template <typename T>
struct Args2 {
  const InstDesc* __restrict__ insts;
  const TileDesc* __restrict__ tiles;
  const BlockDesc* __restrict__ blks;
  const int* __restrict__ inst_active;
  const T* __restrict__ Q;
  const T* __restrict__ Om;
  const double* __restrict__ alpha;
  const RhsState* __restrict__ st;
  const T* __restrict__ y;
  T* w;
  T* g;
  T* u;
  const T* __restrict__ Tm;
  T* Tpart;
  double* dpart;
  double* cpart;
  unsigned long long* bytes;
  int w_nonzero;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-k sum of a per-lane value over the lanes holding right-hand side k.
// red needs NTW doubles.  Lanes with lane_k < 0 contribute nothing.
template <int NTW>
__device__ void reduce_by_k(double v, int lane_k, int K, double* red, double* out) {
  red[threadIdx.x] = (lane_k >= 0) ? v : 0.0;
  __syncthreads();
  if ((int)threadIdx.x < K) {
    double s = 0.0;
    for (int l = threadIdx.x; l < NTW; l += K) s += red[l];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Register double buffering of one sub-tile's slabs.  The slabs (the Q rows
// and up to three vector slabs of the sub-tile) form one concatenated index
// space [0, total); thread tid owns the elements tid + q*NTW (q < EPT), loads
// them with every load in flight, and later writes them to LDS at the same
// index.  While one sub-tile is computed from LDS the next one is being
// loaded into registers.
template <typename T, int NTW, int EPT>
struct Stager {
  const T* s0;
  const T* s1;
  const T* s2;
  const T* s3;
  int b1, b2, b3;   // segment starts (segments past nseg start at `total`)
  int total;
  T reg[EPT];

  __device__ __forceinline__ void set(int ns, const T* p0, int l0, const T* p1, int l1, const T* p2, int l2,
                      const T* p3, int l3) {
    s0 = p0;
    s1 = p1;
    s2 = p2;
    s3 = p3;
    total = l0 + (ns > 1 ? l1 : 0) + (ns > 2 ? l2 : 0) + (ns > 3 ? l3 : 0);
    b1 = ns > 1 ? l0 : total;
    b2 = ns > 2 ? l0 + l1 : total;
    b3 = ns > 3 ? l0 + l1 + l2 : total;
  }
  // One predicated pass per segment: the base pointers stay wave-uniform and
  // every load of the sub-tile is issued before any of them is waited on.
  __device__ __forceinline__ void load() {
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * NTW;
      if (e < b1) reg[q] = s0[e];
    }
    if (b1 < total) {
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NTW;
        if (e >= b1 && e < b2) reg[q] = s1[e - b1];
      }
    }
    if (b2 < total) {
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NTW;
        if (e >= b2 && e < b3) reg[q] = s2[e - b2];
      }
    }
    if (b3 < total) {
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NTW;
        if (e >= b3 && e < total) reg[q] = s3[e - b3];
      }
    }
  }
  __device__ __forceinline__ void store(T* __restrict__ lds) const {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = threadIdx.x + q * NTW;
      if (e < total) lds[e] = reg[q];
    }
  }
};

template <typename T>
struct Ept {
  static constexpr int value = sizeof(T) == 8 ? 16 : 32;
};

template <typename T, int NTW, int GR, int NIM, int MODE>
__global__ void __launch_bounds__(NTW) k_pass_a2(Args2<T> a) {
  const TileDesc& tile = a.tiles[blockIdx.x];
  if (!a.inst_active[tile.inst]) return;
  const InstDesc& in = a.insts[tile.inst];
  const int G = in.G, K = in.K, n = in.n, rs = in.rs, P = G * K;
  const int rpar = in.rpar;
  constexpr int EPT = Ept<T>::value;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  T* Oms = lds + (size_t)NTW * EPT;           // Omega when it is not held in registers
  __shared__ double s_mu[KMAX];
  __shared__ int s_act[KMAX], s_first[KMAX];
  __shared__ double red[NTW];
  __shared__ double dsum[KMAX];
  if ((int)threadIdx.x < K) {
    const RhsState s = a.st[in.rhs0 + threadIdx.x];
    s_act[threadIdx.x] = (s.status == ST_ACTIVE);
    s_first[threadIdx.x] = (s.iters == 0);
    s_mu[threadIdx.x] = s.mu;
  }
  const T* __restrict__ Om = a.Om + in.om_off;
  if (GR == 0)
    for (int e = threadIdx.x; e < G * G; e += NTW) Oms[e] = Om[e];
  const int lane = threadIdx.x;
  const bool on = lane < rpar * P;
  const int r = on ? lane / P : 0;
  const int pr = on ? lane - r * P : 0;
  const int i = pr / K, k = pr - (pr / K) * K;
  const BlockDesc& bd = a.blks[in.blk0 + i];
  T om[GR > 0 ? GR : 1];
  if (GR > 0) {
#pragma unroll
    for (int j = 0; j < GR; ++j) om[j] = (j < G) ? Om[j * G + i] : T(0);
  }
  T tacc[NIM];
#pragma unroll
  for (int c = 0; c < NIM; ++c) tacc[c] = T(0);
  double dacc = 0.0;
  const T* __restrict__ Qg = a.Q + in.q_off;
  const bool have_w = (MODE == A_ITER) || a.w_nonzero;
  const bool have_y = (MODE == A_RHS) && a.y;

  Stager<T, NTW, EPT> sg;
#define GLM_SETUP_A(SUB)                                                                  \
  {                                                                                       \
    const int nr_ = min(rs, tile.rows - (SUB));                                           \
    const int row_ = tile.row0 + (SUB);                                                   \
    const int64_t base_ = in.v_off + (int64_t)row_ * P;                                   \
    const T* q0_ = Qg + (int64_t)row_ * n;                                                \
    if (MODE == A_ITER)                                                                   \
      sg.set(3, q0_, nr_ * n, a.u + base_, nr_ * P, a.g + base_, nr_ * P, nullptr, 0);    \
    else                                                                                  \
      sg.set(1 + (have_w ? 1 : 0) + (have_y ? 1 : 0), q0_, nr_ * n,                       \
             have_w ? a.w + base_ : a.y + base_, nr_ * P, a.y + base_, nr_ * P, nullptr, 0); \
  }
  GLM_SETUP_A(0)
  sg.load();
  __syncthreads();
  int kact = 0;
  for (int kk = 0; kk < K; ++kk) kact += s_act[kk];

  for (int sub = 0; sub < tile.rows; sub += rs) {
    const int nr = min(rs, tile.rows - sub);
    const int row = tile.row0 + sub;
    const int64_t base = in.v_off + (int64_t)row * P;
    T* Qs = lds;
    T* Us = lds + (size_t)nr * n;
    T* Ys = Us + (have_w ? (size_t)nr * P : 0);
    __syncthreads();                 // the previous sub-tile is no longer read
    sg.store(lds);
    __syncthreads();
    if (sub + rs < tile.rows) {      // prefetch the next sub-tile
      GLM_SETUP_A(sub + rs)
      sg.load();
    }
    if (MODE == A_ITER) {
      // u <- g + mu u on the staged slabs (g sits right after u)
      const T* Gs = Us + (size_t)nr * P;
      for (int e = threadIdx.x; e < nr * P; e += NTW) {
        const int kk = e % K;
        if (s_act[kk]) {
          const T nu = s_first[kk] ? Gs[e] : Gs[e] + (T)s_mu[kk] * Us[e];
          Us[e] = nu;
          a.u[base + e] = nu;
        }
      }
      __syncthreads();
    }
    if (on) {
#pragma unroll 1
      for (int t = r; t < nr; t += rpar) {
        const T* qrow = Qs + (size_t)t * n + bd.col;
        T b = T(0);
        const T* urow = Us + (size_t)t * P + k;
        if (have_w) {
          if (GR > 0) {
#pragma unroll
            for (int j = 0; j < GR; ++j)
              if (j < G) b += urow[j * K] * om[j];
          } else {
            for (int j = 0; j < G; ++j) b += urow[j * K] * Oms[j * G + i];
          }
        }
        if (MODE == A_ITER) {
          dacc += (double)urow[i * K] * (double)b;
        } else {
          b = (have_y ? Ys[(size_t)t * P + pr] : T(0)) - b;
        }
#pragma unroll
        for (int c = 0; c < NIM; ++c)
          if (c < bd.ni) tacc[c] += qrow[c] * b;
      }
    }
  }
  if (on) {
    T* tp = a.Tpart + tile.tp_off + (int64_t)r * n * K + (int64_t)bd.col * K + k;
#pragma unroll
    for (int c = 0; c < NIM; ++c)
      if (c < bd.ni) tp[(int64_t)c * K] = tacc[c];
  }
  if (MODE == A_ITER) {
    reduce_by_k<NTW>(dacc, on ? k : -1, K, red, dsum);
    if ((int)threadIdx.x < K) a.dpart[(int64_t)blockIdx.x * KMAX + threadIdx.x] = dsum[threadIdx.x];
  }
  if (a.bytes && threadIdx.x == 0 && MODE == A_ITER) {
    const unsigned long long bq = (unsigned long long)tile.rows * n * sizeof(T);
    const unsigned long long bv = 3ull * tile.rows * G * kact * sizeof(T);
    atomicAdd(a.bytes, bq + bv);
  }
}

template <typename T, int NTW, int GR, int NIM, int MODE>
__global__ void __launch_bounds__(NTW) k_pass_b2(Args2<T> a) {
  const TileDesc& tile = a.tiles[blockIdx.x];
  if (!a.inst_active[tile.inst]) return;
  const InstDesc& in = a.insts[tile.inst];
  const int G = in.G, K = in.K, n = in.n, rs = in.rs, P = G * K;
  const int rpar = in.rpar;
  constexpr int EPT = Ept<T>::value;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  T* Oms = lds + (size_t)NTW * EPT;
  __shared__ double s_lam[KMAX];
  __shared__ int s_act[KMAX];
  __shared__ double red[NTW];
  __shared__ double csum[KMAX];
  __shared__ double s_ialpha;
  if ((int)threadIdx.x < K) {
    const RhsState s = a.st[in.rhs0 + threadIdx.x];
    s_act[threadIdx.x] = (s.status == ST_ACTIVE);
    s_lam[threadIdx.x] = s.lam;
  }
  if (threadIdx.x == 0) s_ialpha = 1.0 / a.alpha[tile.inst];
  const T* __restrict__ Om = a.Om + in.om_off;
  if (GR == 0 && MODE != B_EXPAND)
    for (int e = threadIdx.x; e < G * G; e += NTW) Oms[e] = Om[e];
  const int lane = threadIdx.x;
  const bool on = lane < rpar * P;
  const int r = on ? lane / P : 0;
  const int pr = on ? lane - r * P : 0;
  const int i = pr / K, k = pr - (pr / K) * K;
  const BlockDesc& bd = a.blks[in.blk0 + i];
  T om[GR > 0 ? GR : 1];
  if (GR > 0 && MODE != B_EXPAND) {
#pragma unroll
    for (int j = 0; j < GR; ++j) om[j] = (j < G) ? Om[j * G + i] : T(0);
  }
  T treg[NIM];
  const T* tb = a.Tm + in.t_off + (int64_t)bd.col * K + k;
#pragma unroll
  for (int c = 0; c < NIM; ++c) treg[c] = (on && c < bd.ni) ? tb[(int64_t)c * K] : T(0);
  const T* __restrict__ Qg = a.Q + in.q_off;
  const bool have_u = (MODE == B_ITER) || (MODE == B_INIT && a.w_nonzero);
  const bool have_y = (MODE == B_INIT) && a.y;

  Stager<T, NTW, EPT> sg;
#define GLM_SETUP_B(SUB)                                                                  \
  {                                                                                       \
    const int nr_ = min(rs, tile.rows - (SUB));                                           \
    const int row_ = tile.row0 + (SUB);                                                   \
    const int64_t base_ = in.v_off + (int64_t)row_ * P;                                   \
    const T* q0_ = Qg + (int64_t)row_ * n;                                                \
    if (MODE == B_ITER)                                                                   \
      sg.set(4, q0_, nr_ * n, a.u + base_, nr_ * P, a.g + base_, nr_ * P, a.w + base_,    \
             nr_ * P);                                                                    \
    else if (MODE == B_INIT)                                                              \
      sg.set(1 + (have_u ? 1 : 0) + (have_y ? 1 : 0), q0_, nr_ * n,                       \
             have_u ? a.w + base_ : a.y + base_, nr_ * P, a.y + base_, nr_ * P, nullptr, 0); \
    else                                                                                  \
      sg.set(1, q0_, nr_ * n, nullptr, 0, nullptr, 0, nullptr, 0);                        \
  }
  GLM_SETUP_B(0)
  sg.load();
  __syncthreads();
  const bool act = on && s_act[k];
  const T lam = (T)s_lam[k];
  const T ialpha = (T)s_ialpha;
  int kact = 0;
  for (int kk = 0; kk < K; ++kk) kact += s_act[kk];
  double cacc = 0.0;

  for (int sub = 0; sub < tile.rows; sub += rs) {
    const int nr = min(rs, tile.rows - sub);
    const int row = tile.row0 + sub;
    const int64_t base = in.v_off + (int64_t)row * P;
    T* Qs = lds;
    T* Us = lds + (size_t)nr * n;
    T* Gs = Us + (have_u ? (size_t)nr * P : 0);    // g (ITER) or y (INIT)
    T* Ws = Gs + (size_t)nr * P;                    // w (ITER)
    __syncthreads();
    sg.store(lds);
    __syncthreads();
    if (sub + rs < tile.rows) {
      GLM_SETUP_B(sub + rs)
      sg.load();
    }
    if (act) {
#pragma unroll 1
      for (int t = r; t < nr; t += rpar) {
        const T* qrow = Qs + (size_t)t * n + bd.col;
        const size_t l = (size_t)t * P + pr;
        const int64_t e = base + (int64_t)t * P + pr;
        T b = T(0);
        const T* urow = Us + (size_t)t * P + k;
        if (have_u) {
          if (GR > 0) {
#pragma unroll
            for (int j = 0; j < GR; ++j)
              if (j < G) b += urow[j * K] * om[j];
          } else {
            for (int j = 0; j < G; ++j) b += urow[j * K] * Oms[j * G + i];
          }
        }
        T qt = T(0);
#pragma unroll
        for (int c = 0; c < NIM; ++c)
          if (c < bd.ni) qt += qrow[c] * treg[c];
        if (MODE == B_ITER) {
          const T gg = Gs[l] - lam * ialpha * (b - qt);
          a.g[e] = gg;
          a.w[e] = Ws[l] - lam * urow[i * K];
          cacc += (double)gg * (double)gg;
        } else if (MODE == B_INIT) {
          const T yv = have_y ? Gs[l] : T(0);
          const T gg = -((yv - b) - qt) * ialpha;
          a.g[e] = gg;
          cacc += (double)gg * (double)gg;
        } else {
          a.w[e] = qt;
        }
      }
    }
  }
  if (MODE != B_EXPAND) {
    reduce_by_k<NTW>(cacc, on ? k : -1, K, red, csum);
    if ((int)threadIdx.x < K) a.cpart[(int64_t)blockIdx.x * KMAX + threadIdx.x] = csum[threadIdx.x];
  }
  if (MODE == B_ITER && a.bytes && threadIdx.x == 0) {
    const unsigned long long bq = (unsigned long long)tile.rows * n * sizeof(T);
    const unsigned long long bv = 5ull * tile.rows * G * kact * sizeof(T);
    atomicAdd(a.bytes, bq + bv);
  }
}

template <typename T>
Args2<T> to_args2(const PassLaunch<T>& p) {
  Args2<T> a;
  a.insts = p.insts;
  a.tiles = p.tiles;
  a.blks = p.blks;
  a.inst_active = p.inst_active;
  a.Q = p.Q;
  a.Om = p.Om;
  a.alpha = p.alpha;
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

template <typename T, int NTW, int GR, int NIM>
hipError_t dispatch_a(const PassLaunch<T>& p, int mode, hipStream_t s) {
  Args2<T> a = to_args2(p);
  if (mode == A_ITER)
    hipLaunchKernelGGL((k_pass_a2<T, NTW, GR, NIM, A_ITER>), dim3(p.ntiles), dim3(NTW), p.lds,
                       s, a);
  else
    hipLaunchKernelGGL((k_pass_a2<T, NTW, GR, NIM, A_RHS>), dim3(p.ntiles), dim3(NTW), p.lds,
                       s, a);
  return hipGetLastError();
}

template <typename T, int NTW, int GR, int NIM>
hipError_t dispatch_b(const PassLaunch<T>& p, int mode, hipStream_t s) {
  Args2<T> a = to_args2(p);
  if (mode == B_ITER)
    hipLaunchKernelGGL((k_pass_b2<T, NTW, GR, NIM, B_ITER>), dim3(p.ntiles), dim3(NTW), p.lds,
                       s, a);
  else if (mode == B_INIT)
    hipLaunchKernelGGL((k_pass_b2<T, NTW, GR, NIM, B_INIT>), dim3(p.ntiles), dim3(NTW), p.lds,
                       s, a);
  else
    hipLaunchKernelGGL((k_pass_b2<T, NTW, GR, NIM, B_EXPAND>), dim3(p.ntiles), dim3(NTW), p.lds,
                       s, a);
  return hipGetLastError();
}

// (threads, Omega-in-registers width, block-width bound) buckets
template <typename T, bool PASS_A>
hipError_t dispatch(const PassLaunch<T>& p, int mode, hipStream_t s) {
#define GLM_CASE(NTWV, GRV, NIMV)                                                    \
  if (p.ntw == NTWV && p.gr == GRV && p.nim == NIMV)                                 \
    return PASS_A ? dispatch_a<T, NTWV, GRV, NIMV>(p, mode, s)                       \
                  : dispatch_b<T, NTWV, GRV, NIMV>(p, mode, s);
  GLM_CASE(256, 8, 8) GLM_CASE(256, 8, 16) GLM_CASE(256, 8, 24) GLM_CASE(256, 8, 32)
  GLM_CASE(256, 8, 64) GLM_CASE(256, 16, 8) GLM_CASE(256, 16, 16) GLM_CASE(256, 16, 24)
  GLM_CASE(256, 16, 32) GLM_CASE(256, 16, 64) GLM_CASE(256, 32, 8) GLM_CASE(256, 32, 16)
  GLM_CASE(256, 32, 24) GLM_CASE(256, 32, 32) GLM_CASE(256, 32, 64) GLM_CASE(256, 0, 8)
  GLM_CASE(256, 0, 16) GLM_CASE(256, 0, 24) GLM_CASE(256, 0, 32) GLM_CASE(256, 0, 64)
  GLM_CASE(512, 8, 8) GLM_CASE(512, 8, 16) GLM_CASE(512, 8, 24) GLM_CASE(512, 8, 32)
  GLM_CASE(512, 8, 64) GLM_CASE(512, 16, 8) GLM_CASE(512, 16, 16) GLM_CASE(512, 16, 24)
  GLM_CASE(512, 16, 32) GLM_CASE(512, 16, 64) GLM_CASE(512, 32, 8) GLM_CASE(512, 32, 16)
  GLM_CASE(512, 32, 24) GLM_CASE(512, 32, 32) GLM_CASE(512, 32, 64) GLM_CASE(512, 0, 8)
  GLM_CASE(512, 0, 16) GLM_CASE(512, 0, 24) GLM_CASE(512, 0, 32) GLM_CASE(512, 0, 64)
#undef GLM_CASE
  return hipErrorInvalidValue;
}

}  // namespace

template <typename T>
hipError_t launch_pass_a2(const PassLaunch<T>& p, int mode, hipStream_t s) {
  return dispatch<T, true>(p, mode, s);
}
template <typename T>
hipError_t launch_pass_b2(const PassLaunch<T>& p, int mode, hipStream_t s) {
  return dispatch<T, false>(p, mode, s);
}

template hipError_t launch_pass_a2<double>(const PassLaunch<double>&, int, hipStream_t);
template hipError_t launch_pass_a2<float>(const PassLaunch<float>&, int, hipStream_t);
template hipError_t launch_pass_b2<double>(const PassLaunch<double>&, int, hipStream_t);
template hipError_t launch_pass_b2<float>(const PassLaunch<float>&, int, hipStream_t);

}  // namespace glm
