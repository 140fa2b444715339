// Projection passes of the PCG-Aug iteration (algorithm "The PCG-Aug
// method" with the indefinite preconditioner, carried in projected form:
// one OLS projection per iteration), right-hand-side vectorised form.
//
// A workgroup streams one row tile of one instance.  Lane l owns one
// (row group r, equation i, group of KV right-hand sides) triple and, for
// every row t of its group, produces the KV contiguous elements
// (t, i, kq*KV .. kq*KV+KV-1) of the vectors.  In registers per lane:
//   * column i of Omega        -> B[t][i][k] = sum_j U[t][j][k] Omega[j][i]
//   * the slice T_i[., kq*KV ..] of the projection (pass A accumulates
//     Q_i^T B_i over the tile's rows, pass B holds the reduced T_i)
// Each U row element is read once per KV outputs (one 16-byte LDS read) and
// each Q row element once per KV outputs.
//
// Per sub-tile the vector slabs (KV-wide chunks) and the Q rows (scalars)
// are loaded into registers while the previous sub-tile is being computed
// from LDS (register double buffering), so HBM requests stay in flight
// during the arithmetic.
//
//   pass A  ITER : u <- g + mu u ; B = U Omega ; d += u.B ; T_i += Q_i^T B_i
//           RHS  : B = y - W Omega ; T_i += Q_i^T B_i
//   pass B  ITER : g <- g - (lambda/alpha)(B_i - Q_i T_i) ; w <- w - lambda u ; c += g.g
//           INIT : g <- -((y - W Omega) - Q T)/alpha ; c += g.g
//           EXPAND: w <- Q T
#include "glm_internal.h"

#ifndef GLM_PROJ_T
#error "compile once per precision with -DGLM_PROJ_T=float or -DGLM_PROJ_T=double"
#endif

#include <cmath>

namespace glm {

namespace {

constexpr int PNT = PROJ_NT;   // threads per workgroup
constexpr int NV = PROJ_NV;    // vector chunks per thread per sub-tile
constexpr int NQ = PROJ_NQ;    // Q scalars per thread per sub-tile

template <typename T, int N>
struct alignas(sizeof(T) * N) Vec {
  T v[N];
};

template <typename T, int N>
__device__ __forceinline__ Vec<T, N> vload(const T* p) {
  return *reinterpret_cast<const Vec<T, N>*>(p);
}
template <typename T, int N>
__device__ __forceinline__ void vstore(T* p, const Vec<T, N>& x) {
  *reinterpret_cast<Vec<T, N>*>(p) = x;
}

// HBM accesses through explicitly global pointers: flat accesses would also
// count against the LDS wait counter and stall the LDS reads of the compute
// loop behind the prefetch of the next sub-tile.
#define GLM_GLOBAL __attribute__((address_space(1)))
template <typename T, int N>
__device__ __forceinline__ Vec<T, N> gload(const T* p) {
  Vec<T, N> r;
  if constexpr (N == 1) {
    r.v[0] = *(const GLM_GLOBAL T*)(p);
  } else {
    // a native vector load: an aggregate copy could lose the address space
    typedef T VT __attribute__((ext_vector_type(N)));
    const VT x = *(const GLM_GLOBAL VT*)(p);
#pragma unroll
    for (int v = 0; v < N; ++v) r.v[v] = x[v];
  }
  return r;
}
template <typename T, int N>
__device__ __forceinline__ void gstore(T* p, const Vec<T, N>& x) {
  if constexpr (N == 1) {
    *(GLM_GLOBAL T*)(p) = x.v[0];
  } else {
    typedef T VT __attribute__((ext_vector_type(N)));
    VT y;
#pragma unroll
    for (int v = 0; v < N; ++v) y[v] = x.v[v];
    *(GLM_GLOBAL VT*)(p) = y;
  }
}
template <typename T>
__device__ __forceinline__ T gload1(const T* p) {
  return *(const GLM_GLOBAL T*)(p);
}

template <typename T>
struct Args3 {
  const InstDesc* __restrict__ insts;
  const TileDesc* __restrict__ tiles;
  const BlockDesc* __restrict__ blks;
  const int* __restrict__ inst_active;
  const T* __restrict__ Q;
  const T* __restrict__ Om;
  const double* __restrict__ alpha;
  const double* __restrict__ deq;  // per-block D scalars, or null (D = alpha I)
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

// Sub-tile stager: up to three vector slabs of nr*P elements (moved in
// KV-wide chunks) followed by the Q slab of nr*n scalars and PROJ_QPAD
// zeros.  LDS layout: [slab 0][slab 1][slab 2][Q rows][pad], slab s at
// s*nr*P.
template <typename T, int KV, int NQS = NQ, int NVS = NV>
struct Stage3 {
  const T* v0;
  const T* v1;
  const T* v2;
  const T* q;
  int nvec;      // number of vector slabs
  int slab;      // elements per slab (nr * P)
  int qcnt;      // Q elements (nr * n)
  Vec<T, KV> rv[NVS];
  T rq[NQS];

  __device__ __forceinline__ void load() {
    const int tid = threadIdx.x;
    const int cps = slab / KV;   // chunks per slab
    const uint64_t a0 = reinterpret_cast<uint64_t>(v0);
    const uint64_t d1 = reinterpret_cast<uint64_t>(v1) - a0;
    const uint64_t d2 = reinterpret_cast<uint64_t>(v2) - reinterpret_cast<uint64_t>(v1);
#pragma unroll
    for (int s = 0; s < NVS; ++s) {
      const int c = tid + s * PNT;           // chunk index over all slabs
      if (c < nvec * cps) {
        const bool s1 = c >= cps, s2 = c >= 2 * cps;
        const int off = (c - (s1 + s2) * cps) * KV;
        // slab base by address arithmetic: a select between the pointer
        // members would be lowered to an indexed load from a stack copy
        const uint64_t addr = a0 + (s1 ? d1 : 0) + (s2 ? d2 : 0);
        rv[s] = gload<T, KV>(reinterpret_cast<const T*>(addr) + off);
      }
    }
#pragma unroll
    for (int s = 0; s < NQS; ++s) {
      const int e = tid + s * PNT;
      if (e < qcnt) rq[s] = gload1(q + e);
    }
  }
  __device__ __forceinline__ void store(T* __restrict__ lds) const {
    const int tid = threadIdx.x;
    const int cps = slab / KV;
#pragma unroll
    for (int s = 0; s < NVS; ++s) {
      const int c = tid + s * PNT;
      if (c < nvec * cps) vstore<T, KV>(lds + (size_t)c * KV, rv[s]);
    }
    T* lq = lds + (size_t)nvec * slab;
#pragma unroll
    for (int s = 0; s < NQS; ++s) {
      const int e = tid + s * PNT;
      if (e < qcnt) lq[e] = rq[s];
    }
    // columns past the last block of the last row read zeros
    if (tid < PROJ_QPAD) lq[qcnt + tid] = T(0);
  }
};

// out[k] = sum over lanes of acc[v] for the lanes holding right-hand side k.
// Lane -> rhs group: lane % KQ in the vector-ALU mapping, (lane % 64) / 16 in
// the matrix-core mapping (MF).  The reduction buffer aliases the staging
// area, so every wave must be done reading the last sub-tile first.
template <int KV, bool MF>
__device__ void reduce_k(const double (&acc)[KV], bool on, int K, int KQ, double* red,
                         double* out) {
  __syncthreads();
#pragma unroll
  for (int v = 0; v < KV; ++v) red[threadIdx.x * KV + v] = on ? acc[v] : 0.0;
  __syncthreads();
  if ((int)threadIdx.x < K) {
    const int k = threadIdx.x, kq = k / KV, v = k - kq * KV;
    double s = 0.0;
    if (MF) {
      for (int w = 0; w < PNT / 64; ++w)
        for (int l = 0; l < 16; ++l) s += red[(w * 64 + kq * 16 + l) * KV + v];
    } else {
      for (int l = kq; l < PNT; l += KQ) s += red[l * KV + v];
    }
    out[k] = s;
  }
  __syncthreads();
}

// Loops over the Omega column and the Q row run in chunks of JC with one
// uniform test per chunk, so the LDS reads of a chunk issue back to back.
// Entries past G (or past n_i) inside the last chunk read finite LDS data
// (the staging area is zeroed at kernel start) and meet a zero Omega entry
// (or an accumulator that is never stored, or a zero projection entry).
constexpr int JC = 8;
// Projection columns per uniform test in the Q T and Q^T B loops: twelve when
// the n_i bound allows (more LDS reads in flight per batch), else eight.
template <int NIM>
constexpr int jcq() {
  return NIM % 12 == 0 ? 12 : 8;
}

// b[v] += sum_{j < G} U[j][k0 + v] Omega[j][i] for the lane's right-hand-side
// group, U[j] at urow + j*K.  With the stride K known at compile time the
// LDS offsets fold into the instructions; otherwise one pointer walks the row.
template <typename T, int KV, int KS, int GR>
__device__ __forceinline__ void apply_omega(const T* __restrict__ urow, int K, int G, int i,
                                            const T (&om)[GR > 0 ? GR : 1],
                                            const T* __restrict__ Oms, T (&b)[KV]) {
  if constexpr (GR > 0) {
    const T* pu = urow;
#pragma unroll
    for (int j0 = 0; j0 < GR; j0 += JC) {
      if (j0 < G) {
#pragma unroll
        for (int j = j0; j < j0 + JC; ++j) {
          const Vec<T, KV> uv = vload<T, KV>(KS ? urow + j * KS : pu);
          if (!KS) pu += K;
#pragma unroll
          for (int v = 0; v < KV; ++v) b[v] += uv.v[v] * om[j];
        }
      }
    }
  } else {
    const T* pu = urow;
    const T* po = Oms + i;
    for (int j = 0; j < G; ++j) {
      const Vec<T, KV> uv = vload<T, KV>(pu);
      const T o = *po;
      pu += K;
      po += G;
#pragma unroll
      for (int v = 0; v < KV; ++v) b[v] += uv.v[v] * o;
    }
  }
}

// Zero the dynamic LDS staging area (count elements of T).
template <typename T>
__device__ __forceinline__ void zero_lds(T* lds, int count) {
  for (int e = threadIdx.x; e < count; e += PNT) lds[e] = T(0);
}

// ---- Omega apply on the matrix cores (FP32, sixteen right-hand sides) ------
//
// B[t][i][k] = sum_j U[t][j][k] Omega[j][i] for one block of rows is the
// product of a (k x j) slice of U and a (j x i) block of Omega, done with
// v_mfma_f32_16x16x4f32: M = 16 right-hand sides, N = 16 output columns,
// 4 values of j per instruction.  The result lands as lane l, register r ->
// (column l % 16, rhs 4 (l / 16) + r), so each lane holds the four
// consecutive rhs k0 = 4 (l / 16) .. k0 + 3 of one output column, which is the
// lane layout the rest of the pass uses.
//   Gp = G rounded up to a power of two (at least 4).
//   Gp <= 16: the 16 columns are (row tq, equation i) pairs, tq < 16 / Gp, so
//     one product covers 16 / Gp rows; the K dimension runs over (row, j)
//     pairs and Omega enters block-diagonally (zero across rows).
//   Gp = 32, 64: the columns are 16 equations of one block; waves split the
//     Gp / 16 blocks, and the K dimension runs over j.
// Entries of Omega beyond G are zero, so the U values they meet (the next
// equation's or row's, or zeroed LDS) do not contribute.
typedef float mf4 __attribute__((ext_vector_type(4)));

struct MfMap {
  int Gp, small, RB, WPB, rgrp, tq, i, kq, n16;
};

__device__ __forceinline__ MfMap mf_map(int G) {
  MfMap m;
  m.Gp = G <= 4 ? 4 : G <= 8 ? 8 : G <= 16 ? 16 : G <= 32 ? 32 : 64;
  m.small = m.Gp <= 16;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  m.n16 = l & 15;
  m.kq = l >> 4;
  m.RB = m.small ? 16 / m.Gp : 1;
  m.WPB = m.small ? 4 : 64 / m.Gp;
  m.rgrp = m.small ? w : w % m.WPB;
  m.tq = m.small ? m.n16 / m.Gp : 0;
  m.i = m.small ? m.n16 % m.Gp : (w / m.WPB) * 16 + m.n16;
  return m;
}

// B-operand registers: Omega entries this lane feeds to each product.
template <int NB>
__device__ __forceinline__ void mf_load_omega(const MfMap& m, int G, const float* __restrict__ Om,
                                              float (&bom)[NB]) {
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    float v = 0.f;
    if (m.small) {
      if (q < 4) {
        const int kk = 4 * q + m.kq, tr = kk / m.Gp, j = kk - tr * m.Gp;
        if (tr == m.tq && j < G && m.i < G) v = Om[j * G + m.i];
      }
    } else if (q < m.Gp / 4) {
      const int j = 4 * q + m.kq;
      if (j < G && m.i < G) v = Om[j * G + m.i];
    }
    bom[q] = v;
  }
}

// acc[r] = B[t0 + tq][i][4 kq + r] for the row block starting at t0 (P = 16 G).
template <int NB>
__device__ __forceinline__ mf4 mf_apply(const MfMap& m, const float* __restrict__ Us, int t0,
                                        int P, const float (&bom)[NB]) {
  mf4 acc = {0.f, 0.f, 0.f, 0.f};
  if (m.small) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = 4 * q + m.kq, tr = kk / m.Gp, j = kk - tr * m.Gp;
      const float a = Us[(t0 + tr) * P + j * 16 + m.n16];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bom[q], acc, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (q < m.Gp / 4) {
        const float a = Us[t0 * P + (4 * q + m.kq) * 16 + m.n16];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bom[q], acc, 0, 0, 0);
      }
  }
  return acc;
}

template <typename T, int KV, int KS, int GR, int NIM, int MODE>
__global__ void __launch_bounds__(PNT) k_proj_a(Args3<T> a) {
  const TileDesc tile = a.tiles[blockIdx.x];
  if (!a.inst_active[tile.inst]) return;
  const InstDesc in = a.insts[tile.inst];
  // pass A stages two vector slabs, so its sub-tiles take more Q rows
  const int G = in.G, K = KS ? KS : in.K, n = in.n, rs = rows_a_of<T>(in), P = G * K,
            KQ = K / KV;
  const int PP = G * KQ;           // lanes per row
  const int rpar = rpar_of<T>(in), nimax = in.nimax;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  T* Oms = lds + (size_t)PNT * (NV * KV + PROJ_NQA) + PROJ_QPAD;   // Omega unless in registers
  zero_lds(lds, PNT * (NV * KV + PROJ_NQA) + PROJ_QPAD);
  __shared__ double s_mu[KMAX];
  __shared__ int s_act[KMAX], s_first[KMAX];
  __shared__ double dsum[KMAX];
  if ((int)threadIdx.x < K) {
    const RhsState s = a.st[in.rhs0 + threadIdx.x];
    s_act[threadIdx.x] = (s.status == ST_ACTIVE);
    s_first[threadIdx.x] = (s.iters == 0);
    s_mu[threadIdx.x] = s.mu;
  }
  const T* __restrict__ Om = a.Om + in.om_off;
  if (GR == 0)
    for (int e = threadIdx.x; e < G * G; e += PNT) Oms[e] = Om[e];
  constexpr bool MF = GR < 0;                // Omega apply on the matrix cores
  constexpr int NB = MF ? -GR / 4 : 1;
  const int lane = threadIdx.x;
  bool on;
  int r, i, kq;
  MfMap mm{};
  if constexpr (MF) {
    mm = mf_map(G);
    on = mm.i < G;
    r = mm.rgrp * mm.RB + mm.tq;
    i = on ? mm.i : 0;
    kq = mm.kq;
  } else {
    on = lane < rpar * PP;
    r = on ? lane / PP : 0;
    const int pr = on ? lane - r * PP : 0;
    i = pr / KQ;
    kq = pr - (pr / KQ) * KQ;
  }
  const int k0 = kq * KV;
  // row stride of the lane's rows: the matrix-core mapping fixes it at 64 / Gp
  const int rstep = MF ? mm.WPB * mm.RB : rpar;
  const BlockDesc bd = a.blks[in.blk0 + i];
  const int ni = bd.ni, col = bd.col;
  T om[GR > 0 ? GR : 1];
  if (GR > 0) {
#pragma unroll
    for (int j = 0; j < GR; ++j) om[j] = (j < G) ? Om[j * G + i] : T(0);
  }
  float bom[NB];
  if constexpr (MF) mf_load_omega<NB>(mm, G, Om, bom);
  T tacc[NIM][KV];
#pragma unroll
  for (int c = 0; c < NIM; ++c)
#pragma unroll
    for (int v = 0; v < KV; ++v) tacc[c][v] = T(0);
  double dacc[KV];
#pragma unroll
  for (int v = 0; v < KV; ++v) dacc[v] = 0.0;
  const bool have_w = (MODE == PASS_A_ITER) || a.w_nonzero;
  const bool have_y = (MODE == PASS_A_RHS) && a.y;
  const T* __restrict__ Qg = a.Q + in.q_off;

  Stage3<T, KV, PROJ_NQA> sg;
  int sub = 0;
  {
    const int nr = min(rs, tile.rows);
    const int64_t base = in.v_off + (int64_t)tile.row0 * P;
    sg.slab = nr * P;
    sg.qcnt = nr * n;
    sg.q = Qg + (int64_t)tile.row0 * n;
    if (MODE == PASS_A_ITER) {
      sg.nvec = 2; sg.v0 = a.u + base; sg.v1 = a.g + base; sg.v2 = nullptr;
    } else {
      sg.nvec = (have_w ? 1 : 0) + (have_y ? 1 : 0);
      sg.v0 = have_w ? a.w + base : a.y + base;
      sg.v1 = a.y + base;
      sg.v2 = nullptr;
    }
    sg.load();
  }
  __syncthreads();
  int kact = 0;
  for (int kk = 0; kk < K; ++kk) kact += s_act[kk];

  for (; sub < tile.rows; sub += rs) {
    const int nr = min(rs, tile.rows - sub);
    const int row = tile.row0 + sub;
    const int64_t base = in.v_off + (int64_t)row * P;
    const int slab = nr * P;
    T* Us = lds;                                   // u (ITER) or w (RHS)
    T* Ys = lds + (have_w ? slab : 0);             // g (ITER) or y (RHS)
    T* Qs = lds + (size_t)sg.nvec * slab;
    __syncthreads();
    sg.store(lds);
    __syncthreads();
    if (sub + rs < tile.rows) {                    // prefetch the next sub-tile
      const int nr2 = min(rs, tile.rows - sub - rs);
      const int64_t b2 = base + (int64_t)rs * P;
      sg.slab = nr2 * P;
      sg.qcnt = nr2 * n;
      sg.q = Qg + (int64_t)(row + rs) * n;
      if (MODE == PASS_A_ITER) {
        sg.v0 = a.u + b2; sg.v1 = a.g + b2;
      } else {
        sg.v0 = have_w ? a.w + b2 : a.y + b2;
        sg.v1 = a.y + b2;
      }
      sg.load();
    }
    if (MODE == PASS_A_ITER) {
      // u <- g + mu u on the staged slabs, written back to HBM
      for (int c = threadIdx.x; c < slab / KV; c += PNT) {
        const int e = c * KV;
        const int kk = e % K;
        Vec<T, KV> uo = vload<T, KV>(Us + e);
        const Vec<T, KV> go = vload<T, KV>(Ys + e);
        bool any = false;
#pragma unroll
        for (int v = 0; v < KV; ++v) {
          if (s_act[kk + v]) {
            uo.v[v] = s_first[kk + v] ? go.v[v] : go.v[v] + (T)s_mu[kk + v] * uo.v[v];
            any = true;
          }
        }
        if (any) {
          vstore<T, KV>(Us + e, uo);
          gstore<T, KV>(a.u + base + e, uo);
        }
      }
      __syncthreads();
    }
    // rows t = r + it * rpar; the trip count is uniform across the workgroup
    for (int it = 0; it * rstep < nr; ++it) {
      const int t = r + it * rstep;
      {
        T b[KV];
#pragma unroll
        for (int v = 0; v < KV; ++v) b[v] = T(0);
        if constexpr (MF) {
          if (have_w) {
            const mf4 acc = mf_apply<NB>(mm, Us, t - mm.tq, P, bom);
#pragma unroll
            for (int v = 0; v < KV; ++v) b[v] = acc[v];
          }
        }
        if (!(on && t < nr)) continue;
        const T* urow = Us + (size_t)t * P + k0;
        if constexpr (!MF) {
          if (have_w) apply_omega<T, KV, KS, GR>(urow, K, G, i, om, Oms, b);
        }
        if (MODE == PASS_A_ITER) {
          const Vec<T, KV> ui = vload<T, KV>(urow + i * K);
#pragma unroll
          for (int v = 0; v < KV; ++v) dacc[v] += (double)ui.v[v] * (double)b[v];
        } else {
          if (have_y) {
            const Vec<T, KV> yv = vload<T, KV>(Ys + (size_t)t * P + i * K + k0);
#pragma unroll
            for (int v = 0; v < KV; ++v) b[v] = yv.v[v] - b[v];
          } else {
#pragma unroll
            for (int v = 0; v < KV; ++v) b[v] = -b[v];
          }
        }
        // columns c >= n_i belong to the next block (or the zero pad): their
        // accumulators are never stored
        const T* qrow = Qs + (size_t)t * n + col;
#pragma unroll
        for (int c0 = 0; c0 < NIM; c0 += jcq<NIM>())
          if (c0 < nimax) {
#pragma unroll
            for (int c = c0; c < c0 + jcq<NIM>(); ++c) {
              const T q = qrow[c];
#pragma unroll
              for (int v = 0; v < KV; ++v) tacc[c][v] += q * b[v];
            }
          }
      }
    }
  }
  // The tile's partial Q^T B, one slot per row group; on the matrix-core
  // mapping with gp <= 16 the rows of a wave are summed first by shuffles over
  // the row bits of the lane index, one slot per wave (mf_partial_slots).
  int slot = r;
  bool store = on;
  if constexpr (MF) {
    if (mm.small) {
      for (int sh = mm.Gp; sh < 16; sh <<= 1)
#pragma unroll
        for (int c = 0; c < NIM; ++c)
#pragma unroll
          for (int v = 0; v < KV; ++v) tacc[c][v] += __shfl_xor(tacc[c][v], sh, 64);
      slot = mm.rgrp;
      store = on && mm.tq == 0;
    }
  }
  if (store) {
    T* tp = a.Tpart + tile.tp_off + (int64_t)slot * n * K + (int64_t)col * K + k0;
#pragma unroll
    for (int c = 0; c < NIM; ++c)
      if (c < ni) {
        Vec<T, KV> x;
#pragma unroll
        for (int v = 0; v < KV; ++v) x.v[v] = tacc[c][v];
        gstore<T, KV>(tp + (int64_t)c * K, x);
      }
  }
  if (MODE == PASS_A_ITER) {
    reduce_k<KV, MF>(dacc, on, K, KQ, reinterpret_cast<double*>(smem_raw), dsum);
    if ((int)threadIdx.x < K) a.dpart[(int64_t)blockIdx.x * KMAX + threadIdx.x] = dsum[threadIdx.x];
  }
  // Algorithmic bytes of one iteration: Q twice (once per pass) and each of
  // g, u, w read and written once; pass A is charged Q + (read u, g, write u),
  // pass B Q + (read w, write g, w).  Its reads of u and g re-read vectors
  // pass A already moved and are not counted.  Active right-hand sides only.
  if (a.bytes && threadIdx.x == 0 && MODE == PASS_A_ITER) {
    const unsigned long long bq = (unsigned long long)tile.rows * n * sizeof(T);
    const unsigned long long bv = 3ull * tile.rows * G * kact * sizeof(T);
    atomicAdd(a.bytes, bq + bv);
  }
}

template <typename T, int KV, int KS, int GR, int NIM, int MODE>
__global__ void __launch_bounds__(PNT) k_proj_b(Args3<T> a) {
  const TileDesc tile = a.tiles[blockIdx.x];
  if (!a.inst_active[tile.inst]) return;
  const InstDesc in = a.insts[tile.inst];
  const int G = in.G, K = KS ? KS : in.K, n = in.n, rs = rows_of<T>(in), P = G * K, KQ = K / KV;
  const int PP = G * KQ;
  const int rpar = rpar_of<T>(in), nimax = in.nimax;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  T* Oms = lds + (size_t)PNT * (PROJ_NVB * KV + PROJ_NQB) + PROJ_QPAD;
  zero_lds(lds, PNT * (PROJ_NVB * KV + PROJ_NQB) + PROJ_QPAD);
  __shared__ double s_lam[KMAX];
  __shared__ int s_act[KMAX];
  __shared__ double csum[KMAX];
  __shared__ double s_ialpha;
  if ((int)threadIdx.x < K) {
    const RhsState s = a.st[in.rhs0 + threadIdx.x];
    s_act[threadIdx.x] = (s.status == ST_ACTIVE);
    s_lam[threadIdx.x] = s.lam;
  }
  if (threadIdx.x == 0) s_ialpha = 1.0 / a.alpha[tile.inst];
  const T* __restrict__ Om = a.Om + in.om_off;
  if (GR == 0 && MODE != PASS_B_EXPAND)
    for (int e = threadIdx.x; e < G * G; e += PNT) Oms[e] = Om[e];
  constexpr bool MF = GR < 0;                // Omega apply on the matrix cores
  constexpr int NB = MF ? -GR / 4 : 1;
  const int lane = threadIdx.x;
  bool on;
  int r, i, kq;
  MfMap mm{};
  if constexpr (MF) {
    mm = mf_map(G);
    on = mm.i < G;
    r = mm.rgrp * mm.RB + mm.tq;
    i = on ? mm.i : 0;
    kq = mm.kq;
  } else {
    on = lane < rpar * PP;
    r = on ? lane / PP : 0;
    const int pr = on ? lane - r * PP : 0;
    i = pr / KQ;
    kq = pr - (pr / KQ) * KQ;
  }
  const int k0 = kq * KV;
  // row stride of the lane's rows: the matrix-core mapping fixes it at 64 / Gp
  const int rstep = MF ? mm.WPB * mm.RB : rpar;
  const BlockDesc bd = a.blks[in.blk0 + i];
  const int ni = bd.ni, col = bd.col;
  T om[GR > 0 ? GR : 1];
  if (GR > 0 && MODE != PASS_B_EXPAND) {
#pragma unroll
    for (int j = 0; j < GR; ++j) om[j] = (j < G) ? Om[j * G + i] : T(0);
  }
  float bom[NB];
  if constexpr (MF)
    if (MODE != PASS_B_EXPAND) mf_load_omega<NB>(mm, G, Om, bom);
  T treg[NIM][KV];
  {
    const T* tb = a.Tm + in.t_off + (int64_t)col * K + k0;
#pragma unroll
    for (int c = 0; c < NIM; ++c) {
      Vec<T, KV> x;
#pragma unroll
      for (int v = 0; v < KV; ++v) x.v[v] = T(0);
      if (on && c < ni) x = gload<T, KV>(tb + (int64_t)c * K);
#pragma unroll
      for (int v = 0; v < KV; ++v) treg[c][v] = x.v[v];
    }
  }
  const bool have_u = (MODE == PASS_B_ITER) || (MODE == PASS_B_INIT && a.w_nonzero);
  const bool have_y = (MODE == PASS_B_INIT) && a.y;
  const T* __restrict__ Qg = a.Q + in.q_off;

  Stage3<T, KV, PROJ_NQB, PROJ_NVB> sg;
  {
    const int nr = min(rs, tile.rows);
    const int64_t base = in.v_off + (int64_t)tile.row0 * P;
    sg.slab = nr * P;
    sg.qcnt = nr * n;
    sg.q = Qg + (int64_t)tile.row0 * n;
    if (MODE == PASS_B_ITER) {
      sg.nvec = 3; sg.v0 = a.u + base; sg.v1 = a.g + base; sg.v2 = a.w + base;
    } else if (MODE == PASS_B_INIT) {
      sg.nvec = (have_u ? 1 : 0) + (have_y ? 1 : 0);
      sg.v0 = have_u ? a.w + base : a.y + base;
      sg.v1 = a.y + base;
      sg.v2 = nullptr;
    } else {
      sg.nvec = 0; sg.v0 = sg.v1 = sg.v2 = nullptr;
    }
    sg.load();
  }
  __syncthreads();
  bool actk[KV];
  T lam[KV];
#pragma unroll
  for (int v = 0; v < KV; ++v) {
    actk[v] = on && s_act[k0 + v];
    lam[v] = (T)s_lam[k0 + v];
  }
  bool act = false;
#pragma unroll
  for (int v = 0; v < KV; ++v) act = act || actk[v];
  // D = diag(d) (x) I_M: this lane's equation scales g by 1 / d_i, and
  // c = sum_i d_i ||g_i||^2 is accumulated as alpha * sum_i (d_i / alpha) ||g_i||^2
  T ialpha = (T)s_ialpha;
  double wgt = 1.0;
  if (a.deq && on) {
    const double di = a.deq[in.blk0 + i];
    ialpha = (T)(1.0 / di);
    wgt = di * s_ialpha;
  }
  int kact = 0;
  for (int kk = 0; kk < K; ++kk) kact += s_act[kk];
  double cacc[KV];
#pragma unroll
  for (int v = 0; v < KV; ++v) cacc[v] = 0.0;

  for (int sub = 0; sub < tile.rows; sub += rs) {
    const int nr = min(rs, tile.rows - sub);
    const int row = tile.row0 + sub;
    const int64_t base = in.v_off + (int64_t)row * P;
    const int slab = nr * P;
    T* Us = lds;                                            // u (ITER) or w (INIT)
    T* Gs = lds + (have_u ? slab : 0);                      // g (ITER) or y (INIT)
    T* Ws = Gs + slab;                                      // w (ITER)
    T* Qs = lds + (size_t)sg.nvec * slab;
    __syncthreads();
    sg.store(lds);
    __syncthreads();
    if (sub + rs < tile.rows) {
      const int nr2 = min(rs, tile.rows - sub - rs);
      const int64_t b2 = base + (int64_t)rs * P;
      sg.slab = nr2 * P;
      sg.qcnt = nr2 * n;
      sg.q = Qg + (int64_t)(row + rs) * n;
      if (MODE == PASS_B_ITER) {
        sg.v0 = a.u + b2; sg.v1 = a.g + b2; sg.v2 = a.w + b2;
      } else if (MODE == PASS_B_INIT) {
        sg.v0 = have_u ? a.w + b2 : a.y + b2;
        sg.v1 = a.y + b2;
      }
      sg.load();
    }
    // rows t = r + it * rpar; the trip count is uniform across the workgroup
    for (int it = 0; it * rstep < nr; ++it) {
      const int t = r + it * rstep;
      {
        T b[KV];
#pragma unroll
        for (int v = 0; v < KV; ++v) b[v] = T(0);
        if constexpr (MF) {
          if (have_u) {
            const mf4 acc = mf_apply<NB>(mm, Us, t - mm.tq, P, bom);
#pragma unroll
            for (int v = 0; v < KV; ++v) b[v] = acc[v];
          }
        }
        if (!(act && t < nr)) continue;
        const size_t l = (size_t)t * P + i * K + k0;
        const int64_t e = base + (int64_t)t * P + i * K + k0;
        const T* urow = Us + (size_t)t * P + k0;
        if constexpr (!MF) {
          if (have_u) apply_omega<T, KV, KS, GR>(urow, K, G, i, om, Oms, b);
        }
        T qt[KV];
#pragma unroll
        for (int v = 0; v < KV; ++v) qt[v] = T(0);
        // treg[c] is zero for c >= n_i, where q is the next block's (finite)
        // entry or the zero pad
        const T* qrow = Qs + (size_t)t * n + col;
#pragma unroll
        for (int c0 = 0; c0 < NIM; c0 += jcq<NIM>())
          if (c0 < nimax) {
#pragma unroll
            for (int c = c0; c < c0 + jcq<NIM>(); ++c) {
              const T q = qrow[c];
#pragma unroll
              for (int v = 0; v < KV; ++v) qt[v] += q * treg[c][v];
            }
          }
        if (MODE == PASS_B_ITER) {
          const Vec<T, KV> gv = vload<T, KV>(Gs + l);
          const Vec<T, KV> wv = vload<T, KV>(Ws + l);
          const Vec<T, KV> uv = vload<T, KV>(Us + l);
          Vec<T, KV> gn, wn;
#pragma unroll
          for (int v = 0; v < KV; ++v) {
            if (actk[v]) {
              gn.v[v] = gv.v[v] - lam[v] * ialpha * (b[v] - qt[v]);
              wn.v[v] = wv.v[v] - lam[v] * uv.v[v];
              cacc[v] += wgt * (double)gn.v[v] * (double)gn.v[v];
            } else {
              gn.v[v] = gv.v[v];
              wn.v[v] = wv.v[v];
            }
          }
          gstore<T, KV>(a.g + e, gn);
          gstore<T, KV>(a.w + e, wn);
        } else if (MODE == PASS_B_INIT) {
          Vec<T, KV> yv;
          if (have_y) {
            yv = vload<T, KV>(Gs + l);
          } else {
#pragma unroll
            for (int v = 0; v < KV; ++v) yv.v[v] = T(0);
          }
          Vec<T, KV> gn;
#pragma unroll
          for (int v = 0; v < KV; ++v) {
            const T gg = -((yv.v[v] - b[v]) - qt[v]) * ialpha;
            gn.v[v] = gg;
            if (actk[v]) cacc[v] += wgt * (double)gg * (double)gg;
          }
          // inactive right-hand sides keep their g (never read before INIT)
          gstore<T, KV>(a.g + e, gn);
        } else {
          bool all = true;
#pragma unroll
          for (int v = 0; v < KV; ++v) all = all && actk[v];
          Vec<T, KV> wn;
          if (!all) wn = gload<T, KV>(a.w + e);
#pragma unroll
          for (int v = 0; v < KV; ++v)
            if (actk[v]) wn.v[v] = qt[v];
          gstore<T, KV>(a.w + e, wn);
        }
      }
    }
  }
  if (MODE != PASS_B_EXPAND) {
    reduce_k<KV, MF>(cacc, on, K, KQ, reinterpret_cast<double*>(smem_raw), csum);
    if ((int)threadIdx.x < K) a.cpart[(int64_t)blockIdx.x * KMAX + threadIdx.x] = csum[threadIdx.x];
  }
  // algorithmic bytes: Q + (read w, write g, w); see pass A
  if (MODE == PASS_B_ITER && a.bytes && threadIdx.x == 0) {
    const unsigned long long bq = (unsigned long long)tile.rows * n * sizeof(T);
    const unsigned long long bv = 3ull * tile.rows * G * kact * sizeof(T);
    atomicAdd(a.bytes, bq + bv);
  }
}

template <typename T>
Args3<T> to_args3(const PassLaunch<T>& p) {
  Args3<T> a;
  a.insts = p.insts;
  a.tiles = p.tiles;
  a.blks = p.blks;
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

template <typename T, int KV, int KS, int GR, int NIM>
hipError_t go(const PassLaunch<T>& p, bool pass_a, int mode, hipStream_t s) {
  Args3<T> a = to_args3(p);
  const dim3 grid(p.ntiles), block(PNT);
  if (pass_a) {
    if (mode == PASS_A_ITER)
      hipLaunchKernelGGL((k_proj_a<T, KV, KS, GR, NIM, PASS_A_ITER>), grid, block, p.lds, s, a);
    else
      hipLaunchKernelGGL((k_proj_a<T, KV, KS, GR, NIM, PASS_A_RHS>), grid, block, p.lds, s, a);
  } else {
    if (mode == PASS_B_ITER)
      hipLaunchKernelGGL((k_proj_b<T, KV, KS, GR, NIM, PASS_B_ITER>), grid, block, p.lds, s, a);
    else if (mode == PASS_B_INIT)
      hipLaunchKernelGGL((k_proj_b<T, KV, KS, GR, NIM, PASS_B_INIT>), grid, block, p.lds, s, a);
    else
      hipLaunchKernelGGL((k_proj_b<T, KV, KS, GR, NIM, PASS_B_EXPAND>), grid, block, p.lds, s, a);
  }
  return hipGetLastError();
}

// Only (NIM, KV) pairs whose per-lane projection slice fits kProjSliceRegs
// 32-bit registers are instantiated: larger slices would spill.
template <typename T, int KV, int KS, int GR>
hipError_t by_nim(const PassLaunch<T>& p, bool pass_a, int mode, hipStream_t s) {
  constexpr int W = sizeof(T) / 4;
  switch (p.nim) {
    case 8:
      if constexpr (8 * KV * W <= kProjSliceRegs) return go<T, KV, KS, GR, 8>(p, pass_a, mode, s);
      break;
    case 16:
      if constexpr (16 * KV * W <= kProjSliceRegs) return go<T, KV, KS, GR, 16>(p, pass_a, mode, s);
      break;
    case 24:
      if constexpr (24 * KV * W <= kProjSliceRegs) return go<T, KV, KS, GR, 24>(p, pass_a, mode, s);
      break;
    case 32:
      if constexpr (32 * KV * W <= kProjSliceRegs) return go<T, KV, KS, GR, 32>(p, pass_a, mode, s);
      break;
    case 64:
      if constexpr (64 * KV * W <= kProjSliceRegs) return go<T, KV, KS, GR, 64>(p, pass_a, mode, s);
      break;
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template <typename T, int KV, int KS>
hipError_t by_gr(const PassLaunch<T>& p, bool pass_a, int mode, hipStream_t s) {
  if (p.gr == 32) return by_nim<T, KV, KS, 32>(p, pass_a, mode, s);
  if (p.gr == 0) return by_nim<T, KV, KS, 0>(p, pass_a, mode, s);
  // matrix-core Omega apply: FP32, sixteen rhs, G up to -gr
  if constexpr (sizeof(T) == 4 && KV == 4 && KS == 16) {
    if (p.gr == -16) return by_nim<T, KV, KS, -16>(p, pass_a, mode, s);
    if (p.gr == -32) return by_nim<T, KV, KS, -32>(p, pass_a, mode, s);
    if (p.gr == -64) return by_nim<T, KV, KS, -64>(p, pass_a, mode, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

template <>
hipError_t launch_proj<GLM_PROJ_T>(const PassLaunch<GLM_PROJ_T>& p, bool pass_a, int mode,
                                   hipStream_t s) {
  using T = GLM_PROJ_T;
  constexpr int KVW = sizeof(T) == 4 ? 4 : 2;
  // sixteen right-hand sides per instance (stride known at compile time)
  if (p.ks == 16) return p.kv == KVW ? by_gr<T, KVW, 16>(p, pass_a, mode, s) : hipErrorInvalidValue;
  switch (p.kv) {
    case 1: return by_gr<T, 1, 0>(p, pass_a, mode, s);
    case 2: return by_gr<T, 2, 0>(p, pass_a, mode, s);
    case 4:
      if constexpr (sizeof(T) == 4) return by_gr<T, 4, 0>(p, pass_a, mode, s);
      break;
    default:
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace glm
