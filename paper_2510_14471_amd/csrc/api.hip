// Host orchestration and the C ABI (include/glm.h).
//
// glm_qr_factor builds the static plan (descriptors, tile schedule, workspace
// layout), uploads it once and runs the batched QR.  glm_gls_solve runs the
// PCG-Aug loop as a fixed sequence of launches per iteration
//     pass A -> reduce T -> scalar A (lambda) -> pass B -> scalar B (mu, tests)
// for all instances at once; converged (instance, rhs) pairs are masked on
// the device and the host polls one counter every few iterations.  GLM_MIXED
// wraps single-precision inner solves in double-precision iterative
// refinement on the augmented system.
#include "glm.h"
#include "glm_internal.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

using namespace glm;

static __device__ __align__(256) unsigned char scratch[size_t(64) << 20];

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kLdsBudget = 48 * 1024;  // dynamic LDS per workgroup (U and B slabs)
constexpr size_t kRowOmegaLds = 64 * 1024; // largest Omega the row-vector passes stage in LDS
constexpr int kRowsPerLane = 16;            // row-vector passes: rows per lane and sub-tile
constexpr int kTargetTiles = 12288;       // row tiles over the whole batch (equal cost)
constexpr int kMinTileRows = 16;          // keeps the per-tile partial sums small
// streaming cost (elements) below which a tile is not cut: a small batch (the
// n + 1 rows of a reduced model) gets fewer, larger tiles
constexpr double kMinTileCost = 32768.0;
constexpr int kPollEvery = 8;             // iterations between host convergence polls
// Stagnation windows: iterations in which c must at least halve.  Slowly
// converging systems (singular Omega with a wide nonzero spectrum) need
// thousands of iterations and plateaus of hundreds, so the windows only end
// solves that sit on their rounding floor.
constexpr int kStallFP64 = 2000;
constexpr int kStallInner = 400;
constexpr double kInnerTol = 1e-3;        // inner single-precision relative tolerance
constexpr int kInnerMaxit = 20000;        // cap of one inner solve
constexpr int kMaxOuter = 12;             // refinement steps

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// GLM_FP64 or GLM_MIXED, optionally with the GLM_REDUCED and GLM_PRECOND_EQ flags
bool prec_ok(glm_precision p) {
  const int v = (int)p & ~(GLM_REDUCED | GLM_PRECOND_EQ);
  return v == GLM_FP64 || v == GLM_MIXED;
}

// Device scratch of glm_qr_factor_static, for callers that cannot allocate
// device memory: one copy per GPU, held until the process ends.  Host code
// never uses the symbol's name as an address (it is a host-side stand-in);
// it takes each device's address from hipGetSymbolAddress, once per device
// with that device current, and passes that.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// The current device's address of `scratch`, looked up on first use.
hipError_t static_scratch(void** out) {
  static_assert(sizeof(scratch) == kStaticScratchBytes, "one size for both");
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev)) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) return e;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

// Progress trace on stderr when the environment variable GLM_LOG is set.
bool log_on() {
  static const bool on = std::getenv("GLM_LOG") != nullptr;
  return on;
}

double now_s() {
  using clk = std::chrono::steady_clock;
  static const clk::time_point t0 = clk::now();
  return std::chrono::duration<double>(clk::now() - t0).count();
}

struct PassCfg {
  int rowpass = 0, kv = 1, ks = 0, gr = 0, nim = 8;
  size_t lds = 0;
};

// Pass configuration for element size sv over the whole batch: the
// row-vector passes when every instance fits them, else the column-slot passes.
PassCfg choose_cfg(const glm_shape* s, size_t sv, bool allow_rows) {
  PassCfg c;
  const int words = (int)(sv / 4);
  int maxG = 0, maxni = 0;
  bool k_div[5] = {true, true, true, true, true};   // K % 1, 2, 4 == 0
  bool all16 = true;
  int64_t off = 0;
  for (int b = 0; b < s->batch; ++b) {
    maxG = std::max(maxG, s->G[b]);
    for (int i = 0; i < s->G[b]; ++i) maxni = std::max(maxni, s->n[off + i]);
    off += s->G[b];
    k_div[2] = k_div[2] && s->K[b] % 2 == 0;
    k_div[4] = k_div[4] && s->K[b] % 4 == 0;
    all16 = all16 && s->K[b] == 16;
  }
  c.nim = maxni <= 8 ? 8 : maxni <= 16 ? 16 : maxni <= 24 ? 24 : maxni <= 32 ? 32 : 64;
  c.kv = 1;
  for (int kv = (sv == 4) ? 4 : 2; kv > 1; kv /= 2)
    if (k_div[kv] && c.nim * kv * words <= kProjSliceRegs) {
      c.kv = kv;
      break;
    }
  c.ks = (all16 && c.kv == ((sv == 4) ? 4 : 2)) ? 16 : 0;
  // FP32 with sixteen rhs everywhere: the Omega apply runs on the matrix cores
  // (gr < 0 encodes the largest padded G, -16 / -32 / -64)
  if (sv == 4 && all16 && maxG <= 64 && c.nim <= 32 && allow_rows) {
    c.kv = 4;
    c.ks = 16;
    c.gr = maxG <= 16 ? -16 : maxG <= 32 ? -32 : -64;
    c.rowpass = 1;
    c.lds = ((size_t)PROJ_NT * std::max(PROJ_NV * c.kv + PROJ_NQA, PROJ_NVB * c.kv + PROJ_NQB) +
             PROJ_QPAD) * sv;
    return c;
  }
  // the Omega column in registers next to the projection slice, else in LDS
  c.gr = (maxG <= 32 && (32 + c.nim * c.kv) * words <= kProjSliceRegs) ? 32 : 0;
  bool fits = c.nim * words <= kProjSliceRegs;
  if (c.gr == 0) fits = fits && (size_t)maxG * maxG * sv <= kRowOmegaLds;
  for (int b = 0; b < s->batch; ++b) fits = fits && s->G[b] * s->K[b] / c.kv <= PROJ_NT;
  c.rowpass = (fits && allow_rows) ? 1 : 0;
  if (c.rowpass)
    c.lds = ((size_t)PROJ_NT * std::max(PROJ_NV * c.kv + PROJ_NQA, PROJ_NVB * c.kv + PROJ_NQB) +
             PROJ_QPAD) * sv + (c.gr == 0 ? (size_t)maxG * maxG * sv : 0);
  return c;
}

struct Plan {
  int B = 0;
  glm_precision prec = GLM_FP64;
  bool deq = false;   // D = diag(omega_ii) (x) I_M instead of alpha I
  std::vector<InstDesc> inst;
  std::vector<BlockDesc> blk;
  std::vector<TileDesc> tile;
  std::vector<QRJob> qr_sur, qr_nb;
  std::vector<RedChunk> chunks;
  std::vector<int> rinst, rinst_index, colblk;
  int64_t sumMn = 0, sumMGK = 0, sumnK = 0, sumTK = 0, sumG2 = 0, sumR = 0, sumNb = 0,
          sumCK = 0, sumTp = 0, sumRc = 0;
  int nrhs = 0, ntiles = 0, nblk = 0, maxK = 0, maxn = 0, maxni = 0, maxkc = 0;
  int kc_t = 1, sl = 1;
  // projection-pass configuration per arithmetic precision (index 0 = FP32
  // inner solves of the mixed path, 1 = FP64 solves)
  PassCfg cfg[2];
  // byte offsets inside the workspace
  size_t o_Q64, o_Q32, o_R, o_Nb, o_colblk, o_inst, o_blk, o_tile, o_qrs, o_qrn, o_chunks,
      o_rinst, o_rinst_index, o_flags, o_active, o_icount, o_count, o_st, o_ost, o_alpha, o_deq,
      o_Om32, o_g, o_u, o_wf, o_yf, o_y64, o_Tpart, o_Tm, o_dpart, o_cpart, o_gc, o_uc, o_wc,
      o_wc64, o_rho0, o_rhoc, o_lb, o_eye, o_mone, o_ypart, o_bytes, o_ne_oinv, o_ne_a,
      o_ne_r, o_ne_z, o_ne_p;
  size_t total = 0;
};

int pick_kc(int k) {
  int v = 1;
  while (v < k) v <<= 1;
  return v;
}

int validate(const glm_shape* s) {
  if (!s || s->batch < 1 || !s->G || !s->M || !s->K || !s->n) return GLM_EINVAL;
  int64_t off = 0;
  for (int b = 0; b < s->batch; ++b) {
    const int G = s->G[b], M = s->M[b], K = s->K[b], kc = s->k ? s->k[b] : 0;
    if (G < 1 || M < 1 || K < 1 || K > KMAX || kc < 0) return GLM_EINVAL;
    int64_t n = 0;
    for (int i = 0; i < G; ++i) {
      const int ni = s->n[off + i];
      if (ni < 1 || ni > M) return GLM_EINVAL;
      if (ni > QR_NMAX) return GLM_EUNSUPPORTED;
      n += ni;
    }
    off += G;
    if (kc > n) return GLM_EINVAL;
    if (n >= (int64_t)G * M + kc) return GLM_EINVAL;  // m + k > n needed for the augmented system
    if (kc > 64) return GLM_EUNSUPPORTED;
    // column slots per thread of the projection passes: up to 4 for any K,
    // up to 8 (n <= 2048) when K <= 4
    if (n > NMAX_INST) return GLM_EUNSUPPORTED;
    const int slots = (int)((n + NT - 1) / NT);
    if (slots > 4 && pick_kc(K) > 4) return GLM_EUNSUPPORTED;
    if ((int64_t)G * G > 64 * 1024) return GLM_EUNSUPPORTED;
  }
  return GLM_OK;
}

// allow_rows[pi]: the row-vector passes may be used for precision index pi
int make_plan(const glm_shape* s, glm_precision prec_flags, Plan& p, bool allow32 = true,
              bool allow64 = true) {
  int rc = validate(s);
  if (rc != GLM_OK) return rc;
  // GLM_PRECOND_EQ selects D = diag(omega_ii) (x) I_M; the rest is the precision
  const glm_precision prec = (glm_precision)((int)prec_flags & ~(GLM_PRECOND_EQ | GLM_REDUCED));
  p = Plan();
  p.B = s->batch;
  p.prec = prec;
  p.deq = ((int)prec_flags & GLM_PRECOND_EQ) != 0;
  int64_t sum_rows = 0;
  for (int b = 0; b < p.B; ++b) sum_rows += s->M[b];
  // Row tiles of about equal streaming cost (Q row + three vector rows per
  // observation), so that the workgroups of one launch finish together.
  double total_cost = 0.0;
  {
    int64_t off = 0;
    for (int b = 0; b < p.B; ++b) {
      int64_t nb = 0;
      for (int i = 0; i < s->G[b]; ++i) nb += s->n[off + i];
      off += s->G[b];
      total_cost += (double)s->M[b] * (double)(nb + 3 * (int64_t)s->G[b] * s->K[b]);
    }
  }
  const double tile_cost = std::max(kMinTileCost, total_cost / kTargetTiles);
  (void)sum_rows;
  // FP64 solves run in both modes (in the mixed path as the continuation of
  // a refinement the FP32 inner solves no longer advance)
  const bool need32 = prec == GLM_MIXED;
  p.cfg[0] = choose_cfg(s, sizeof(float), allow32 && need32);
  p.cfg[1] = choose_cfg(s, sizeof(double), allow64);
  bool rows_fit[2] = {true, true};
  int64_t noff = 0;
  for (int b = 0; b < p.B; ++b) {
    InstDesc in{};
    in.G = s->G[b];
    in.M = s->M[b];
    in.K = s->K[b];
    in.kc = s->k ? s->k[b] : 0;
    int n = 0;
    for (int i = 0; i < in.G; ++i) {
      n += s->n[noff + i];
      in.nimax = std::max(in.nimax, s->n[noff + i]);
    }
    in.n = n;
    in.blk0 = (int)p.blk.size();
    in.rhs0 = p.nrhs;
    in.q_off = p.sumMn;
    in.v_off = p.sumMGK;
    in.om_off = p.sumG2;
    in.b_off = p.sumnK;
    in.t_off = p.sumTK;
    in.col_off = (int64_t)p.colblk.size();
    in.c_off = p.sumCK;
    in.rc_off = p.sumRc;
    in.nb_off = p.sumNb;
    in.maxit = (int)std::min<int64_t>((int64_t)in.G * in.M + in.kc - n + 1, 1 << 30);
    const size_t per_row = 2 * (size_t)in.G * in.K;
    for (int pi = 1; pi >= 0; --pi) {
      if (pi == 0 && !need32) {   // FP64 only: one configuration
        in.rs_t[0] = in.rs_t[1];
        in.rsa_t[0] = in.rsa_t[1];
        in.rpar_t[0] = in.rpar_t[1];
        in.tps_t[0] = in.tps_t[1];
        continue;
      }
      const size_t svp = pi ? sizeof(double) : sizeof(float);
      PassCfg& c = p.cfg[pi];
      if (c.rowpass) {
        const int P = in.G * in.K;
        // matrix-core passes: 64 / Gp row slots (Gp = G padded to a power of two >= 4)
        const int gp = in.G <= 4 ? 4 : in.G <= 8 ? 8 : in.G <= 16 ? 16 : in.G <= 32 ? 32 : 64;
        int rpar = c.gr < 0 ? 64 / gp : PROJ_NT / (P / c.kv);
        // rows per sub-tile: the three vector slabs of pass B and the Q rows
        // must fit the stager's per-thread registers
        const int rows_v = PROJ_NVB * PROJ_NT * c.kv / (3 * P);
        const int rows_q = PROJ_NQB * PROJ_NT / n;
        int rs = std::min(std::min(rows_v, rows_q), rpar * kRowsPerLane);
        // every row group needs a row per sub-tile: with wide Q rows the
        // vector-ALU mapping keeps as many row groups as rows fit (lanes past
        // them idle); the matrix-core mapping fixes its row groups, and
        // without room for a single row the column-slot passes take over
        if (rs < rpar) {
          if (c.gr >= 0 && rs >= 1) rpar = rs;
          else rows_fit[pi] = false;
        }
        rs = rs / rpar * rpar;   // whole rows per row group
        in.rs_t[pi] = std::max(rs, 1);
        in.rpar_t[pi] = rpar;
        in.tps_t[pi] = c.gr < 0 ? mf_partial_slots(gp) : rpar;
        // pass A: two vector slabs and PROJ_NQA Q scalars per thread
        const int rows_va = PROJ_NV * PROJ_NT * c.kv / (2 * P);
        const int rows_qa = PROJ_NQA * PROJ_NT / n;
        int rsa = std::min(std::min(rows_va, rows_qa), rpar * kRowsPerLane);
        rsa = std::max(rsa / rpar * rpar, in.rs_t[pi]);
        in.rsa_t[pi] = rsa;
      } else {
        in.rs_t[pi] = (int)std::max<size_t>(1, std::min<size_t>(64, kLdsBudget / (per_row * svp)));
        in.rsa_t[pi] = in.rs_t[pi];
        in.rpar_t[pi] = 1;
        in.tps_t[pi] = 1;
        c.lds = std::max(c.lds, per_row * svp * in.rs_t[pi]);
      }
    }
    // blocks
    int col = 0;
    for (int i = 0; i < in.G; ++i) {
      const int ni = s->n[noff + i];
      BlockDesc bd{};
      bd.inst = b;
      bd.eq = i;
      bd.col = col;
      bd.ni = ni;
      bd.r_off = p.sumR;
      p.sumR += (int64_t)ni * ni;
      QRJob qj{};
      qj.a_off = in.q_off + col;
      qj.rows = in.M;
      qj.cols = ni;
      qj.ld = n;
      qj.flag = (int)p.blk.size();
      qj.r_off = bd.r_off;
      p.qr_sur.push_back(qj);
      p.blk.push_back(bd);
      for (int c = 0; c < ni; ++c) p.colblk.push_back(i);
      col += ni;
      p.maxni = std::max(p.maxni, ni);
    }
    noff += in.G;
    // tiles: rows per tile a multiple of both sub-tile heights
    int step = std::max(in.rs_t[0], in.rs_t[1]);
    step = std::max(step, std::max(in.rsa_t[0], in.rsa_t[1]));
    const double row_cost = (double)(n + 3 * in.G * in.K);
    const int want = std::max(kMinTileRows, (int)std::min(1e9, tile_cost / row_cost));
    int trows = std::max(step, (want + step - 1) / step * step);
    in.tile0 = (int)p.tile.size();
    in.tp_stride = std::max<int64_t>(
        (int64_t)std::max(in.tps_t[0], in.tps_t[1]) * n * in.K, (int64_t)in.G * in.G);
    int part = 0;
    for (int r0 = 0; r0 < in.M; r0 += trows) {
      TileDesc td{};
      td.inst = b;
      td.row0 = r0;
      td.rows = std::min(trows, in.M - r0);
      td.part = part++;
      td.tp_off = p.sumTp;
      p.sumTp += in.tp_stride;
      p.tile.push_back(td);
    }
    in.ntiles = part;
    for (int p0 = 0; p0 < n * in.K; p0 += NT) p.chunks.push_back(RedChunk{b, p0});
    if (in.kc > 0) {
      p.rinst_index.push_back((int)p.rinst.size());
      QRJob qj{};
      qj.a_off = in.nb_off;
      qj.rows = n + in.kc;
      qj.cols = in.kc;
      qj.ld = in.kc;
      qj.flag = -1;  // set below
      qj.r_off = -1;
      p.qr_nb.push_back(qj);
      p.rinst.push_back(b);
      p.maxkc = std::max(p.maxkc, in.kc);
    } else {
      p.rinst_index.push_back(-1);
    }
    p.sumMn += (int64_t)in.M * n;
    p.sumMGK += (int64_t)in.M * in.G * in.K;
    p.sumnK += (int64_t)n * in.K;
    p.sumTK += (int64_t)(n + in.kc) * in.K;
    p.sumG2 += (int64_t)in.G * in.G;
    p.sumCK += (int64_t)in.kc * in.K;
    p.sumRc += (int64_t)in.kc * n;
    p.sumNb += (int64_t)(n + in.kc) * in.kc;
    p.nrhs += in.K;
    p.maxK = std::max(p.maxK, in.K);
    p.maxn = std::max(p.maxn, n);
    p.inst.push_back(in);
  }
  // an instance does not suit the row-vector passes of some precision: plan
  // again with the column-slot passes for that precision
  if ((p.cfg[0].rowpass && !rows_fit[0]) || (p.cfg[1].rowpass && !rows_fit[1]))
    return make_plan(s, prec_flags, p, allow32 && rows_fit[0], allow64 && rows_fit[1]);
  p.nblk = (int)p.blk.size();
  p.ntiles = (int)p.tile.size();
  for (size_t r = 0; r < p.qr_nb.size(); ++r) p.qr_nb[r].flag = p.nblk + (int)r;
  p.kc_t = pick_kc(p.maxK);
  const int slots = (p.maxn + NT - 1) / NT;
  p.sl = slots <= 4 ? slots : 8;
  if (p.kc_t > 4 && p.sl == 8) return GLM_EUNSUPPORTED;  // mixed K / n extremes in one batch
  // layout
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return at;
  };
  p.o_Q64 = take(8 * p.sumMn);
  p.o_Q32 = take(prec == GLM_MIXED ? 4 * p.sumMn : 0);
  p.o_R = take(8 * p.sumR);
  p.o_Nb = take(8 * p.sumNb);
  p.o_colblk = take(4 * p.colblk.size());
  p.o_inst = take(sizeof(InstDesc) * p.inst.size());
  p.o_blk = take(sizeof(BlockDesc) * p.blk.size());
  p.o_tile = take(sizeof(TileDesc) * p.tile.size());
  p.o_qrs = take(sizeof(QRJob) * p.qr_sur.size());
  p.o_qrn = take(sizeof(QRJob) * p.qr_nb.size());
  p.o_chunks = take(sizeof(RedChunk) * p.chunks.size());
  p.o_rinst = take(4 * p.rinst.size());
  p.o_rinst_index = take(4 * p.rinst_index.size());
  p.o_flags = take(4 * (p.nblk + p.rinst.size()));
  p.o_active = take(4 * p.B);
  p.o_icount = take(4 * p.B);
  p.o_count = take(16);
  p.o_st = take(sizeof(RhsState) * p.nrhs);
  p.o_ost = take(4 * p.nrhs);
  p.o_alpha = take(8 * p.B);
  p.o_deq = take(8 * (size_t)p.nblk);
  p.o_Om32 = take(prec == GLM_MIXED ? 4 * p.sumG2 : 0);
  // iteration vectors hold FP64 values in both modes (FP32 inner solves use
  // the first half of each)
  p.o_g = take(8 * p.sumMGK);
  p.o_u = take(8 * p.sumMGK);
  p.o_wf = take(prec == GLM_MIXED ? 8 * p.sumMGK : 0);   // inner correction (FP32 or FP64)
  p.o_yf = take(prec == GLM_MIXED ? 4 * p.sumMGK : 0);   // refinement residual, FP32 copy
  p.o_y64 = take(prec == GLM_MIXED ? 8 * p.sumMGK : 0);  // refinement residual, FP64
  p.o_Tpart = take(8 * p.sumTp);
  p.o_Tm = take(8 * p.sumTK);
  p.o_dpart = take(8 * (size_t)p.ntiles * KMAX);
  p.o_cpart = take(8 * (size_t)p.ntiles * KMAX);
  p.o_gc = take(8 * p.sumCK);
  p.o_uc = take(8 * p.sumCK);
  p.o_wc = take(8 * p.sumCK);
  p.o_wc64 = take(8 * p.sumCK);
  p.o_rho0 = take(8 * p.sumnK);
  p.o_rhoc = take(8 * p.sumCK);
  p.o_lb = take(8 * p.sumnK);
  // refinement residual by the FP64 passes: identity blocks, alpha = -1, and
  // the per-tile partial norms of y (fixed over the refinement)
  p.o_eye = take(prec == GLM_MIXED ? 8 * p.sumG2 : 0);
  p.o_mone = take(prec == GLM_MIXED ? 8 * p.B : 0);
  p.o_ypart = take(prec == GLM_MIXED ? 8 * (size_t)p.ntiles * KMAX : 0);
  p.o_bytes = take(2 * sizeof(unsigned long long));
  // normal-equations solver: Omega^-1 (and its work area), r, z and p
  p.o_ne_oinv = take(8 * p.sumG2);
  p.o_ne_a = take(8 * p.sumG2);
  p.o_ne_r = take(8 * p.sumTK);
  p.o_ne_z = take(8 * p.sumTK);
  p.o_ne_p = take(8 * p.sumTK);
  p.total = o;
  return GLM_OK;
}

struct EventPair {
  hipEvent_t a, b;
  int kid;
};

// Launch arguments that differ between the captured iteration chunks of one
// handle (everything else is fixed by the plan and the workspace).
struct GraphKey {
  size_t elem;
  const void *Q, *Om, *y, *w;
  double tol;
  int stall, maxit_cap;
  bool operator==(const GraphKey& o) const {
    return elem == o.elem && Q == o.Q && Om == o.Om && y == o.y && w == o.w && tol == o.tol &&
           stall == o.stall && maxit_cap == o.maxit_cap;
  }
};
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
};

// Iteration chunks run as HIP graphs unless GLM_GRAPHS=0 in the environment.
bool graphs_on() {
  static const bool on = [] {
    const char* v = std::getenv("GLM_GRAPHS");
    return !(v && v[0] == '0');
  }();
  return on;
}

// The pass configuration of a plan in the glm_stats fields (index 0: FP32
// inner solves of the mixed path, -1 when there are none; 1: FP64 solves).
void pass_stats(const Plan& p, glm_stats* st) {
  for (int pi = 0; pi < 2; ++pi) {
    const PassCfg& c = p.cfg[pi];
    const bool used = pi == 1 || p.prec == GLM_MIXED;
    st->pass_rowvec[pi] = used ? c.rowpass : -1;
    st->pass_kv[pi] = used ? c.kv : -1;
    st->pass_ks[pi] = used ? c.ks : -1;
    st->pass_omega[pi] = used ? c.gr : -1;
    st->pass_nim[pi] = used ? c.nim : -1;
  }
}

}  // namespace

namespace {

// Model reduction: per-instance descriptors, the reduced shape (the same
// equations and blocks with min(M, n + 1) observations) and the layout of
// the reduction buffers, followed by the reduced problem's own workspace.
struct RedPlan {
  int B = 0, maxpan = 0, maxn = 0, maxM = 0, maxMr = 0, maxseg = 0;
  int dchunks = 0;   // row chunks of k_red_delta
  std::vector<RedDesc> d;
  // the device copy of the descriptors, tallest instance first: every
  // reduction kernel takes its instance from its descriptor, so the order
  // only sets the launch order, and the sequential panel kernel then
  // schedules the longest jobs first
  std::vector<RedDesc> d_dev;
  // output tiles of Q1^T Y (t1) and of Q1 D (t2), grouped by XCD
  std::vector<GemmTile> t1, t2;
  std::vector<int32_t> G, M, K, k, n;
  // common regressors: W is Z0 (N_b columns) and the reduced regressors of
  // equation i are the columns sel of R (sum of n_i entries per instance)
  bool common = false;
  std::vector<int32_t> sel;
  glm_shape sub{};
  int64_t sumMn = 0, sumMGK = 0, sumMrn = 0, sumMrGK = 0, sumn = 0, sumT = 0, sumG2 = 0,
          sumZp = 0, sumMMr = 0, sumnK = 0, sumLeaf = 0;
  double gemm1_bytes = 0.0;   // algorithmic bytes of one Q1^T Y over the batch
  size_t o_desc = 0, o_W = 0, o_tau = 0, o_T = 0, o_Tleaf = 0, o_Stk = 0, o_Q1 = 0, o_Xr = 0,
         o_yr = 0, o_ur = 0,
         o_dd = 0, o_Og = 0, o_Ow = 0, o_sing = 0, o_t1 = 0, o_t2 = 0, o_Zp = 0, o_lb = 0,
         o_cexp = 0, o_sel = 0, o_sub = 0, sub_bytes = 0, total = 0;
};

// Tile table of a batched product: every instance's output tiles (rows x
// cols in 64 x 64 tiles) go to one XCD, chosen greedily by the work already
// there (weight per tile `w`, instances in device order), and workgroup x of
// the launch runs on XCD x mod 8: an instance's tiles share one L2.
std::vector<GemmTile> xcd_tiles(const std::vector<RedDesc>& dd, bool out_rows_full) {
  constexpr int kXcd = 8;
  std::vector<std::vector<GemmTile>> lists(kXcd);
  double load[kXcd] = {0};
  for (int q = 0; q < (int)dd.size(); ++q) {
    const RedDesc& d = dd[q];
    const int rows = out_rows_full ? d.M : d.Mr, cols = d.G * d.K;
    const double w = out_rows_full ? (double)d.Mr : (double)d.M;   // reduction length
    int x = 0;
    for (int c = 1; c < kXcd; ++c)
      if (load[c] < load[x]) x = c;
    for (int i0 = 0; i0 < rows; i0 += 64)
      for (int j0 = 0; j0 < cols; j0 += 64) {
        lists[x].push_back(GemmTile{q, i0, j0, 0});
        load[x] += w;
      }
  }
  size_t lmax = 0;
  for (const auto& l : lists) lmax = std::max(lmax, l.size());
  std::vector<GemmTile> out(lmax * kXcd, GemmTile{-1, 0, 0, 0});
  for (int x = 0; x < kXcd; ++x)
    for (size_t q = 0; q < lists[x].size(); ++q) out[q * kXcd + x] = lists[x][q];
  return out;
}

// wcols (host [B], or null): common regressors Z0 with wcols[b] columns,
// equation i keeping the columns sel (host, sum of n_i entries per instance,
// strictly increasing within an equation, each below wcols[b])
int make_red_plan(const glm_shape* s, glm_precision base, RedPlan& r,
                  const int32_t* wcols = nullptr, const int32_t* sel = nullptr) {
  int rc = validate(s);
  if (rc != GLM_OK) return rc;
  if (wcols && !sel) return GLM_EINVAL;
  r = RedPlan();
  r.B = s->batch;
  r.common = wcols != nullptr;
  int64_t noff = 0, rhs = 0, om = 0;
  for (int b = 0; b < r.B; ++b) {
    RedDesc d{};
    d.M = s->M[b];
    d.G = s->G[b];
    d.K = s->K[b];
    d.inst = b;
    int nsub = 0;
    for (int i = 0; i < d.G; ++i) nsub += s->n[noff + i];
    d.nsub = nsub;
    int n = nsub;
    if (wcols) {
      n = wcols[b];
      if (n < 1 || n > NMAX_INST) return n < 1 ? GLM_EINVAL : GLM_EUNSUPPORTED;
      d.sel_off = (int)r.sel.size();
      for (int i = 0; i < d.G; ++i) {
        const int ni = s->n[noff + i];
        if (ni > n) return GLM_EINVAL;
        for (int c = 0; c < ni; ++c) {
          const int v = sel[r.sel.size()];
          if (v < 0 || v >= n || (c > 0 && v <= r.sel.back())) return GLM_EINVAL;
          r.sel.push_back(v);
        }
      }
    }
    d.n = n;
    {
      // one row of X and Y must fit the full-model u kernel's LDS
      const int rowlds = RED_U_LDS - (d.G <= 32 ? d.G * d.G : 0);
      if (n + d.G * d.K > rowlds) return GLM_EUNSUPPORTED;
    }
    d.Mr = std::min(d.M, n + 1);
    d.kr = std::min(d.M, n);
    d.rhs0 = (int)rhs;
    d.w_off = r.sumMn;
    d.q1_off = r.sumMMr;
    d.b_off = r.sumnK;
    d.v_off = r.sumMGK;
    d.xr_off = r.sumMrn;
    d.vr_off = r.sumMrGK;
    d.tau_off = r.sumn;
    d.t_off = r.sumT;
    d.om_off = om;
    d.zp_off = r.sumZp;
    const int npan = (d.kr + RED_PANEL - 1) / RED_PANEL;
    d.nseg0 = (d.M + RED_LEAF - 1) / RED_LEAF;
    d.leaf_off = r.sumLeaf;
    d.stk_off = r.sumLeaf;
    r.sumLeaf += (int64_t)npan * d.nseg0 * RED_PANEL * RED_PANEL;
    r.maxseg = std::max(r.maxseg, d.nseg0);
    const int P = d.G * d.K;
    const int rows = std::max(1, std::min(32, 4096 / P));
    r.dchunks = std::max(r.dchunks, (d.Mr + rows - 1) / rows);
    r.maxpan = std::max(r.maxpan, npan);
    r.maxn = std::max(r.maxn, n);
    r.maxM = std::max(r.maxM, d.M);
    r.maxMr = std::max(r.maxMr, d.Mr);
    r.sumMn += (int64_t)d.M * n;
    r.sumMMr += (int64_t)d.M * d.Mr;
    r.sumnK += (int64_t)nsub * d.K;
    r.sumMGK += (int64_t)d.M * P;
    r.sumMrn += (int64_t)d.Mr * nsub;
    r.sumMrGK += (int64_t)d.Mr * P;
    r.sumn += n;
    r.sumT += (int64_t)npan * RED_PANEL * RED_PANEL;
    r.sumZp += (int64_t)((d.M + RED_SEG - 1) / RED_SEG) * d.G * d.G;
    r.gemm1_bytes += 8.0 * ((double)d.M * d.Mr + (double)d.M * P + (double)d.Mr * P);
    om += (int64_t)d.G * d.G;
    r.sumG2 = om;
    rhs += d.K;
    r.d.push_back(d);
    r.G.push_back(d.G);
    r.M.push_back(d.Mr);
    r.K.push_back(d.K);
    r.k.push_back(s->k ? s->k[b] : 0);
    noff += d.G;
  }
  r.n.assign(s->n, s->n + noff);
  r.d_dev = r.d;
  std::stable_sort(r.d_dev.begin(), r.d_dev.end(),
                   [](const RedDesc& a, const RedDesc& b) { return a.M > b.M; });
  r.t1 = xcd_tiles(r.d_dev, false);
  r.t2 = xcd_tiles(r.d_dev, true);
  r.sub.batch = r.B;
  r.sub.G = r.G.data();
  r.sub.M = r.M.data();
  r.sub.K = r.K.data();
  r.sub.k = r.k.data();
  r.sub.n = r.n.data();
  rc = validate(&r.sub);
  if (rc != GLM_OK) return rc;
  Plan sp;
  rc = make_plan(&r.sub, base, sp);
  if (rc != GLM_OK) return rc;
  r.sub_bytes = sp.total;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return at;
  };
  r.o_desc = take(sizeof(RedDesc) * r.d.size());
  r.o_t1 = take(sizeof(GemmTile) * r.t1.size());
  r.o_t2 = take(sizeof(GemmTile) * r.t2.size());
  r.o_W = take(8 * r.sumMn);
  r.o_tau = take(8 * r.sumn);
  r.o_cexp = take(4 * r.sumn);
  r.o_sel = take(4 * r.sel.size());
  r.o_T = take(8 * r.sumT);
  r.o_Tleaf = take(8 * r.sumLeaf);
  r.o_Stk = take(8 * r.sumLeaf);
  r.o_Q1 = take(8 * r.sumMMr);
  r.o_Xr = take(8 * r.sumMrn);
  r.o_yr = take(8 * r.sumMrGK);
  r.o_ur = take(8 * r.sumMrGK);
  r.o_dd = take(8 * r.sumMrGK);
  r.o_Og = take(8 * r.sumG2);
  r.o_Ow = take(8 * r.sumG2);
  r.o_sing = take(4 * (size_t)r.B);
  r.o_Zp = take(8 * r.sumZp);
  r.o_lb = take(8 * r.sumnK);
  r.o_sub = take(r.sub_bytes);
  r.total = o;
  return GLM_OK;
}

}  // namespace

struct glm_factor {
  Plan p;
  bool reduced = false;
  RedPlan rp;
  glm_factor* sub = nullptr;   // factor of the reduced problem
  char* ws = nullptr;
  const double* X = nullptr;
  const double* Rc = nullptr;
  int* h_count = nullptr;   // pinned, or h_count_host when pinned memory is not wanted
  bool h_count_pinned = false;
  int h_count_host[4] = {0, 0, 0, 0};
  // HIP graphs of the iteration chunks, keyed by their launch arguments, and
  // the private stream they are captured on (never on the caller's stream,
  // which may be the null stream)
  bool use_graphs = false;
  hipStream_t cap_stream = nullptr;
  std::vector<GraphEntry> graphs;
  glm_stats stats{};
  bool prof = false;
  std::vector<EventPair> ev_used, ev_free;
  int64_t prof_launch[3] = {0, 0, 0};
  double prof_ms[3] = {0, 0, 0};
  double prof_bytes_host = 0.0;   // reduced handle: algorithmic bytes of the timed applies
  int launches = 0;

  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
  const InstDesc* d_inst() const { return at<InstDesc>(p.o_inst); }
  const TileDesc* d_tile() const { return at<TileDesc>(p.o_tile); }
  const BlockDesc* d_blk() const { return at<BlockDesc>(p.o_blk); }
  int* d_active() const { return at<int>(p.o_active); }
  RhsState* d_st() const { return at<RhsState>(p.o_st); }
};

namespace {

#define GLM_CHECK(expr)                        \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return GLM_EHIP;     \
  } while (0)

EventPair get_event(glm_factor* f, int kid) {
  EventPair e;
  if (!f->ev_free.empty()) {
    e = f->ev_free.back();
    f->ev_free.pop_back();
  } else {
    (void)hipEventCreate(&e.a);
    (void)hipEventCreate(&e.b);
  }
  e.kid = kid;
  return e;
}

template <typename T>
PassLaunch<T> pass_args(glm_factor* f, const T* Q, const T* Om, const T* y, T* w, T* g, T* u,
                        bool prof) {
  const Plan& p = f->p;
  PassLaunch<T> a{};
  a.insts = f->d_inst();
  a.tiles = f->d_tile();
  a.ntiles = p.ntiles;
  a.blks = f->d_blk();
  a.colblk = f->at<int>(p.o_colblk);
  a.inst_active = f->d_active();
  a.Q = Q;
  a.Om = Om;
  a.alpha = f->at<double>(p.o_alpha);
  a.deq = p.deq ? f->at<double>(p.o_deq) : nullptr;
  a.st = f->d_st();
  a.y = y;
  a.w = w;
  a.g = g;
  a.u = u;
  a.Tm = f->at<T>(p.o_Tm);
  a.Tpart = f->at<T>(p.o_Tpart);
  a.dpart = f->at<double>(p.o_dpart);
  a.cpart = f->at<double>(p.o_cpart);
  a.bytes = prof ? f->at<unsigned long long>(p.o_bytes) : nullptr;
  a.w_nonzero = 0;
  a.kc_t = p.kc_t;
  a.sl = p.sl;
  const PassCfg& c = p.cfg[sizeof(T) == 8];
  a.lds = c.lds;
  a.rowpass = c.rowpass;
  a.kv = c.kv;
  a.ks = c.ks;
  a.gr = c.gr;
  a.nim = c.nim;
  return a;
}

template <typename T>
int run_pass_a(glm_factor* f, PassLaunch<T> a, int mode, hipStream_t s) {
  const bool timed = f->prof && mode == PASS_A_ITER;
  EventPair e{};
  if (timed) {
    e = get_event(f, 0);
    GLM_CHECK(hipEventRecord(e.a, s));
    a.bytes = f->at<unsigned long long>(f->p.o_bytes);
  } else {
    a.bytes = nullptr;
  }
  GLM_CHECK(a.rowpass ? launch_proj<T>(a, true, mode, s) : launch_pass_a<T>(a, mode, s));
  ++f->launches;
  if (timed) {
    GLM_CHECK(hipEventRecord(e.b, s));
    f->ev_used.push_back(e);
  }
  return GLM_OK;
}

template <typename T>
int run_pass_b(glm_factor* f, PassLaunch<T> a, int mode, hipStream_t s) {
  const bool timed = f->prof && mode == PASS_B_ITER;
  EventPair e{};
  if (timed) {
    e = get_event(f, 1);
    GLM_CHECK(hipEventRecord(e.a, s));
    a.bytes = f->at<unsigned long long>(f->p.o_bytes) + 1;
  } else {
    a.bytes = nullptr;
  }
  GLM_CHECK(a.rowpass ? launch_proj<T>(a, false, mode, s) : launch_pass_b<T>(a, mode, s));
  ++f->launches;
  if (timed) {
    GLM_CHECK(hipEventRecord(e.b, s));
    f->ev_used.push_back(e);
  }
  return GLM_OK;
}

// Projection  T <- [Q^T (y - Sigma w) ; r]  followed by the restriction correction.
template <typename T>
int project_rhs(glm_factor* f, const T* Q, const T* Om, const T* y, T* w, bool w_nonzero,
                const double* rvec, hipStream_t s) {
  const Plan& p = f->p;
  PassLaunch<T> a = pass_args<T>(f, Q, Om, y, w, nullptr, nullptr, false);
  a.w_nonzero = w_nonzero;
  if (int rc = run_pass_a<T>(f, a, PASS_A_RHS, s)) return rc;
  GLM_CHECK(launch_reduce_t<T>(f->d_inst(), f->d_tile(), f->d_active(),
                               f->at<RedChunk>(p.o_chunks), (int)p.chunks.size(),
                               f->at<T>(p.o_Tpart), f->at<T>(p.o_Tm),
                               p.cfg[sizeof(T) == 8].rowpass, s));
  GLM_CHECK(launch_scalar_a<T>(f->d_inst(), f->d_tile(), f->d_active(), f->d_st(),
                               f->at<double>(p.o_dpart), f->at<T>(p.o_Tm),
                               f->at<double>(p.o_Nb), rvec, p.B, 0, 0, s));
  f->launches += 3;
  return GLM_OK;
}

// One PCG-Aug solve of [Sigma X; X^T 0][w; beta] = [y; h2] (+ restriction rows r)
// in precision T for every (instance, rhs) whose state is ST_ACTIVE.
// beta_out receives (or, with beta_add, accumulates) the estimate.
template <typename T>
int core_solve(glm_factor* f, const T* Q, const T* Om, const T* y, const double* h2,
               const double* rvec, T* w, double* beta_out, bool beta_add, double tol,
               int stall, int maxit_cap, hipStream_t s) {
  const Plan& p = f->p;
  T* g = f->at<T>(p.o_g);
  T* u = f->at<T>(p.o_u);
  T* Tm = f->at<T>(p.o_Tm);
  double* gc = f->at<double>(p.o_gc);
  double* uc = f->at<double>(p.o_uc);
  double* wc = f->at<double>(p.o_wc);
  const bool t_double = sizeof(T) == 8;
  // start: w_1 = X* h2 (zero without a lower right-hand side)
  GLM_CHECK(launch_fill<T>(w, p.sumMGK, T(0), s));
  GLM_CHECK(launch_fill<double>(wc, std::max<int64_t>(p.sumCK, 0), 0.0, s));
  f->launches += 2;
  bool w_nonzero = false;
  if (h2) {
    GLM_CHECK((launch_trisolve<double, T, false, false>(f->d_inst(), f->d_blk(), p.nblk,
                                                        f->d_active(), f->d_st(), 1,
                                                        f->at<double>(p.o_R), h2, 0, Tm, 1, s)));
    GLM_CHECK(launch_scalar_a<T>(f->d_inst(), f->d_tile(), f->d_active(), f->d_st(),
                                 f->at<double>(p.o_dpart), Tm, f->at<double>(p.o_Nb), nullptr,
                                 p.B, 1, 0, s));
    PassLaunch<T> a = pass_args<T>(f, Q, Om, y, w, g, u, false);
    if (int rc = run_pass_b<T>(f, a, PASS_B_EXPAND, s)) return rc;
    if (p.sumCK) GLM_CHECK(launch_copy_tc<T>(f->d_inst(), p.B, Tm, wc, s));
    f->launches += 3;
    w_nonzero = true;
  }
  // g_1 = -Pi (y - Sigma w_1), c_1
  if (int rc = project_rhs<T>(f, Q, Om, y, w, w_nonzero, rvec, s)) return rc;
  {
    PassLaunch<T> a = pass_args<T>(f, Q, Om, y, w, g, u, false);
    a.w_nonzero = w_nonzero;
    if (int rc = run_pass_b<T>(f, a, PASS_B_INIT, s)) return rc;
  }
  GLM_CHECK(launch_scalar_b(f->d_inst(), f->d_active(), f->at<int>(p.o_icount), f->d_st(),
                            f->at<double>(p.o_cpart), f->at<double>(p.o_alpha), Tm, t_double,
                            gc, uc, wc, rvec, p.B, 0, tol, stall, maxit_cap, s));
  ++f->launches;
  // iterations
  int64_t maxit_all = 0;
  for (const auto& in : p.inst) maxit_all = std::max<int64_t>(maxit_all, in.maxit);
  if (maxit_cap > 0) maxit_all = std::min<int64_t>(maxit_all, maxit_cap);
  PassLaunch<T> aa = pass_args<T>(f, Q, Om, y, w, g, u, false);
  // one PCG iteration: pass A, the sum of its partials, lambda, pass B, mu and
  // the stopping tests; every kernel reads the (instance, rhs) states, so an
  // iteration after convergence does nothing
  auto iteration = [&](hipStream_t st) -> int {
    if (int rc = run_pass_a<T>(f, aa, PASS_A_ITER, st)) return rc;
    GLM_CHECK(launch_reduce_t<T>(f->d_inst(), f->d_tile(), f->d_active(),
                                 f->at<RedChunk>(p.o_chunks), (int)p.chunks.size(),
                                 f->at<T>(p.o_Tpart), Tm,
                                 p.cfg[sizeof(T) == 8].rowpass, st));
    GLM_CHECK(launch_scalar_a<T>(f->d_inst(), f->d_tile(), f->d_active(), f->d_st(),
                                 f->at<double>(p.o_dpart), Tm, f->at<double>(p.o_Nb),
                                 nullptr, p.B, 1, 1, st));
    if (int rc = run_pass_b<T>(f, aa, PASS_B_ITER, st)) return rc;
    GLM_CHECK(launch_scalar_b(f->d_inst(), f->d_active(), f->at<int>(p.o_icount), f->d_st(),
                              f->at<double>(p.o_cpart), f->at<double>(p.o_alpha), Tm,
                              t_double, gc, uc, wc, nullptr, p.B, 1, tol, stall, maxit_cap,
                              st));
    f->launches += 3;
    return GLM_OK;
  };
  // the kPollEvery iterations between two polls, captured once per argument
  // set in a HIP graph and replayed (not while the kernel timers run, whose
  // events sit between the launches)
  hipGraphExec_t chunk = nullptr;
  if (f->use_graphs && !f->prof) {
    const GraphKey key{sizeof(T), Q, Om, y, w, tol, stall, maxit_cap};
    for (const auto& ge : f->graphs)
      if (ge.key == key) chunk = ge.exec;
    if (!chunk) {
      if (!f->cap_stream)
        GLM_CHECK(hipStreamCreateWithFlags(&f->cap_stream, hipStreamNonBlocking));
      GLM_CHECK(hipStreamBeginCapture(f->cap_stream, hipStreamCaptureModeThreadLocal));
      int rc = GLM_OK;
      const int l0 = f->launches;
      for (int j = 0; j < kPollEvery && rc == GLM_OK; ++j) rc = iteration(f->cap_stream);
      f->launches = l0;
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(f->cap_stream, &graph);
      if (rc != GLM_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc != GLM_OK ? rc : GLM_EHIP;
      }
      const hipError_t ei = hipGraphInstantiate(&chunk, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return GLM_EHIP;
      f->graphs.push_back(GraphEntry{key, chunk});
    }
  }
  for (int64_t it = 0; it < maxit_all + 1; it += kPollEvery) {
    GLM_CHECK(launch_count(f->at<int>(p.o_icount), p.B, f->at<int>(p.o_count), s));
    GLM_CHECK(hipMemcpyAsync(f->h_count, f->at<int>(p.o_count), sizeof(int),
                             hipMemcpyDeviceToHost, s));
    GLM_CHECK(hipStreamSynchronize(s));
    if (log_on() && (it % (kPollEvery * 16) == 0 || *f->h_count == 0))
      std::fprintf(stderr, "[glm %.3fs] %s pcg it %lld active rhs %d\n", now_s(),
                   sizeof(T) == 8 ? "fp64" : "fp32", (long long)it, *f->h_count);
    if (*f->h_count == 0) break;
    if (chunk) {
      GLM_CHECK(hipGraphLaunch(chunk, s));
      f->launches += 5 * kPollEvery;
    } else {
      // iterations past the bound are stopped by the per-rhs limits on the device
      const int64_t nit = std::min<int64_t>(kPollEvery, maxit_all + 1 - it);
      for (int64_t j = 0; j < nit; ++j)
        if (int rc = iteration(s)) return rc;
    }
  }
  // termination: beta = X*^T (y - Sigma w) for every solved rhs
  GLM_CHECK(launch_activate(f->d_inst(), p.B, f->d_st(), f->d_active(), s));
  if (int rc = project_rhs<T>(f, Q, Om, y, w, true, rvec, s)) return rc;
  if (beta_add) {
    GLM_CHECK((launch_trisolve<T, double, true, true>(f->d_inst(), f->d_blk(), p.nblk,
                                                      f->d_active(), f->d_st(), 1,
                                                      f->at<double>(p.o_R), Tm, 1, beta_out,
                                                      0, s)));
  } else {
    GLM_CHECK((launch_trisolve<T, double, true, false>(f->d_inst(), f->d_blk(), p.nblk,
                                                       f->d_active(), f->d_st(), 1,
                                                       f->at<double>(p.o_R), Tm, 1, beta_out,
                                                       0, s)));
  }
  f->launches += 2;
  return GLM_OK;
}

int map_info_and_stats(glm_factor* f, int32_t* info, int32_t* iters, bool mixed,
                       hipStream_t s) {
  const Plan& p = f->p;
  std::vector<RhsState> st(p.nrhs);
  std::vector<int> ost(p.nrhs, 0);
  GLM_CHECK(hipMemcpyAsync(st.data(), f->d_st(), sizeof(RhsState) * p.nrhs,
                           hipMemcpyDeviceToHost, s));
  if (mixed)
    GLM_CHECK(hipMemcpyAsync(ost.data(), f->at<int>(p.o_ost), 4 * p.nrhs,
                             hipMemcpyDeviceToHost, s));
  GLM_CHECK(hipStreamSynchronize(s));
  std::vector<int32_t> hinfo(p.nrhs), hit(p.nrhs);
  int64_t tot = 0;
  int mx = 0;
  for (int r = 0; r < p.nrhs; ++r) {
    const int stt = mixed ? ost[r] : st[r].status;
    int code;
    switch (stt) {
      case ST_CONVERGED: code = GLM_INFO_CONVERGED; break;
      case ST_STAGNATED: code = GLM_INFO_STAGNATED; break;
      case ST_BREAKDOWN: code = GLM_INFO_BREAKDOWN; break;
      case ST_RANK: code = GLM_INFO_RANK; break;
      default: code = GLM_INFO_NOCONV; break;
    }
    hinfo[r] = code;
    hit[r] = st[r].total_iters;
    tot += st[r].total_iters;
    mx = std::max(mx, st[r].total_iters);
  }
  f->stats.pcg_iterations = tot;
  f->stats.max_iterations = mx;
  if (info)
    GLM_CHECK(hipMemcpyAsync(info, hinfo.data(), 4 * p.nrhs, hipMemcpyHostToDevice, s));
  if (iters)
    GLM_CHECK(hipMemcpyAsync(iters, hit.data(), 4 * p.nrhs, hipMemcpyHostToDevice, s));
  GLM_CHECK(hipStreamSynchronize(s));
  return GLM_OK;
}

// Common driver of solve and backward: y (may be null = 0), h2 (may be null),
// rvec (may be null) -> beta_out, u_out (double), uc_out (may be null).
int solve_driver(glm_factor* f, const double* Om, const double* y, const double* h2,
                 const double* rvec, double tol, int32_t max_iter, double* beta_out,
                 double* u_out, double* uc_out, int32_t* info, int32_t* iters, hipStream_t s) {
  const Plan& p = f->p;
  f->launches = 0;
  f->stats = glm_stats{};
  const bool mixed = p.prec == GLM_MIXED;
  pass_stats(p, &f->stats);
  GLM_CHECK(launch_alpha(f->d_inst(), p.B, Om, f->at<double>(p.o_alpha),
                         mixed ? f->at<float>(p.o_Om32) : nullptr,
                         p.deq ? f->at<double>(p.o_deq) : nullptr, s));
  GLM_CHECK(launch_state_init(f->d_inst(), p.B, f->at<int>(p.o_flags), p.nblk,
                              f->at<int>(p.o_rinst_index), f->d_st(), f->d_active(),
                              f->at<int>(p.o_ost), s));
  GLM_CHECK(launch_fill<double>(beta_out, p.sumnK, 0.0, s));
  f->launches += 3;
  if (!mixed) {
    int rc = core_solve<double>(f, f->at<double>(p.o_Q64), Om, y, h2, rvec, u_out, beta_out,
                                false, tol, kStallFP64, max_iter, s);
    if (rc) return rc;
    f->stats.outer_steps = 1;
    if (uc_out && p.sumCK)
      GLM_CHECK(hipMemcpyAsync(uc_out, f->at<double>(p.o_wc), 8 * p.sumCK,
                               hipMemcpyDeviceToDevice, s));
  } else {
    double* wc64 = f->at<double>(p.o_wc64);
    GLM_CHECK(launch_fill<double>(u_out, p.sumMGK, 0.0, s));
    GLM_CHECK(launch_fill<double>(wc64, std::max<int64_t>(p.sumCK, 0), 0.0, s));
    f->launches += 2;
    float* yf = f->at<float>(p.o_yf);
    double* y64 = f->at<double>(p.o_y64);
    double* Tm64 = f->at<double>(p.o_Tm);
    GLM_CHECK(launch_eye(f->d_inst(), p.B, f->at<double>(p.o_eye), s));
    GLM_CHECK(launch_fill<double>(f->at<double>(p.o_mone), p.B, -1.0, s));
    f->launches += 2;
    int step = 0;
    for (step = 0; step <= kMaxOuter; ++step) {
      // Double-precision residual of the augmented system with the FP64
      // passes, X in place of Q:
      //   rho_y = y - W Omega - X beta   (pass B, INIT form, with T := beta
      //           and alpha := -1; its c partials are ||rho_y||^2)
      //   X^T W                          (pass A, RHS form, with y := 0 and
      //           Omega := I, which yields -X^T W)
      GLM_CHECK(launch_select_inner(f->d_inst(), p.B, f->d_st(), f->at<int>(p.o_ost),
                                    f->d_active(), -2, s));
      GLM_CHECK(launch_beta_to_t(f->d_inst(), p.B, beta_out, Tm64, s));
      f->launches += 2;
      {
        PassLaunch<double> a = pass_args<double>(f, f->X, Om, y, u_out, y64, nullptr, false);
        a.alpha = f->at<double>(p.o_mone);
        a.deq = nullptr;
        a.w_nonzero = step > 0;
        if (int rc = run_pass_b<double>(f, a, PASS_B_INIT, s)) return rc;
      }
      if (step == 0)   // rho_y = y: keep the partial norms of y
        GLM_CHECK(hipMemcpyAsync(f->at<double>(p.o_ypart), f->at<double>(p.o_cpart),
                                 8 * (size_t)p.ntiles * KMAX, hipMemcpyDeviceToDevice, s));
      {
        PassLaunch<double> a = pass_args<double>(f, f->X, f->at<double>(p.o_eye), nullptr,
                                                 u_out, nullptr, nullptr, false);
        a.w_nonzero = 1;
        if (int rc = run_pass_a<double>(f, a, PASS_A_RHS, s)) return rc;
      }
      GLM_CHECK(launch_reduce_t<double>(f->d_inst(), f->d_tile(), f->d_active(),
                                        f->at<RedChunk>(p.o_chunks), (int)p.chunks.size(),
                                        f->at<double>(p.o_Tpart), Tm64,
                                        p.cfg[1].rowpass, s));
      GLM_CHECK(launch_to_float(y64, yf, p.sumMGK, s));
      GLM_CHECK(launch_outer_check(f->d_inst(), f->d_blk(), f->at<double>(p.o_R), p.B,
                                   f->d_active(), f->d_st(),
                                   f->at<int>(p.o_ost), f->at<double>(p.o_cpart),
                                   f->at<double>(p.o_ypart), Tm64, -1.0, h2, f->Rc, rvec,
                                   beta_out, wc64, f->at<double>(p.o_rho0),
                                   f->at<double>(p.o_rhoc), tol, step, step == kMaxOuter, s));
      f->launches += 3;
      // anything left?
      GLM_CHECK(launch_count(f->d_active(), p.B, f->at<int>(p.o_count), s));
      GLM_CHECK(hipMemcpyAsync(f->h_count, f->at<int>(p.o_count), sizeof(int),
                               hipMemcpyDeviceToHost, s));
      GLM_CHECK(hipStreamSynchronize(s));
      if (log_on()) {
        RhsState h0{};
        GLM_CHECK(hipMemcpy(&h0, f->d_st(), sizeof(RhsState), hipMemcpyDeviceToHost));
        std::fprintf(stderr,
                     "[glm %.3fs] refinement step %d: %d instances need work; first rhs: "
                     "relative residual %.3e after %d inner iterations\n",
                     now_s(), step, *f->h_count, std::sqrt(h0.rnorm2 / h0.ynorm2),
                     h0.total_iters);
      }
      if (*f->h_count == 0) break;
      // inner solves: FP32 for the rhs it still advances, FP64 for the others
      for (int want = 0; want < 2; ++want) {
        GLM_CHECK(launch_select_inner(f->d_inst(), p.B, f->d_st(), f->at<int>(p.o_ost),
                                      f->d_active(), want, s));
        GLM_CHECK(launch_count(f->d_active(), p.B, f->at<int>(p.o_count), s));
        GLM_CHECK(hipMemcpyAsync(f->h_count, f->at<int>(p.o_count), sizeof(int),
                                 hipMemcpyDeviceToHost, s));
        GLM_CHECK(hipStreamSynchronize(s));
        f->launches += 2;
        if (*f->h_count == 0) continue;
        const double* rhoc = p.sumCK ? f->at<double>(p.o_rhoc) : nullptr;
        if (want == 0) {
          float* wf = f->at<float>(p.o_wf);
          int rc = core_solve<float>(f, f->at<float>(p.o_Q32), f->at<float>(p.o_Om32), yf,
                                     f->at<double>(p.o_rho0), rhoc, wf, beta_out, true,
                                     kInnerTol, kStallInner,
                                     (max_iter > 0 && max_iter < kInnerMaxit) ? max_iter
                                                                              : kInnerMaxit,
                                     s);
          if (rc) return rc;
          GLM_CHECK(launch_update_u<float>(f->d_inst(), f->d_tile(), p.ntiles, f->d_active(),
                                           f->d_st(), wf, u_out, s));
        } else {
          if (log_on())
            std::fprintf(stderr, "[glm %.3fs] refinement step %d: %d instances continue in FP64\n",
                         now_s(), step, *f->h_count);
          double* w64 = f->at<double>(p.o_wf);
          int rc = core_solve<double>(f, f->at<double>(p.o_Q64), Om, y64,
                                      f->at<double>(p.o_rho0), rhoc, w64, beta_out, true,
                                      kInnerTol, kStallFP64, max_iter, s);
          if (rc) return rc;
          GLM_CHECK(launch_update_u<double>(f->d_inst(), f->d_tile(), p.ntiles, f->d_active(),
                                            f->d_st(), w64, u_out, s));
        }
        if (p.sumCK)
          GLM_CHECK(launch_update_c(f->d_inst(), p.B, f->d_st(), f->at<double>(p.o_wc), wc64, s));
        f->launches += 2;
      }
      // the next refinement residual covers every rhs still refining
      GLM_CHECK(launch_select_inner(f->d_inst(), p.B, f->d_st(), f->at<int>(p.o_ost),
                                    f->d_active(), -1, s));
      ++f->launches;
    }
    f->stats.outer_steps = step;
    if (uc_out && p.sumCK)
      GLM_CHECK(hipMemcpyAsync(uc_out, wc64, 8 * p.sumCK, hipMemcpyDeviceToDevice, s));
  }
  f->stats.launches = f->launches;
  return map_info_and_stats(f, info, iters, mixed, s);
}

// PCG-NE (CG on the normal equations, block-Jacobi preconditioner) on an
// unreduced handle in double precision.  The products with the normal
// matrix run on the projection passes with X in place of Q and Omega^-1 in
// place of Omega:
//   T = X^T (0 - w Omega^-1)   pass A, RHS form (w := X p; -b with w := y)
//   w = X T                    pass B, EXPAND form with T := p
int ne_driver(glm_factor* f, const double* Om, const double* y, double tol, int32_t max_iter,
              double* beta, int32_t* info, int32_t* iters, hipStream_t s) {
  const Plan& p = f->p;
  if (p.sumCK > 0) return GLM_EUNSUPPORTED;
  f->launches = 0;
  f->stats = glm_stats{};
  pass_stats(p, &f->stats);
  double* Oinv = f->at<double>(p.o_ne_oinv);
  double* w = f->at<double>(p.o_g);
  double* Tm = f->at<double>(p.o_Tm);
  double* rv = f->at<double>(p.o_ne_r);
  double* zv = f->at<double>(p.o_ne_z);
  double* pv = f->at<double>(p.o_ne_p);
  int* icount = f->at<int>(p.o_icount);
  GLM_CHECK(launch_state_init(f->d_inst(), p.B, f->at<int>(p.o_flags), p.nblk,
                              f->at<int>(p.o_rinst_index), f->d_st(), f->d_active(), nullptr,
                              s));
  GLM_CHECK(launch_ne_oinv(f->d_inst(), p.B, Om, f->at<double>(p.o_ne_a), Oinv, f->d_st(),
                           f->d_active(), s));
  GLM_CHECK(launch_fill<double>(w, p.sumMGK, 0.0, s));
  f->launches += 3;
  auto normal_product = [&](const double* wsrc) -> int {
    // the RHS form only reads w
    PassLaunch<double> a =
        pass_args<double>(f, f->X, Oinv, nullptr, const_cast<double*>(wsrc), nullptr, nullptr,
                          false);
    a.deq = nullptr;
    a.w_nonzero = 1;
    if (int rc = run_pass_a<double>(f, a, PASS_A_RHS, s)) return rc;
    GLM_CHECK(launch_reduce_t<double>(f->d_inst(), f->d_tile(), f->d_active(),
                                      f->at<RedChunk>(p.o_chunks), (int)p.chunks.size(),
                                      f->at<double>(p.o_Tpart), Tm, p.cfg[1].rowpass, s));
    ++f->launches;
    return GLM_OK;
  };
  // T = -X^T Sigma^-1 y, then r = b, z, p, rho
  if (int rc = normal_product(y)) return rc;
  GLM_CHECK(launch_ne_start(f->d_inst(), f->d_blk(), p.B, f->at<double>(p.o_R), Oinv, Tm, beta,
                            rv, zv, pv, f->d_st(), f->d_active(), icount, s));
  ++f->launches;
  int64_t maxit_all = 0;
  for (const auto& in : p.inst)
    maxit_all = std::max<int64_t>(maxit_all, max_iter > 0 ? max_iter : in.n);
  for (int64_t it = 0; it < maxit_all; it += kPollEvery) {
    GLM_CHECK(launch_count(icount, p.B, f->at<int>(p.o_count), s));
    GLM_CHECK(hipMemcpyAsync(f->h_count, f->at<int>(p.o_count), sizeof(int),
                             hipMemcpyDeviceToHost, s));
    GLM_CHECK(hipStreamSynchronize(s));
    if (log_on() && (it % (kPollEvery * 16) == 0 || *f->h_count == 0))
      std::fprintf(stderr, "[glm %.3fs] pcg-ne it %lld active rhs %d\n", now_s(), (long long)it,
                   *f->h_count);
    if (*f->h_count == 0) break;
    const int64_t nit = std::min<int64_t>(kPollEvery, maxit_all - it);
    for (int64_t j = 0; j < nit; ++j) {
      PassLaunch<double> a = pass_args<double>(f, f->X, Oinv, nullptr, w, nullptr, nullptr, false);
      a.deq = nullptr;
      a.Tm = pv;
      if (int rc = run_pass_b<double>(f, a, PASS_B_EXPAND, s)) return rc;
      if (int rc = normal_product(w)) return rc;
      GLM_CHECK(launch_ne_step(f->d_inst(), f->d_blk(), p.B, f->at<double>(p.o_R), Oinv, Tm,
                               beta, rv, zv, pv, f->d_st(), f->d_active(), icount, tol,
                               max_iter, s));
      ++f->launches;
    }
  }
  f->stats.outer_steps = 1;
  f->stats.launches = f->launches;
  return map_info_and_stats(f, info, iters, false, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

namespace {

// Y_red = Q1^T Y over the batch; while profiling, bracketed by HIP events
// (kernel id 2) with its algorithmic bytes counted on the host: Q1 and Y read
// once, Y_red written once.
int timed_gemm1(glm_factor* f, const double* Y, double* Yr, hipStream_t s) {
  const RedPlan& r = f->rp;
  EventPair e{};
  if (f->prof) {
    e = get_event(f, 2);
    GLM_CHECK(hipEventRecord(e.a, s));
    f->prof_bytes_host += r.gemm1_bytes;
  }
  GLM_CHECK(launch_red_gemm_tn(f->at<RedDesc>(r.o_desc), f->at<GemmTile>(r.o_t1),
                               (int)r.t1.size(), f->at<double>(r.o_Q1), Y, Yr, s));
  if (f->prof) {
    GLM_CHECK(hipEventRecord(e.b, s));
    f->ev_used.push_back(e);
  }
  return GLM_OK;
}

// glm_qr_factor with GLM_REDUCED: copy X, factor W = [X_1 ... X_G] panel by
// panel (each panel's block reflector applied to the columns right of it),
// form Q1 = Q [I; 0] backwards, take the reduced regressors from R and
// factor the reduced problem in the rest of the workspace.
int factor_entry(const glm_shape* shape, glm_precision prec, const double* X,
                 const double* Rc, void* ws, size_t ws_bytes, hipStream_t stream,
                 glm_factor** out, bool pinned);

int factor_reduced(const glm_shape* shape, glm_precision base, const double* X,
                   const double* Rc, void* ws, size_t ws_bytes, hipStream_t stream,
                   glm_factor** out, bool pinned, const int32_t* wcols = nullptr,
                   const int32_t* sel = nullptr) {
  glm_factor* f = new (std::nothrow) glm_factor();
  if (!f) return GLM_EINVAL;
  int rc = make_red_plan(shape, base, f->rp, wcols, sel);
  if (rc != GLM_OK) {
    delete f;
    return rc;
  }
  const RedPlan& r = f->rp;
  bool any_k = false;
  for (int32_t v : r.k) any_k = any_k || v > 0;
  if (any_k && !Rc) {
    delete f;
    return GLM_EINVAL;
  }
  if (!ws || ws_bytes < r.total) {
    delete f;
    return GLM_EWORKSPACE;
  }
  f->reduced = true;
  f->ws = static_cast<char*>(ws);
  f->X = X;
  f->Rc = Rc;
  const RedDesc* dd = f->at<RedDesc>(r.o_desc);
  double* W = f->at<double>(r.o_W);
  double* T = f->at<double>(r.o_T);
  double* Q1 = f->at<double>(r.o_Q1);
  double* Tleaf = f->at<double>(r.o_Tleaf);
  double* Stk = f->at<double>(r.o_Stk);
  // the descriptor vectors live in the handle, so the copies may stay in flight
  hipError_t e = hipMemcpyAsync(f->ws + r.o_desc, r.d_dev.data(),
                                sizeof(RedDesc) * r.d_dev.size(), hipMemcpyHostToDevice, stream);
  if (!e)
    e = hipMemcpyAsync(f->ws + r.o_t1, r.t1.data(), sizeof(GemmTile) * r.t1.size(),
                       hipMemcpyHostToDevice, stream);
  if (!e)
    e = hipMemcpyAsync(f->ws + r.o_t2, r.t2.data(), sizeof(GemmTile) * r.t2.size(),
                       hipMemcpyHostToDevice, stream);
  if (!e && r.common)
    e = hipMemcpyAsync(f->ws + r.o_sel, r.sel.data(), 4 * r.sel.size(), hipMemcpyHostToDevice,
                       stream);
  // W = X with power-of-two column scaling (undone in the extracted R rows)
  if (!e) e = launch_fill<int>(f->at<int>(r.o_cexp), r.sumn, INT_MIN, stream);
  if (!e) e = launch_red_equilibrate(dd, r.B, r.maxM, X, f->at<int>(r.o_cexp), W, stream);
  for (int p = 0; p < r.maxpan && !e; ++p)
    // trailing columns: n - c0 - w, with w < 32 where kr = min(M, n) ends the
    // panel early, so the bound is n - c0
    e = launch_red_panel(dd, r.B, p, r.maxseg, r.maxn - p * RED_PANEL, W, Tleaf, Stk,
                         f->at<double>(r.o_tau), T, stream);
  if (!e) e = launch_red_qinit(dd, r.B, Q1, stream);
  for (int p = r.maxpan - 1; p >= 0 && !e; --p)
    e = launch_red_q1_panel(dd, r.B, p, r.maxseg, r.maxMr - p * RED_PANEL, W, Tleaf, Stk, T, Q1,
                            stream);
  if (!e)
    e = launch_red_extract(dd, r.B, W, f->at<int>(r.o_cexp),
                           r.common ? f->at<int>(r.o_sel) : nullptr, f->at<double>(r.o_Xr),
                           stream);
  if (e != hipSuccess) {
    delete f;
    return GLM_EHIP;
  }
  rc = factor_entry(&f->rp.sub, base, f->at<double>(r.o_Xr), Rc, f->ws + r.o_sub,
                    r.sub_bytes, stream, &f->sub, pinned);
  if (rc != GLM_OK) {
    delete f;
    return rc;
  }
  *out = f;
  return GLM_OK;
}

// The full model's u-like vector from the reduced solution:
//   U = (Y - [X_i b_i]) Omega^g  (+ Q1 (U_red - U_red Omega Omega^g) where
// Omega is singular).  Y may be null (zero).
int red_full_u(glm_factor* f, const double* Omega, const double* Y, const double* b,
               double* U, hipStream_t s) {
  const RedPlan& rp = f->rp;
  const RedDesc* dd = f->at<RedDesc>(rp.o_desc);
  int* sing = f->at<int>(rp.o_sing);
  GLM_CHECK(launch_red_ginv(dd, rp.B, Omega, f->at<double>(rp.o_Ow), f->at<double>(rp.o_Og),
                            sing, s));
  GLM_CHECK(launch_red_u(dd, rp.B, rp.maxM, f->sub->d_inst(), f->sub->d_blk(),
                         rp.common ? f->at<int>(rp.o_sel) : nullptr, f->X, b, Y,
                         f->at<double>(rp.o_Og), U, s));
  std::vector<int> hs(rp.B, 0);
  GLM_CHECK(hipMemcpyAsync(hs.data(), sing, 4 * (size_t)rp.B, hipMemcpyDeviceToHost, s));
  GLM_CHECK(hipStreamSynchronize(s));
  bool any = false;
  for (int v : hs) any = any || v != 0;
  if (any)
    GLM_CHECK(launch_red_singular(dd, rp.B, rp.dchunks, f->at<GemmTile>(rp.o_t2),
                                  (int)rp.t2.size(), sing, Omega, f->at<double>(rp.o_Og),
                                  f->at<double>(rp.o_Q1), f->at<double>(rp.o_ur),
                                  f->at<double>(rp.o_dd), U, s));
  return GLM_OK;
}

// glm_gls_solve on a reduced handle: Y_red = Q1^T Y, the reduced solve on its
// Mr rows, then the full model's u.
int solve_reduced(glm_factor* f, const double* Omega, const double* y, const double* r,
                  double tol, int32_t max_iter, double* beta, double* u, double* uc,
                  int32_t* info, int32_t* iters, hipStream_t stream) {
  const RedPlan& rp = f->rp;
  if (int rc = timed_gemm1(f, y, f->at<double>(rp.o_yr), stream)) return rc;
  int rc = glm_gls_solve(f->sub, Omega, f->at<double>(rp.o_yr), r, tol, max_iter, beta,
                         f->at<double>(rp.o_ur), uc, info, iters, stream);
  if (rc != GLM_OK) return rc;
  if ((rc = red_full_u(f, Omega, y, beta, u, stream))) return rc;
  f->stats = f->sub->stats;
  f->stats.launches += 4;
  return GLM_OK;
}

// glm_gls_backward on a reduced handle: the adjoint system is the augmented
// system with right-hand side [g_u; g_beta], so it goes through the same
// reduction (lower right-hand side g_beta on the reduced problem); then the
// gradients of the full model.
int backward_reduced(glm_factor* f, const double* Omega, const double* beta, const double* u,
                     const double* g_beta, const double* g_u, double tol, int32_t max_iter,
                     double* dy, double* dOmega, double* dX, int32_t* info, int32_t* iters,
                     hipStream_t s) {
  const RedPlan& rp = f->rp;
  double* yr = f->at<double>(rp.o_yr);
  double* lb = f->at<double>(rp.o_lb);
  if (g_u) {
    if (int rc = timed_gemm1(f, g_u, yr, s)) return rc;
  } else {
    GLM_CHECK(launch_fill<double>(yr, rp.sumMrGK, 0.0, s));
  }
  int rc = solve_driver(f->sub, Omega, yr, g_beta, nullptr, tol, max_iter, lb,
                        f->at<double>(rp.o_ur), nullptr, info, iters, s);
  if (rc != GLM_OK) return rc;
  if ((rc = red_full_u(f, Omega, g_u, lb, dy, s))) return rc;
  GLM_CHECK(launch_red_grad(f->at<RedDesc>(rp.o_desc), rp.B, rp.maxM, f->sub->d_inst(),
                            f->sub->at<int>(f->sub->p.o_colblk), dy, u, beta, lb,
                            f->at<double>(rp.o_Zp), dOmega, dX, s));
  GLM_CHECK(hipStreamSynchronize(s));
  f->stats = f->sub->stats;
  return GLM_OK;
}

}  // namespace

extern "C" {

int glm_validate_shape(const glm_shape* shape) { return validate(shape); }

size_t glm_workspace_bytes(const glm_shape* shape, glm_precision prec) {
  if (!prec_ok(prec)) return 0;
  if ((int)prec & GLM_REDUCED) {
    const glm_precision base = (glm_precision)((int)prec & ~GLM_REDUCED);
    RedPlan r;
    if (make_red_plan(shape, base, r) != GLM_OK) return 0;
    return r.total;
  }
  Plan p;
  if (make_plan(shape, prec, p) != GLM_OK) return 0;
  return p.total;
}

int glm_qr_factor(const glm_shape* shape, glm_precision prec, const double* X,
                  const double* Rc, void* ws, size_t ws_bytes, hipStream_t stream,
                  glm_factor** out) {
  return factor_entry(shape, prec, X, Rc, ws, ws_bytes, stream, out, true);
}

size_t glm_workspace_bytes_common(const glm_shape* shape, glm_precision prec,
                                  const int32_t* N, const int32_t* sel) {
  if (!prec_ok(prec) || !N || !sel) return 0;
  const glm_precision base = (glm_precision)((int)prec & ~GLM_REDUCED);
  RedPlan r;
  if (make_red_plan(shape, base, r, N, sel) != GLM_OK) return 0;
  return r.total;
}

int glm_qr_factor_common(const glm_shape* shape, glm_precision prec, const double* Z0,
                         const int32_t* N, const int32_t* sel, const double* Rc, void* ws,
                         size_t ws_bytes, hipStream_t stream, glm_factor** out) {
  if (!shape || !Z0 || !N || !sel || !out || !prec_ok(prec)) return GLM_EINVAL;
  *out = nullptr;
  const glm_precision base = (glm_precision)((int)prec & ~GLM_REDUCED);
  return factor_reduced(shape, base, Z0, Rc, ws, ws_bytes, stream, out, true, N, sel);
}

int glm_qr_factor_static(const glm_shape* shape, glm_precision prec, const double* X,
                         const double* Rc, hipStream_t stream, glm_factor** out) {
  if (!out || !X) return GLM_EINVAL;
  *out = nullptr;
  const size_t need = glm_workspace_bytes(shape, prec);
  if (need == 0) {
    const int rc = validate(shape);
    return rc != GLM_OK ? rc : GLM_EINVAL;
  }
  if (need > kStaticScratchBytes) return GLM_EWORKSPACE;
  void* ws = nullptr;
  if (static_scratch(&ws) != hipSuccess || !ws) return GLM_EHIP;
  return factor_entry(shape, prec, X, Rc, ws, kStaticScratchBytes, stream, out, false);
}

}  // extern "C"

namespace {

int factor_entry(const glm_shape* shape, glm_precision prec, const double* X,
                 const double* Rc, void* ws, size_t ws_bytes, hipStream_t stream,
                 glm_factor** out, bool pinned) {
  if (!out || !X) return GLM_EINVAL;
  *out = nullptr;
  if (!prec_ok(prec)) return GLM_EINVAL;
  if ((int)prec & GLM_REDUCED) {
    const glm_precision base = (glm_precision)((int)prec & ~GLM_REDUCED);
    return factor_reduced(shape, base, X, Rc, ws, ws_bytes, stream, out, pinned);
  }
  glm_factor* f = new (std::nothrow) glm_factor();
  if (!f) return GLM_EINVAL;
  int rc = make_plan(shape, prec, f->p);
  if (rc != GLM_OK) {
    delete f;
    return rc;
  }
  const Plan& p = f->p;
  if (p.sumRc > 0 && !Rc) {
    delete f;
    return GLM_EINVAL;
  }
  if (!ws || ws_bytes < p.total) {
    delete f;
    return GLM_EWORKSPACE;
  }
  f->ws = static_cast<char*>(ws);
  f->X = X;
  f->Rc = Rc;
  if (pinned) {
    if (hipHostMalloc((void**)&f->h_count, sizeof(int) * 4, hipHostMallocDefault) != hipSuccess) {
      delete f;
      return GLM_EHIP;
    }
    f->h_count_pinned = true;
    f->use_graphs = graphs_on();
  } else {
    f->h_count = f->h_count_host;   // pageable: the poll copy completes at the stream sync
  }
  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(f->ws + off, src, bytes, hipMemcpyHostToDevice, stream);
  };
  hipError_t e = hipSuccess;
  if (!e) e = up(p.o_inst, p.inst.data(), sizeof(InstDesc) * p.inst.size());
  if (!e) e = up(p.o_blk, p.blk.data(), sizeof(BlockDesc) * p.blk.size());
  if (!e) e = up(p.o_tile, p.tile.data(), sizeof(TileDesc) * p.tile.size());
  if (!e) e = up(p.o_qrs, p.qr_sur.data(), sizeof(QRJob) * p.qr_sur.size());
  if (!e) e = up(p.o_qrn, p.qr_nb.data(), sizeof(QRJob) * p.qr_nb.size());
  if (!e) e = up(p.o_chunks, p.chunks.data(), sizeof(RedChunk) * p.chunks.size());
  if (!e) e = up(p.o_rinst, p.rinst.data(), 4 * p.rinst.size());
  if (!e) e = up(p.o_rinst_index, p.rinst_index.data(), 4 * p.rinst_index.size());
  if (!e) e = up(p.o_colblk, p.colblk.data(), 4 * p.colblk.size());
  // the host descriptor vectors must outlive the asynchronous copies
  if (!e) e = hipStreamSynchronize(stream);
  if (!e) e = hipMemcpyAsync(f->ws + p.o_Q64, X, 8 * p.sumMn, hipMemcpyDeviceToDevice, stream);
  if (!e) e = launch_fill<int>(f->at<int>(p.o_flags), p.nblk + (int64_t)p.rinst.size(), 0, stream);
  if (!e)
    e = launch_qr(f->at<QRJob>(p.o_qrs), (int)p.qr_sur.size(), p.maxni, f->at<double>(p.o_Q64),
                  f->at<double>(p.o_R), f->at<int>(p.o_flags), stream);
  if (!e && !p.rinst.empty()) {
    e = launch_nullbasis_input(f->d_inst(), f->at<int>(p.o_rinst), (int)p.rinst.size(),
                               f->d_blk(), f->at<double>(p.o_R), Rc, f->at<double>(p.o_Nb),
                               stream);
    if (!e)
      e = launch_qr(f->at<QRJob>(p.o_qrn), (int)p.qr_nb.size(), p.maxkc,
                    f->at<double>(p.o_Nb), f->at<double>(p.o_R), f->at<int>(p.o_flags), stream);
  }
  if (!e && p.prec == GLM_MIXED)
    e = launch_to_float(f->at<double>(p.o_Q64), f->at<float>(p.o_Q32), p.sumMn, stream);
  if (e != hipSuccess) {
    if (f->h_count_pinned) (void)hipHostFree(f->h_count);
    delete f;
    return GLM_EHIP;
  }
  *out = f;
  return GLM_OK;
}

}  // namespace

extern "C" {

int glm_gls_solve(glm_factor* f, const double* Omega, const double* y, const double* r,
                  double tol, int32_t max_iter, double* beta, double* u, double* uc,
                  int32_t* info, int32_t* iters, hipStream_t stream) {
  if (!f || !Omega || !y || !beta || !u) return GLM_EINVAL;
  if (!(tol >= 0.0)) return GLM_EINVAL;
  if (f->reduced)
    return solve_reduced(f, Omega, y, r, tol, max_iter, beta, u, uc, info, iters, stream);
  if (f->p.sumCK > 0 && !r) return GLM_EINVAL;
  return solve_driver(f, Omega, y, nullptr, r, tol, max_iter, beta, u, uc, info, iters, stream);
}

int glm_gls_solve_ne(glm_factor* f, const double* Omega, const double* y, double tol,
                     int32_t max_iter, double* beta, int32_t* info, int32_t* iters,
                     hipStream_t stream) {
  if (!f || !Omega || !y || !beta) return GLM_EINVAL;
  if (!(tol >= 0.0)) return GLM_EINVAL;
  if (!f->reduced) return ne_driver(f, Omega, y, tol, max_iter, beta, info, iters, stream);
  // the GLS estimate of the reduced model is that of the full model
  if (f->sub->p.sumCK > 0) return GLM_EUNSUPPORTED;
  if (int rc = timed_gemm1(f, y, f->at<double>(f->rp.o_yr), stream)) return rc;
  const int rc = ne_driver(f->sub, Omega, f->at<double>(f->rp.o_yr), tol, max_iter, beta, info,
                           iters, stream);
  f->stats = f->sub->stats;
  ++f->stats.launches;
  return rc;
}

int glm_gls_backward(glm_factor* f, const double* Omega, const double* beta, const double* u,
                     const double* g_beta, const double* g_u, double tol, int32_t max_iter,
                     double* dy, double* dOmega, double* dX, int32_t* info, int32_t* iters,
                     hipStream_t stream) {
  if (!f || !Omega || !beta || !u || !g_beta || !dy) return GLM_EINVAL;
  if (!(tol >= 0.0)) return GLM_EINVAL;
  if (f->reduced && f->rp.common) return GLM_EUNSUPPORTED;
  if (f->reduced)
    return backward_reduced(f, Omega, beta, u, g_beta, g_u, tol, max_iter, dy, dOmega, dX,
                            info, iters, stream);
  const Plan& p = f->p;
  double* lb = f->at<double>(p.o_lb);
  // adjoint system [Sigma X; X^T 0][l_u; l_beta] = [g_u; g_beta] (restriction rows: 0)
  int rc = solve_driver(f, Omega, g_u, g_beta, nullptr, tol, max_iter, lb, dy, nullptr, info,
                        iters, stream);
  if (rc) return rc;
  GLM_CHECK(launch_grad(f->d_inst(), f->d_tile(), p.ntiles, p.B, f->at<int>(p.o_colblk), dy, u,
                        beta, lb, f->at<double>(p.o_Tpart), dOmega, dX, stream));
  GLM_CHECK(hipStreamSynchronize(stream));
  return GLM_OK;
}

int glm_copy_factors(const glm_factor* f, double* Q, double* R, int32_t* rank,
                     hipStream_t stream) {
  if (!f) return GLM_EINVAL;
  if (f->reduced) return GLM_EUNSUPPORTED;
  const Plan& p = f->p;
  if (Q)
    GLM_CHECK(hipMemcpyAsync(Q, f->ws + p.o_Q64, 8 * p.sumMn, hipMemcpyDeviceToDevice, stream));
  if (R)
    GLM_CHECK(hipMemcpyAsync(R, f->ws + p.o_R, 8 * p.sumR, hipMemcpyDeviceToDevice, stream));
  if (rank)
    GLM_CHECK(hipMemcpyAsync(rank, f->ws + p.o_flags, 4 * (size_t)p.nblk,
                             hipMemcpyDeviceToDevice, stream));
  return GLM_OK;
}

int glm_plan_passes(const glm_shape* shape, glm_precision prec, glm_stats* out) {
  if (!out) return GLM_EINVAL;
  *out = glm_stats{};
  if (!prec_ok(prec)) return GLM_EINVAL;
  const glm_precision base = (glm_precision)((int)prec & ~GLM_REDUCED);
  Plan p;
  if ((int)prec & GLM_REDUCED) {
    RedPlan r;
    if (int rc = make_red_plan(shape, base, r)) return rc;
    if (int rc = make_plan(&r.sub, base, p)) return rc;
  } else if (int rc = make_plan(shape, base, p)) {
    return rc;
  }
  pass_stats(p, out);
  return GLM_OK;
}

int glm_get_stats(const glm_factor* f, glm_stats* out) {
  if (!f || !out) return GLM_EINVAL;
  *out = f->stats;
  return GLM_OK;
}

int glm_profile_enable(glm_factor* f, int on) {
  if (!f) return GLM_EINVAL;
  if (f->reduced) {
    f->prof = on != 0;
    return glm_profile_enable(f->sub, on);
  }
  f->prof = on != 0;
  return GLM_OK;
}

int glm_profile_read(glm_factor* f, int kernel_id, int64_t* launches, double* total_ms,
                     double* total_bytes) {
  if (!f || kernel_id < 0 || kernel_id > 2) return GLM_EINVAL;
  if (f->reduced && kernel_id < 2)
    return glm_profile_read(f->sub, kernel_id, launches, total_ms, total_bytes);
  if (!f->reduced && kernel_id == 2) {
    if (launches) *launches = 0;
    if (total_ms) *total_ms = 0.0;
    if (total_bytes) *total_bytes = 0.0;
    return GLM_OK;
  }
  if (hipDeviceSynchronize() != hipSuccess) return GLM_EHIP;
  for (auto& e : f->ev_used) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) return GLM_EHIP;
    f->prof_ms[e.kid] += ms;
    f->prof_launch[e.kid] += 1;
    f->ev_free.push_back(e);
  }
  f->ev_used.clear();
  if (f->reduced) {
    // Q1^T Y products: bytes counted on the host when launched
    if (launches) *launches = f->prof_launch[2];
    if (total_ms) *total_ms = f->prof_ms[2];
    if (total_bytes) *total_bytes = f->prof_bytes_host;
    f->prof_launch[2] = 0;
    f->prof_ms[2] = 0.0;
    f->prof_bytes_host = 0.0;
    return GLM_OK;
  }
  unsigned long long hb[2] = {0, 0};
  if (hipMemcpy(hb, f->ws + f->p.o_bytes, sizeof(hb), hipMemcpyDeviceToHost) != hipSuccess)
    return GLM_EHIP;
  if (launches) *launches = f->prof_launch[kernel_id];
  if (total_ms) *total_ms = f->prof_ms[kernel_id];
  if (total_bytes) *total_bytes = (double)hb[kernel_id];
  // clear this kernel's counters
  f->prof_launch[kernel_id] = 0;
  f->prof_ms[kernel_id] = 0.0;
  hb[kernel_id] = 0;
  if (hipMemcpy(f->ws + f->p.o_bytes, hb, sizeof(hb), hipMemcpyHostToDevice) != hipSuccess)
    return GLM_EHIP;
  return GLM_OK;
}

void glm_factor_destroy(glm_factor* f) {
  if (!f) return;
  if (f->sub) glm_factor_destroy(f->sub);
  for (auto& e : f->ev_used) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto& e : f->ev_free) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto& ge : f->graphs) (void)hipGraphExecDestroy(ge.exec);
  if (f->cap_stream) (void)hipStreamDestroy(f->cap_stream);
  if (f->h_count_pinned) (void)hipHostFree(f->h_count);
  delete f;
}

const char* glm_strerror(int code) {
  switch (code) {
    case GLM_OK: return "ok / converged";
    case GLM_EINVAL: return "invalid argument or shape";
    case GLM_EWORKSPACE: return "workspace missing or too small";
    case GLM_EHIP: return "HIP runtime error";
    case GLM_EUNSUPPORTED: return "shape outside the supported limits";
    case GLM_INFO_STAGNATED: return "terminated: c_i stopped decreasing";
    case GLM_INFO_NOCONV: return "iteration limit reached";
    case GLM_INFO_BREAKDOWN: return "breakdown: d_i <= 0 or not finite";
    case GLM_INFO_RANK: return "numerically rank-deficient regressor block";
    default: return "unknown code";
  }
}

}  // extern "C"
