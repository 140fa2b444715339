// Streaming ceiling of a read/write mix: a plain kernel that moves the bytes
// of a projection pass in the same pattern (read-only streams, streams read
// and overwritten in place, write-only streams) with nothing else to do, so
// that the passes' touched bandwidth can be compared with what this part
// reaches for that mix rather than against the HBM peak alone.
//
// Thread t of workgroup b handles the 16-byte chunks b * SU * 256 + j * 256 + t,
// j < SU, of every stream (consecutive lanes, consecutive chunks): all of a
// thread's loads are issued before any store.
#include "glm.h"
#include "glm_internal.h"

#include <algorithm>

namespace glm {

namespace {

constexpr int SNT = 256;   // threads per workgroup
constexpr int SU = 4;      // 16-byte chunks per thread and stream

struct StreamArgs {
  const float4* ro[GLM_STREAM_MAX];
  int64_t ro_len[GLM_STREAM_MAX];   // in 16-byte chunks
  float4* rw[GLM_STREAM_MAX];
  float4* wo[GLM_STREAM_MAX];
  int64_t rw_len, wo_len;           // in 16-byte chunks
  int nro, nrw, nwo;
  float never;                      // a value no sum takes (NaN)
};

__device__ float g_stream_sink;

__device__ __forceinline__ float4 add4(float4 a, float4 b) {
  return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

// Stream counts are template arguments and indices past a stream's end are
// clamped to its last chunk (the value is then discarded), so that no load
// sits under a branch and all of a thread's loads are in flight together.
template <int NRO, int NRW, int NWO>
__global__ void __launch_bounds__(SNT) k_stream_mix(StreamArgs a) {
  const int64_t base = (int64_t)blockIdx.x * SU * SNT + threadIdx.x;
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 rd[NRO > 0 ? NRO : 1][SU], old[NRW > 0 ? NRW : 1][SU];
#pragma unroll
  for (int s = 0; s < NRO; ++s)
#pragma unroll
    for (int j = 0; j < SU; ++j)
      rd[s][j] = a.ro[s][min(base + (int64_t)j * SNT, a.ro_len[s] - 1)];
#pragma unroll
  for (int s = 0; s < NRW; ++s)
#pragma unroll
    for (int j = 0; j < SU; ++j) old[s][j] = a.rw[s][min(base + (int64_t)j * SNT, a.rw_len - 1)];
#pragma unroll
  for (int j = 0; j < SU; ++j) {
    const int64_t e = base + (int64_t)j * SNT;
    float4 acc = zero;
#pragma unroll
    for (int s = 0; s < NRO; ++s)
      if (e < a.ro_len[s]) acc = add4(acc, rd[s][j]);
#pragma unroll
    for (int s = 0; s < NRW; ++s) {
      const float4 o = old[s][j];
      if (e < a.rw_len)
        a.rw[s][e] = make_float4(0.5f * o.x + acc.x, 0.5f * o.y + acc.y, 0.5f * o.z + acc.z,
                                 0.5f * o.w + acc.w);
    }
#pragma unroll
    for (int s = 0; s < NWO; ++s)
      if (e < a.wo_len) a.wo[s][e] = acc;
    // keeps the reads of chunks that no written stream covers
    if (acc.x == a.never) g_stream_sink = acc.y;
  }
}

using StreamLaunch = void (*)(const StreamArgs&, unsigned, hipStream_t);

template <int NRO, int NRW, int NWO>
void launch_mix(const StreamArgs& a, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL((k_stream_mix<NRO, NRW, NWO>), dim3(blocks), dim3(SNT), 0, s, a);
}

template <int NRO, int NRW>
constexpr StreamLaunch pick_wo(int nwo) {
  return nwo == 0 ? launch_mix<NRO, NRW, 0> : nwo == 1 ? launch_mix<NRO, NRW, 1>
       : nwo == 2 ? launch_mix<NRO, NRW, 2> : nwo == 3 ? launch_mix<NRO, NRW, 3>
                  : launch_mix<NRO, NRW, 4>;
}
template <int NRO>
StreamLaunch pick_rw(int nrw, int nwo) {
  return nrw == 0 ? pick_wo<NRO, 0>(nwo) : nrw == 1 ? pick_wo<NRO, 1>(nwo)
       : nrw == 2 ? pick_wo<NRO, 2>(nwo) : nrw == 3 ? pick_wo<NRO, 3>(nwo)
                  : pick_wo<NRO, 4>(nwo);
}
StreamLaunch pick(int nro, int nrw, int nwo) {
  return nro == 0 ? pick_rw<0>(nrw, nwo) : nro == 1 ? pick_rw<1>(nrw, nwo)
       : nro == 2 ? pick_rw<2>(nrw, nwo) : nro == 3 ? pick_rw<3>(nrw, nwo)
                  : pick_rw<4>(nrw, nwo);
}
static_assert(GLM_STREAM_MAX == 4, "the dispatch above covers 0..4 streams of each kind");

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

}  // namespace glm

using namespace glm;

extern "C" int glm_stream_mix(const float* const* ro, const int64_t* ro_len, int32_t n_ro,
                              float* const* rw, int32_t n_rw, int64_t rw_len,
                              float* const* wo, int32_t n_wo, int64_t wo_len,
                              hipStream_t stream) {
  if (n_ro < 0 || n_rw < 0 || n_wo < 0 || n_ro > GLM_STREAM_MAX || n_rw > GLM_STREAM_MAX ||
      n_wo > GLM_STREAM_MAX || (n_ro && (!ro || !ro_len)) || (n_rw && !rw) || (n_wo && !wo) ||
      (n_rw && rw_len <= 0) || (n_wo && wo_len <= 0) || (rw_len & 3) || (wo_len & 3))
    return GLM_EINVAL;
  StreamArgs a{};
  a.nro = n_ro;
  a.nrw = n_rw;
  a.nwo = n_wo;
  a.rw_len = n_rw ? rw_len / 4 : 0;
  a.wo_len = n_wo ? wo_len / 4 : 0;
  a.never = __builtin_nanf("");
  int64_t chunks = std::max(a.rw_len, a.wo_len);
  for (int s = 0; s < n_ro; ++s) {
    if (ro_len[s] <= 0 || (ro_len[s] & 3) || !ro[s] || !aligned16(ro[s])) return GLM_EINVAL;
    a.ro[s] = reinterpret_cast<const float4*>(ro[s]);
    a.ro_len[s] = ro_len[s] / 4;
    chunks = std::max(chunks, a.ro_len[s]);
  }
  for (int s = 0; s < n_rw; ++s) {
    if (!rw[s] || !aligned16(rw[s])) return GLM_EINVAL;
    a.rw[s] = reinterpret_cast<float4*>(rw[s]);
  }
  for (int s = 0; s < n_wo; ++s) {
    if (!wo[s] || !aligned16(wo[s])) return GLM_EINVAL;
    a.wo[s] = reinterpret_cast<float4*>(wo[s]);
  }
  if (chunks == 0) return GLM_OK;
  const int64_t per_block = (int64_t)SU * SNT;
  const int64_t blocks = (chunks + per_block - 1) / per_block;
  if (blocks > INT32_MAX) return GLM_EINVAL;
  pick(n_ro, n_rw, n_wo)(a, (unsigned)blocks, stream);
  return hipGetLastError() == hipSuccess ? GLM_OK : GLM_EHIP;
}
