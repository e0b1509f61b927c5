// Multi-hop propagation (Algorithm 1; Eqs. update-Z and PX).
//
// With L = D_U^-1/2 B D_V^-1/2 the Horner step Z <- X' + alpha L (L^T Z) is
// evaluated on W = D_U^-1/2 Z as two CSR SpMMs with per-row scales:
//   T[v] = D_V^-1[v]   * sum_u w(u,v) W[u]                    (rows of B^T)
//   Z[u] = X'[u] + alpha D_U^-1/2[u] * sum_v w(u,v) T[v]       (rows of B)
//   W[u] = D_U^-1/2[u] Z[u]   for the next hop,
// and the last hop stores (1 - alpha) Z, which is Eq. PX.  Isolated nodes have
// zero scales, so an isolated u keeps Z[u] = X'[u] (the r = 0 term alone).
//
// Kernel shape (d-wide FP32 rows, d a power of two): a neighbour row of d
// floats is read by a group of d/4 lanes with float4 loads.  Ordinary rows
// (at most kHubChunk neighbours) take one lane group each, so a wave works on
// 64/(d/4) output rows at once and keeps eight gathers in flight per lane;
// their column ids come in with one load per group and are handed out with
// cross-lane permutes.  Rows with more than kHubChunk neighbours are split
// into chunks of one wave each, in the same launch; a second kernel adds the
// chunk partials in chunk order, so every sum has a fixed order (bitwise
// reproducible).  The hub work is walked by a fixed grid of kHubBlocks
// workgroups, so that a launch holds no waves for chunks that do not exist.

#include <algorithm>

#include "dev_common.hpp"
#include "tpo_internal.hpp"

namespace tpo {

typedef float v4f_t __attribute__((ext_vector_type(4)));

enum SpmmMode { kModeV = 0, kModeUMid = 1, kModeUFinal = 2 };

template <int D>
struct SpmmShape {
  static constexpr int LPR = D / 4;        // lanes per neighbour row
  static constexpr int RPI = 64 / LPR;     // neighbour rows per wave step
  static constexpr int UNROLL = RPI >= 16 ? 1 : (RPI >= 4 ? 4 : 8);
};

template <int D>
__device__ __forceinline__ float4 gather_sum(const int32_t* __restrict__ col, const float* __restrict__ val,
                                             bool has_vals, const float* __restrict__ src, int b, int e) {
  using S = SpmmShape<D>;
  const int lane = threadIdx.x & 63;
  const int g = lane / S::LPR;
  const int q = lane % S::LPR;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int base = b; base < e; base += 64) {
    const int cnt = min(64, e - base);
    const int myidx = lane < cnt ? col[base + lane] : 0;
    const float myval = (has_vals && lane < cnt) ? val[base + lane] : 1.0f;
    for (int j0 = 0; j0 < cnt; j0 += S::RPI * S::UNROLL) {
      float4 x[S::UNROLL];
      float wv[S::UNROLL];
#pragma unroll
      for (int u = 0; u < S::UNROLL; ++u) {
        const int j = j0 + u * S::RPI + g;
        const int jj = j < 64 ? j : 63;
        int nb = __shfl(myidx, jj, 64);
        float w = has_vals ? __shfl(myval, jj, 64) : 1.0f;
        if (j >= cnt) {
          nb = myidx;  // any valid row; its contribution is discarded
          w = 0.0f;
        }
        x[u] = *reinterpret_cast<const float4*>(src + static_cast<int64_t>(nb) * D + q * 4);
        wv[u] = (j < cnt) ? w : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < S::UNROLL; ++u) {
        const int j = j0 + u * S::RPI + g;
        if (j < cnt) {
          acc.x += wv[u] * x[u].x;
          acc.y += wv[u] * x[u].y;
          acc.z += wv[u] * x[u].z;
          acc.w += wv[u] * x[u].w;
        }
      }
    }
  }
#pragma unroll
  for (int o = S::LPR; o < 64; o <<= 1) {
    acc.x += __shfl_xor(acc.x, o, 64);
    acc.y += __shfl_xor(acc.y, o, 64);
    acc.z += __shfl_xor(acc.z, o, 64);
    acc.w += __shfl_xor(acc.w, o, 64);
  }
  return acc;
}

template <int D, int MODE>
__device__ __forceinline__ void spmm_epilogue(int r, float4 acc, const float* __restrict__ rscale,
                                              const float* __restrict__ xp, float alpha, float one_minus_alpha,
                                              float* __restrict__ dst) {
  const int lane = threadIdx.x & 63;
  if (lane >= SpmmShape<D>::LPR) return;
  const int q = lane;
  const float sc = rscale[r];
  float4 o;
  if (MODE == kModeV) {
    o = make_float4(sc * acc.x, sc * acc.y, sc * acc.z, sc * acc.w);
  } else {
    const float4 x = *reinterpret_cast<const float4*>(xp + static_cast<int64_t>(r) * D + q * 4);
    const float f = alpha * sc;
    float4 z = make_float4(x.x + f * acc.x, x.y + f * acc.y, x.z + f * acc.z, x.w + f * acc.w);
    if (MODE == kModeUMid)
      o = make_float4(sc * z.x, sc * z.y, sc * z.z, sc * z.w);
    else
      o = make_float4(one_minus_alpha * z.x, one_minus_alpha * z.y, one_minus_alpha * z.z,
                      one_minus_alpha * z.w);
  }
  *reinterpret_cast<float4*>(dst + static_cast<int64_t>(r) * D + q * 4) = o;
}

// One row per lane group: the LPR = D/4 lanes of a group own float4 column
// slices of the output row, so no cross-group reduction is needed; a wave
// carries 64/LPR rows at once.  Column ids come LPR at a time from one load
// by the group and are handed out with cross-lane permutes.
template <int D>
__device__ __forceinline__ float4 gather_row_group(const int32_t* __restrict__ col, const float* __restrict__ val,
                                                   bool has_vals, const float* __restrict__ src, int b, int e) {
  using S = SpmmShape<D>;
  constexpr int U = 8;  // gathers in flight per lane
  const int lane = threadIdx.x & 63;
  const int q = lane % S::LPR;
  const int g0 = lane - q;  // first lane of this group
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int base = b; base < e; base += S::LPR) {
    const int cnt = min(S::LPR, e - base);
    const int myidx = q < cnt ? col[base + q] : 0;
    const float myval = (has_vals && q < cnt) ? val[base + q] : 1.0f;
    for (int j0 = 0; j0 < cnt; j0 += U) {
      float4 x[U];
      float wv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u;
        const int jj = j < S::LPR ? j : S::LPR - 1;
        int nb = __shfl(myidx, g0 + jj, 64);
        const float w = has_vals ? __shfl(myval, g0 + jj, 64) : 1.0f;
        if (j >= cnt) nb = myidx;  // any valid row (a cache hit); its term is skipped
        x[u] = *reinterpret_cast<const float4*>(src + static_cast<int64_t>(nb) * D + q * 4);
        wv[u] = (j < cnt) ? w : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (j0 + u < cnt) {
          acc.x += wv[u] * x[u].x;
          acc.y += wv[u] * x[u].y;
          acc.z += wv[u] * x[u].z;
          acc.w += wv[u] * x[u].w;
        }
      }
    }
  }
  return acc;
}

template <int D, int MODE>
__device__ __forceinline__ void spmm_epilogue_group(int r, float4 acc, const float* __restrict__ rscale,
                                                    const float* __restrict__ xp, float alpha,
                                                    float one_minus_alpha, float* __restrict__ dst) {
  const int q = (threadIdx.x & 63) % SpmmShape<D>::LPR;
  const float sc = rscale[r];
  float4 o;
  if (MODE == kModeV) {
    o = make_float4(sc * acc.x, sc * acc.y, sc * acc.z, sc * acc.w);
  } else {
    const float4 x = *reinterpret_cast<const float4*>(xp + static_cast<int64_t>(r) * D + q * 4);
    const float f = alpha * sc;
    float4 z = make_float4(x.x + f * acc.x, x.y + f * acc.y, x.z + f * acc.z, x.w + f * acc.w);
    if (MODE == kModeUMid)
      o = make_float4(sc * z.x, sc * z.y, sc * z.z, sc * z.w);
    else
      o = make_float4(one_minus_alpha * z.x, one_minus_alpha * z.y, one_minus_alpha * z.z,
                      one_minus_alpha * z.w);
  }
  __builtin_nontemporal_store(v4f_t{o.x, o.y, o.z, o.w},
                              reinterpret_cast<v4f_t*>(dst + static_cast<int64_t>(r) * D + q * 4));
}

// One launch per SpMM side.  The first `chunk_blocks` workgroups walk the hub
// chunks, one wave per chunk, and write partial sums to `partial`; the
// remaining workgroups take the rows of at most kHubChunk neighbours, one row
// per lane group.
template <int D, int MODE>
__global__ void __launch_bounds__(256)
k_spmm_rowgroup(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col, const float* __restrict__ val,
                const DevStatus* __restrict__ st, const int32_t* __restrict__ n_chunks,
                const int4* __restrict__ chunks, int chunk_blocks, const float* __restrict__ src, int nrows,
                const float* __restrict__ rscale, const float* __restrict__ xp, float alpha, float one_minus_alpha,
                float* __restrict__ dst, float* __restrict__ partial) {
  const bool has_vals = st->has_vals != 0;
  if (static_cast<int>(blockIdx.x) < chunk_blocks) {
    constexpr int LPR = SpmmShape<D>::LPR;
    const int lane = threadIdx.x & 63;
    const int nc = *n_chunks;
    const int waves = chunk_blocks * (256 / 64);
    for (int c = static_cast<int>(blockIdx.x) * 4 + static_cast<int>(threadIdx.x >> 6); c < nc; c += waves) {
      const int4 ch = chunks[c];
      const float4 acc = gather_sum<D>(col, val, has_vals, src, ch.y, ch.z);
      if (lane < LPR) *reinterpret_cast<float4*>(partial + static_cast<int64_t>(ch.w) * D + lane * 4) = acc;
    }
    return;
  }
  constexpr int LPR = SpmmShape<D>::LPR;
  const int64_t gidx = (static_cast<int64_t>(blockIdx.x - chunk_blocks) * blockDim.x + threadIdx.x) / LPR;
  if (gidx >= nrows) return;
  const int r = static_cast<int>(gidx);
  const int b = rowptr[r], e = rowptr[r + 1];
  if (e - b > kHubChunk) return;
  const float4 acc = gather_row_group<D>(col, val, has_vals, src, b, e);
  spmm_epilogue_group<D, MODE>(r, acc, rscale, xp, alpha, one_minus_alpha, dst);
}

// One wave per hub row: add its chunk partials in order, then the epilogue.
// The kHubBlocks workgroups (or fewer) walk the hub list.
template <int D, int MODE>
__global__ void __launch_bounds__(256)
k_spmm_hubs(const int32_t* __restrict__ n_hubs, const int4* __restrict__ hubs, const float* __restrict__ partial,
            const float* __restrict__ rscale, const float* __restrict__ xp, float alpha, float one_minus_alpha,
            float* __restrict__ dst) {
  const int lane = threadIdx.x & 63;
  const int nh = *n_hubs;
  const int waves = static_cast<int>(gridDim.x) * 4;
  for (int h = static_cast<int>(blockIdx.x) * 4 + static_cast<int>(threadIdx.x >> 6); h < nh; h += waves) {
    const int4 hb = hubs[h];
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (lane < SpmmShape<D>::LPR) {
      // chunk partials in chunk order; eight loads in flight at a time
      for (int k0 = 0; k0 < hb.z; k0 += 8) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (k0 + u < hb.z)
            v[u] = *reinterpret_cast<const float4*>(partial + static_cast<int64_t>(hb.y + k0 + u) * D + lane * 4);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (k0 + u < hb.z) {
            acc.x += v[u].x;
            acc.y += v[u].y;
            acc.z += v[u].z;
            acc.w += v[u].w;
          }
        }
      }
    }
    spmm_epilogue<D, MODE>(hb.x, acc, rscale, xp, alpha, one_minus_alpha, dst);
  }
}

// W0 = D_U^-1/2 X'  (or Z = (1 - alpha) X' when gamma = 0); one float4 per
// thread (D a power of two, at least 4)
template <int D>
__global__ void k_scale_rows(const float* __restrict__ x, int n, const float* __restrict__ rscale, float c,
                             float* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(n) * (D / 4)) return;
  const int r = static_cast<int>(i / (D / 4));
  const float f = (rscale ? rscale[r] : 1.0f) * c;
  const float4 v = reinterpret_cast<const float4*>(x)[i];
  reinterpret_cast<float4*>(out)[i] = make_float4(f * v.x, f * v.y, f * v.z, f * v.w);
}

template <int D, int MODE>
static void spmm_side(const Plan& p, void* ws, const int32_t* rowptr, const int32_t* col, const float* val,
                      const int32_t* n_chunks, const int4* chunks, unsigned chunk_blocks, const float* src,
                      int nrows, const float* rscale, const float* xp, float alpha, float oma, float* dst,
                      float* partial, hipStream_t s) {
  const DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  const unsigned rows_blocks = ceil_div(static_cast<int64_t>(nrows) * SpmmShape<D>::LPR, 256);
  hipLaunchKernelGGL((k_spmm_rowgroup<D, MODE>), dim3(chunk_blocks + rows_blocks), dim3(256), 0, s, rowptr, col, val,
                     st, n_chunks, chunks, static_cast<int>(chunk_blocks), src, nrows, rscale, xp, alpha, oma, dst,
                     partial);
  TPO_LAUNCH_CHECK();
}

template <int D>
static void propagate_impl(const Plan& p, void* ws, const float* xp, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  const int n = p.n, m = p.m;
  const float alpha = static_cast<float>(p.par.alpha);
  const float oma = static_cast<float>(1.0 - p.par.alpha);
  float* w0 = bufp<float>(p, ws, B_W0);
  float* w1 = bufp<float>(p, ws, B_W1);
  float* t = bufp<float>(p, ws, B_T);
  float* z = bufp<float>(p, ws, B_Z);
  float* partial = bufp<float>(p, ws, B_PARTIAL);
  const float* isq = bufp<float>(p, ws, B_ISQ_U);
  const float* invv = bufp<float>(p, ws, B_INV_V);
  if (p.par.gamma == 0) {
    hipLaunchKernelGGL(k_scale_rows<D>, dim3(ceil_div(static_cast<int64_t>(n) * (D / 4), 256)), dim3(256), 0, s, xp,
                       n, nullptr, oma, z);
    TPO_LAUNCH_CHECK();
    return;
  }
  hipLaunchKernelGGL(k_scale_rows<D>, dim3(ceil_div(static_cast<int64_t>(n) * (D / 4), 256)), dim3(256), 0, s, xp, n,
                     isq, 1.0f, w0);
  TPO_LAUNCH_CHECK();
  // hub-chunk workgroups: enough for every chunk the plan allows, at most
  // kHubBlocks (they loop over the chunks ingest found)
  const unsigned ch_v = std::min<int64_t>(ceil_div(static_cast<int64_t>(p.max_chunks_v) * 64, 256), kHubBlocks);
  const unsigned ch_u = std::min<int64_t>(ceil_div(static_cast<int64_t>(p.max_chunks_u) * 64, 256), kHubBlocks);
  float* cur = w0;
  float* nxt = w1;
  for (int hop = 1; hop <= p.par.gamma; ++hop) {
    const bool tm = p.timing && p.kev_made && hop <= kMaxTimedHops;
    const hipEvent_t* ev = p.kev + 4 * (hop - 1);
    // V side: T = D_V^-1 B^T W
    if (tm) TPO_HIP_CHECK(hipEventRecord(ev[0], s));
    spmm_side<D, kModeV>(p, ws, bufp<int32_t>(p, ws, B_ROWPTR_V), bufp<int32_t>(p, ws, B_COL_V),
                         bufp<float>(p, ws, B_VAL_V), &st->hub_chunks_v, bufp<int4>(p, ws, B_CHUNK_V), ch_v, cur, m,
                         invv, nullptr, alpha, oma, t, partial, s);
    if (tm) TPO_HIP_CHECK(hipEventRecord(ev[1], s));
    if (p.max_chunks_v > 0) {
      hipLaunchKernelGGL((k_spmm_hubs<D, kModeV>), dim3(ch_v), dim3(256), 0, s, &st->hub_rows_v,
                         bufp<int4>(p, ws, B_HUBLIST_V), partial, invv, nullptr, alpha, oma, t);
      TPO_LAUNCH_CHECK();
    }
    // U side: Z = X' + alpha D_U^-1/2 B T  (W = D_U^-1/2 Z between hops)
    const bool last = hop == p.par.gamma;
    float* dst = last ? z : nxt;
    if (tm) TPO_HIP_CHECK(hipEventRecord(ev[2], s));
    if (last)
      spmm_side<D, kModeUFinal>(p, ws, bufp<int32_t>(p, ws, B_ROWPTR_U), bufp<int32_t>(p, ws, B_COL_U),
                                bufp<float>(p, ws, B_VAL_U), &st->hub_chunks_u, bufp<int4>(p, ws, B_CHUNK_U), ch_u, t,
                                n, isq, xp, alpha, oma, dst, partial, s);
    else
      spmm_side<D, kModeUMid>(p, ws, bufp<int32_t>(p, ws, B_ROWPTR_U), bufp<int32_t>(p, ws, B_COL_U),
                              bufp<float>(p, ws, B_VAL_U), &st->hub_chunks_u, bufp<int4>(p, ws, B_CHUNK_U), ch_u, t, n,
                              isq, xp, alpha, oma, dst, partial, s);
    if (tm) TPO_HIP_CHECK(hipEventRecord(ev[3], s));
    if (p.max_chunks_u > 0) {
      if (last)
        hipLaunchKernelGGL((k_spmm_hubs<D, kModeUFinal>), dim3(ch_u), dim3(256), 0, s, &st->hub_rows_u,
                           bufp<int4>(p, ws, B_HUBLIST_U), partial, isq, xp, alpha, oma, dst);
      else
        hipLaunchKernelGGL((k_spmm_hubs<D, kModeUMid>), dim3(ch_u), dim3(256), 0, s, &st->hub_rows_u,
                           bufp<int4>(p, ws, B_HUBLIST_U), partial, isq, xp, alpha, oma, dst);
      TPO_LAUNCH_CHECK();
    }
    if (!last) std::swap(cur, nxt);
  }
}

void launch_propagate(const Plan& p, void* ws, const float* xprime, int64_t ldxp, hipStream_t s) {
  (void)ldxp;  // X' is always materialised with row stride p.dp
  switch (p.dp) {
    case 8: propagate_impl<8>(p, ws, xprime, s); break;
    case 16: propagate_impl<16>(p, ws, xprime, s); break;
    case 32: propagate_impl<32>(p, ws, xprime, s); break;
    case 64: propagate_impl<64>(p, ws, xprime, s); break;
    case 128: propagate_impl<128>(p, ws, xprime, s); break;
    case 256: propagate_impl<256>(p, ws, xprime, s); break;
    default: throw std::runtime_error("unsupported padded width");
  }
}

}  // namespace tpo
