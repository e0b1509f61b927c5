// Multi-hop propagation (Algorithm 1 lines 1-4; Eqs. update-Z and PX).
//
// With L = D_U^-1/2 B D_V^-1/2 the Horner step Z <- X' + alpha L (L^T Z) is
// evaluated on W = D_U^-1/2 Z as two CSR SpMMs with per-row scales:
//   T[v] = D_V^-1[v]   * sum_u w(u,v) W[u]                    (rows of B^T)
//   Z[u] = X'[u] + alpha D_U^-1/2[u] * sum_v w(u,v) T[v]       (rows of B)
//   W[u] = D_U^-1/2[u] Z[u]   for the next hop,
// and the last hop stores (1 - alpha) Z, which is Eq. PX.  Isolated nodes have
// zero scales, so an isolated u keeps Z[u] = X'[u] (the r = 0 term alone).
//
// Kernel shape (d-wide FP32 rows, d a power of two): one wave per output row;
// a neighbour row of d floats is read by d/4 lanes with float4 loads, so one
// wave instruction gathers 64/(d/4) neighbour rows.  Column indices are read
// 64 at a time with one coalesced load and handed to the lane groups with
// cross-lane permutes.  Rows with more than kHubChunk neighbours are split
// into chunks (one wave each) whose partial sums a second kernel adds in chunk
// order, so every sum has a fixed order (bitwise reproducible).
#include "dev_common.hpp"
#include "tpo_internal.hpp"

namespace tpo {

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

// Items [0, nrows): rows (hub rows skipped); items [nrows, nrows + n_chunks):
// hub chunks writing partial sums.
template <int D, int MODE>
__global__ void __launch_bounds__(256)
k_spmm_rows(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col, const float* __restrict__ val,
            const DevStatus* __restrict__ st, const int32_t* __restrict__ n_chunks, const int4* __restrict__ chunks,
            const float* __restrict__ src, int nrows, const float* __restrict__ rscale,
            const float* __restrict__ xp, float alpha, float one_minus_alpha, float* __restrict__ dst,
            float* __restrict__ partial) {
  const int item = static_cast<int>((static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
  const bool has_vals = st->has_vals != 0;
  if (item < nrows) {
    const int b = rowptr[item], e = rowptr[item + 1];
    if (e - b > kHubChunk) return;
    const float4 acc = gather_sum<D>(col, val, has_vals, src, b, e);
    spmm_epilogue<D, MODE>(item, acc, rscale, xp, alpha, one_minus_alpha, dst);
  } else {
    const int c = item - nrows;
    if (c >= *n_chunks) return;
    const int4 ch = chunks[c];
    const float4 acc = gather_sum<D>(col, val, has_vals, src, ch.y, ch.z);
    const int lane = threadIdx.x & 63;
    if (lane < SpmmShape<D>::LPR)
      *reinterpret_cast<float4*>(partial + static_cast<int64_t>(ch.w) * D + lane * 4) = acc;
  }
}

// One wave per hub row: add its chunk partials in order, then the epilogue.
template <int D, int MODE>
__global__ void __launch_bounds__(256)
k_spmm_hubs(const int32_t* __restrict__ n_hubs, const int4* __restrict__ hubs, const float* __restrict__ partial,
            const float* __restrict__ rscale, const float* __restrict__ xp, float alpha, float one_minus_alpha,
            float* __restrict__ dst) {
  const int h = static_cast<int>((static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
  if (h >= *n_hubs) return;
  const int4 hb = hubs[h];
  const int lane = threadIdx.x & 63;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  if (lane < SpmmShape<D>::LPR) {
    for (int c = 0; c < hb.z; ++c) {
      const float4 v = *reinterpret_cast<const float4*>(partial + static_cast<int64_t>(hb.y + c) * D + lane * 4);
      acc.x += v.x;
      acc.y += v.y;
      acc.z += v.z;
      acc.w += v.w;
    }
  }
  spmm_epilogue<D, MODE>(hb.x, acc, rscale, xp, alpha, one_minus_alpha, dst);
}

// W0 = D_U^-1/2 X'  (or Z = (1 - alpha) X' when gamma = 0)
__global__ void k_scale_rows(const float* __restrict__ x, int n, int D, const float* __restrict__ rscale,
                             float c, float* __restrict__ out) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(n) * D) return;
  const int r = static_cast<int>(i / D);
  out[i] = (rscale ? rscale[r] : 1.0f) * c * x[i];
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
    hipLaunchKernelGGL(k_scale_rows, dim3(ceil_div(static_cast<int64_t>(n) * D, 256)), dim3(256), 0, s, xp, n, D,
                       nullptr, oma, z);
    TPO_LAUNCH_CHECK();
    return;
  }
  hipLaunchKernelGGL(k_scale_rows, dim3(ceil_div(static_cast<int64_t>(n) * D, 256)), dim3(256), 0, s, xp, n, D,
                     isq, 1.0f, w0);
  TPO_LAUNCH_CHECK();
  const unsigned grid_v = ceil_div((static_cast<int64_t>(m) + p.max_chunks_v) * 64, 256);
  const unsigned grid_u = ceil_div((static_cast<int64_t>(n) + p.max_chunks_u) * 64, 256);
  const unsigned hub_v = ceil_div(static_cast<int64_t>(p.max_chunks_v) * 64, 256);
  const unsigned hub_u = ceil_div(static_cast<int64_t>(p.max_chunks_u) * 64, 256);
  float* cur = w0;
  float* nxt = w1;
  for (int hop = 1; hop <= p.par.gamma; ++hop) {
    const bool tm = p.timing && p.kev_made && hop <= kMaxTimedHops;
    const hipEvent_t* ev = p.kev + 4 * (hop - 1);
    if (tm) TPO_HIP_CHECK(hipEventRecord(ev[0], s));
    hipLaunchKernelGGL((k_spmm_rows<D, kModeV>), dim3(grid_v), dim3(256), 0, s,
                       bufp<int32_t>(p, ws, B_ROWPTR_V), bufp<int32_t>(p, ws, B_COL_V), bufp<float>(p, ws, B_VAL_V),
                       st, &st->hub_chunks_v, bufp<int4>(p, ws, B_CHUNK_V), cur, m, invv, nullptr, alpha, oma, t,
                       partial);
    TPO_LAUNCH_CHECK();
    if (tm) TPO_HIP_CHECK(hipEventRecord(ev[1], s));
    if (p.max_chunks_v > 0) {
      hipLaunchKernelGGL((k_spmm_hubs<D, kModeV>), dim3(hub_v), dim3(256), 0, s, &st->hub_rows_v,
                         bufp<int4>(p, ws, B_HUBLIST_V), partial, invv, nullptr, alpha, oma, t);
      TPO_LAUNCH_CHECK();
    }
    const bool last = hop == p.par.gamma;
    float* dst = last ? z : nxt;
    if (tm) TPO_HIP_CHECK(hipEventRecord(ev[2], s));
    if (last) {
      hipLaunchKernelGGL((k_spmm_rows<D, kModeUFinal>), dim3(grid_u), dim3(256), 0, s,
                         bufp<int32_t>(p, ws, B_ROWPTR_U), bufp<int32_t>(p, ws, B_COL_U),
                         bufp<float>(p, ws, B_VAL_U), st, &st->hub_chunks_u, bufp<int4>(p, ws, B_CHUNK_U), t, n,
                         isq, xp, alpha, oma, dst, partial);
      TPO_LAUNCH_CHECK();
      if (tm) TPO_HIP_CHECK(hipEventRecord(ev[3], s));
      if (p.max_chunks_u > 0) {
        hipLaunchKernelGGL((k_spmm_hubs<D, kModeUFinal>), dim3(hub_u), dim3(256), 0, s, &st->hub_rows_u,
                           bufp<int4>(p, ws, B_HUBLIST_U), partial, isq, xp, alpha, oma, dst);
        TPO_LAUNCH_CHECK();
      }
    } else {
      hipLaunchKernelGGL((k_spmm_rows<D, kModeUMid>), dim3(grid_u), dim3(256), 0, s,
                         bufp<int32_t>(p, ws, B_ROWPTR_U), bufp<int32_t>(p, ws, B_COL_U),
                         bufp<float>(p, ws, B_VAL_U), st, &st->hub_chunks_u, bufp<int4>(p, ws, B_CHUNK_U), t, n,
                         isq, xp, alpha, oma, dst, partial);
      TPO_LAUNCH_CHECK();
      if (tm) TPO_HIP_CHECK(hipEventRecord(ev[3], s));
      if (p.max_chunks_u > 0) {
        hipLaunchKernelGGL((k_spmm_hubs<D, kModeUMid>), dim3(hub_u), dim3(256), 0, s, &st->hub_rows_u,
                           bufp<int4>(p, ws, B_HUBLIST_U), partial, isq, xp, alpha, oma, dst);
        TPO_LAUNCH_CHECK();
      }
      std::swap(cur, nxt);
    }
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
