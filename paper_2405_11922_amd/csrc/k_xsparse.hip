// Sparse attributes X_U in CSR (TPO_X_CSR), for the attribute reduction of
// Section 3.2.1 (Eq. Xd) on sparse text rows such as TF-IDF vectors.
//
// * Column scales s_j = max_i |x_ij| / 448 (the largest finite E4M3 value),
//   over the columns of the transpose (a maximum does not depend on order);
//   a column stored twice in a row counts once, with its summed value.
// * FP8 staging: a group of rows is scattered from the transpose into a
//   zeroed byte tile of E4M3 codes of x_ij / s_j (round to nearest even,
//   e4m3_encode), which the FP8 Gram kernel reads like a dense FP8 X_U.  The
//   dense codes of all rows never exist at once.
// * Products with the exact FP32 values for the refinement step and the
//   projection: Y = X B by rows of the CSR (one wave per row, FP64 sums in
//   the row's stored order), and P = X^T Y by columns of the transpose (CSC,
//   rows ascending), each column cut into chunks of kXChunk entries whose
//   FP64 partials are added in chunk order.  Every sum has a fixed order.
#include "dev_common.hpp"
#include "tpo_internal.hpp"

namespace tpo {

constexpr int kXChunk = 8192;  // CSC entries per column chunk

__global__ void k_fill_u32x(uint32_t* __restrict__ a, int64_t n, uint32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_zero_u32x4(uint4* __restrict__ a, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = make_uint4(0u, 0u, 0u, 0u);
}

// The value of X at the entry t of the transpose that starts a run of one
// row (entries of one column stored twice in a row are adjacent, in stored
// order, and add up): that run's sum in stored order.  False for an entry
// inside a run (its run's first entry counts it).
__device__ __forceinline__ bool xcsc_run(const int32_t* __restrict__ rows, const float* __restrict__ cval, int t,
                                         int cb, int ce, int r, float& v) {
  if (t > cb && rows[t - 1] == r) return false;
  v = cval[t];
  for (int u = t + 1; u < ce && rows[u] == r; ++u) v += cval[u];
  return true;
}

// |x_ij| maxima per column (as float bits: non-negative floats order like
// their bit patterns) from the transpose: one workgroup per column chunk,
// one global atomic maximum per wave.
__global__ void __launch_bounds__(256)
k_xcsc_colmax(const int4* __restrict__ chunk, const int32_t* __restrict__ nchunks, const int32_t* __restrict__ colptr,
              const int32_t* __restrict__ rows, const float* __restrict__ cval, uint32_t* __restrict__ colmax) {
  const int nc = *nchunks;
  for (int c = blockIdx.x; c < nc; c += gridDim.x) {
    const int4 ch = chunk[c];
    const int cb = colptr[ch.x], ce = colptr[ch.x + 1];
    uint32_t m = 0u;
    for (int t = ch.y + static_cast<int>(threadIdx.x); t < ch.z; t += blockDim.x) {
      float v;
      if (xcsc_run(rows, cval, t, cb, ce, rows[t], v)) {
        v = fabsf(v);
        if (isfinite(v)) m = max(m, __float_as_uint(v));
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), o, 64)));
    if ((threadIdx.x & 63) == 0 && m) atomicMax(&colmax[ch.x], m);
  }
}

__global__ void k_xcsr_scales(const uint32_t* __restrict__ colmax, int du, float* __restrict__ scale) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= du) return;
  const float m = __uint_as_float(colmax[j]);
  scale[j] = m > 0.0f ? m / 448.0f : 1.0f;
}

static unsigned xcsc_grid(const Plan& p) {
  return static_cast<unsigned>(std::min<int64_t>(std::max<int64_t>(p.xchunks_max, 1), 4096));
}

void xcsr_scales(const Plan& p, void* ws, hipStream_t s) {
  uint32_t* colmax = bufp<uint32_t>(p, ws, B_XS_COLMAX);
  hipLaunchKernelGGL(k_fill_u32x, dim3(ceil_div(p.du, 256)), dim3(256), 0, s, colmax, static_cast<int64_t>(p.du), 0u);
  TPO_LAUNCH_CHECK();
  if (p.xnnz > 0) {
    const int32_t* nchunks = reinterpret_cast<const int32_t*>(bufp<int2>(p, ws, B_XT_CINFO) + p.du);
    hipLaunchKernelGGL(k_xcsc_colmax, dim3(xcsc_grid(p)), dim3(256), 0, s, bufp<int4>(p, ws, B_XT_CHUNK), nchunks,
                       bufp<int32_t>(p, ws, B_XT_COLPTR), bufp<int32_t>(p, ws, B_XT_ROW), bufp<float>(p, ws, B_XT_VA),
                       colmax);
    TPO_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_xcsr_scales, dim3(ceil_div(p.du, 256)), dim3(256), 0, s, colmax, p.du,
                     bufp<float>(p, ws, B_XS_SCALE));
  TPO_LAUNCH_CHECK();
}

// Rows [r0, r0 + nrows) as E4M3 codes of x / s_j at byte (i - r0) ld + j of
// the (zeroed) staging tile, from the transpose: one wave per column chunk.
// Rows ascend within a column, so a chunk's entries of these rows are the
// ones from its cursor (chunk[c].w, the first entry not yet staged) up to
// the first row past the group; the cursor then moves there.
__global__ void __launch_bounds__(256)
k_xcsc_stage_fp8(int4* __restrict__ chunk, const int32_t* __restrict__ nchunks, const int32_t* __restrict__ colptr,
                 const int32_t* __restrict__ rows, const float* __restrict__ cval, const float* __restrict__ scale,
                 int64_t r0, int nrows, int ld, uint8_t* __restrict__ stage) {
  const int lane = threadIdx.x & 63;
  const int wv = static_cast<int>((static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
  const int nwaves = static_cast<int>((static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6);
  const int nc = *nchunks;
  const int64_t r1 = r0 + nrows;
  for (int c = wv; c < nc; c += nwaves) {
    const int4 ch = chunk[c];
    const int cb = colptr[ch.x], ce = colptr[ch.x + 1];
    const float sc = scale[ch.x];
    int t0 = ch.w;
    while (t0 < ch.z) {
      const int t = t0 + lane;
      const int r = t < ch.z ? rows[t] : 0;
      const bool in = t < ch.z && r < r1;
      float v;
      if (in && xcsc_run(rows, cval, t, cb, ce, r, v) && isfinite(v))
        stage[static_cast<int64_t>(r - r0) * ld + ch.x] = e4m3_encode(v / sc);
      const int cnt = __popcll(__ballot(in));  // the group's entries are a prefix
      t0 += cnt;
      if (cnt < 64) break;
    }
    if (lane == 0) chunk[c].w = t0;
  }
}

void xcsr_stage_fp8(const Plan& p, void* ws, int64_t r0, int rows, int ld, hipStream_t s) {
  if (rows <= 0) return;
  uint8_t* stage = bufp<uint8_t>(p, ws, B_XS_STAGE);
  const int64_t words = static_cast<int64_t>(rows) * ld / 16;
  hipLaunchKernelGGL(k_zero_u32x4, dim3(ceil_div(words, 256)), dim3(256), 0, s, reinterpret_cast<uint4*>(stage), words);
  TPO_LAUNCH_CHECK();
  if (p.xnnz > 0) {
    const int32_t* nchunks = reinterpret_cast<const int32_t*>(bufp<int2>(p, ws, B_XT_CINFO) + p.du);
    hipLaunchKernelGGL(k_xcsc_stage_fp8, dim3(ceil_div(xcsc_grid(p), 4)), dim3(256), 0, s,
                       bufp<int4>(p, ws, B_XT_CHUNK), nchunks, bufp<int32_t>(p, ws, B_XT_COLPTR),
                       bufp<int32_t>(p, ws, B_XT_ROW), bufp<float>(p, ws, B_XT_VA), bufp<float>(p, ws, B_XS_SCALE),
                       r0, rows, ld, stage);
    TPO_LAUNCH_CHECK();
  }
}

// Without the reduction (d_u <= 128): X' rows written densely (zero padded
// to dp columns); one wave per row builds the row in LDS first.
__global__ void __launch_bounds__(256)
k_xcsr_dense(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col, const float* __restrict__ val,
             int n, int64_t nnz, int du, int dp, float* __restrict__ xp, int32_t* __restrict__ err_bits) {
  __shared__ float rowbuf[4][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + w;
  if (r >= n) return;
  float* rb = rowbuf[w];
  for (int c = lane; c < dp; c += 64) rb[c] = 0.0f;
  wave_sync();
  int64_t b = rowptr[r], e = rowptr[r + 1];
  if ((b < 0 || e > nnz || b > e || (r == 0 && b != 0) || (r == n - 1 && e != nnz)) && lane == 0)
    atomicOr(err_bits, 128);
  b = min(max(b, static_cast<int64_t>(0)), nnz);
  e = min(max(e, b), nnz);
  for (int64_t t = b + lane; t < e; t += 64) {
    const int c = col[t];
    const float v = val[t];
    if (c < 0 || c >= du) {
      atomicOr(err_bits, 128);
    } else if (!isfinite(v)) {
      atomicOr(err_bits, 4);
    } else {
      atomicAdd(&rb[c], v);
    }
  }
  wave_sync();
  for (int c = lane; c < dp; c += 64) xp[r * dp + c] = rb[c];
}

void xcsr_dense(const Plan& p, void* ws, const int64_t* rowptr, const int32_t* col, const float* val, float* xp,
                hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  hipLaunchKernelGGL(k_xcsr_dense, dim3(ceil_div(p.n, 4)), dim3(256), 0, s, rowptr, col, val, p.n, p.xnnz, p.du, p.dp,
                     xp, &st->err_bits);
  TPO_LAUNCH_CHECK();
}

// out[i][c] = sum over the stored entries (j, x_ij) of row i of x_ij B[j][c]
// for c < lb (FP64 sums in the row's stored order, rounded to FP32), zero for
// lb <= c < wo.  One wave per row; lane q holds columns q and q + 64.
__global__ void __launch_bounds__(256)
k_xcsr_rowgather(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col, const float* __restrict__ val,
                 int n, int64_t nnz, int du, const double* __restrict__ B, int lb, int ldb, float* __restrict__ out,
                 int ldo, int wo) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (r >= n) return;
  const int64_t b = min(max(rowptr[r], static_cast<int64_t>(0)), nnz);
  const int64_t e = min(max(rowptr[r + 1], b), nnz);
  double a0 = 0.0, a1 = 0.0;
  for (int64_t t0 = b; t0 < e; t0 += 64) {
    const int cnt = static_cast<int>(min(static_cast<int64_t>(64), e - t0));
    int myc = 0;
    float myv = 0.0f;
    if (lane < cnt) {
      myc = col[t0 + lane];
      myv = val[t0 + lane];
      if (myc < 0 || myc >= du || !isfinite(myv)) {
        myc = 0;
        myv = 0.0f;
      }
    }
    for (int j = 0; j < cnt; ++j) {
      const int c = __shfl(myc, j, 64);
      const double v = static_cast<double>(__shfl(myv, j, 64));
      const double* brow = B + static_cast<int64_t>(c) * ldb;
      if (lane < lb) a0 = fma(v, brow[lane], a0);
      if (lane + 64 < lb) a1 = fma(v, brow[lane + 64], a1);
    }
  }
  float* orow = out + r * ldo;
  if (lane < wo) orow[lane] = lane < lb ? static_cast<float>(a0) : 0.0f;
  if (lane + 64 < wo) orow[lane + 64] = lane + 64 < lb ? static_cast<float>(a1) : 0.0f;
}

void xcsr_rowgather(const Plan& p, const int64_t* rowptr, const int32_t* col, const float* val, const double* B,
                    int lb, int ldb, float* out, int ldo, int wo, hipStream_t s) {
  hipLaunchKernelGGL(k_xcsr_rowgather, dim3(ceil_div(static_cast<int64_t>(p.n) * 64, 256)), dim3(256), 0, s, rowptr,
                     col, val, p.n, p.xnnz, p.du, B, lb, ldb, out, ldo, wo);
  TPO_LAUNCH_CHECK();
}

// Column chunks of the transpose: cinfo[j] = {first chunk, chunk count} and
// chunk[c] = {column, begin, end, staging cursor (= begin)}.  One workgroup;
// thread j takes column j's count, a sequential scan gives the offsets.
__global__ void __launch_bounds__(1024)
k_xcsc_chunks(const int32_t* __restrict__ colptr, int du, int4* __restrict__ chunk, int2* __restrict__ cinfo,
              int32_t* __restrict__ nchunks_out) {
  __shared__ int cnt[kXMaxDu];
  for (int j = threadIdx.x; j < du; j += blockDim.x) {
    const int len = colptr[j + 1] - colptr[j];
    cnt[j] = (len + kXChunk - 1) / kXChunk;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int j = 0; j < du; ++j) {
      const int c = cnt[j];
      cnt[j] = run;
      run += c;
    }
    *nchunks_out = run;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < du; j += blockDim.x) {
    const int b = colptr[j], e = colptr[j + 1];
    const int nc = (e - b + kXChunk - 1) / kXChunk;
    cinfo[j] = make_int2(cnt[j], nc);
    for (int q = 0; q < nc; ++q) {
      const int qb = b + q * kXChunk;
      chunk[cnt[j] + q] = make_int4(j, qb, min(e, qb + kXChunk), qb);
    }
  }
}

// One column chunk per workgroup: the four waves take consecutive quarters of
// the chunk's entries (lanes over the l columns of Y), then the quarters are
// added in order.  cpart[c][0..l) = sum of x_ij Y[i][:], cpart[c][l] = sum of
// x_ij (the column sum of X).
__global__ void __launch_bounds__(256)
k_xcsc_gather(const int4* __restrict__ chunk, const int32_t* __restrict__ nchunks, const int32_t* __restrict__ rows,
              const float* __restrict__ cval, const float* __restrict__ Y, int l, int ldy, double* __restrict__ cpart) {
  __shared__ double q4[4][129];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nc = *nchunks;
  for (int c = blockIdx.x; c < nc; c += gridDim.x) {
    const int4 ch = chunk[c];
    const int len = ch.z - ch.y;
    const int qb = ch.y + (len * w) / 4, qe = ch.y + (len * (w + 1)) / 4;
    double a0 = 0.0, a1 = 0.0, cs = 0.0;
    for (int t0 = qb; t0 < qe; t0 += 64) {
      const int cnt = min(64, qe - t0);
      int myr = 0;
      float myv = 0.0f;
      if (lane < cnt) {
        myr = rows[t0 + lane];
        myv = cval[t0 + lane];
      }
      for (int j = 0; j < cnt; ++j) {
        const int64_t rr = __shfl(myr, j, 64);
        const double v = static_cast<double>(__shfl(myv, j, 64));
        const float* yrow = Y + rr * ldy;
        if (lane < l) a0 = fma(v, static_cast<double>(yrow[lane]), a0);
        if (lane + 64 < l) a1 = fma(v, static_cast<double>(yrow[lane + 64]), a1);
        cs += v;
      }
    }
    q4[w][lane] = a0;
    if (lane + 64 <= 128) q4[w][lane + 64] = a1;
    if (lane == 0) q4[w][128] = cs;
    __syncthreads();
    double* o = cpart + static_cast<int64_t>(c) * (l + 1);
    for (int x = threadIdx.x; x <= l; x += 256) {
      const int src = x < l ? x : 128;
      o[x] = ((q4[0][src] + q4[1][src]) + q4[2][src]) + q4[3][src];
    }
    __syncthreads();
  }
}

// P[j][:] and colsum[j]: column j's chunk partials added in chunk order.
__global__ void __launch_bounds__(256)
k_xcsc_colsum(const int2* __restrict__ cinfo, const double* __restrict__ cpart, int du, int l, double* __restrict__ P,
              int ldp, double* __restrict__ colsum) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(du) * (l + 1)) return;
  const int j = static_cast<int>(idx / (l + 1)), x = static_cast<int>(idx % (l + 1));
  const int2 ci = cinfo[j];
  double s = 0.0;
  for (int q = 0; q < ci.y; ++q) s += cpart[static_cast<int64_t>(ci.x + q) * (l + 1) + x];
  if (x < l) {
    if (P) P[static_cast<int64_t>(j) * ldp + x] = s;
  } else {
    colsum[j] = s;
  }
}

void xcsc_make_chunks(const Plan& p, void* ws, hipStream_t s) {
  int32_t* nchunks = reinterpret_cast<int32_t*>(bufp<int2>(p, ws, B_XT_CINFO) + p.du);
  hipLaunchKernelGGL(k_xcsc_chunks, dim3(1), dim3(1024), 0, s, bufp<int32_t>(p, ws, B_XT_COLPTR), p.du,
                     bufp<int4>(p, ws, B_XT_CHUNK), bufp<int2>(p, ws, B_XT_CINFO), nchunks);
  TPO_LAUNCH_CHECK();
}

void xcsc_colgather(const Plan& p, void* ws, const float* Y, int l, int ldy, double* P, int ldp, double* colsum,
                    hipStream_t s) {
  const int32_t* nchunks = reinterpret_cast<const int32_t*>(bufp<int2>(p, ws, B_XT_CINFO) + p.du);
  hipLaunchKernelGGL(k_xcsc_gather, dim3(xcsc_grid(p)), dim3(256), 0, s, bufp<int4>(p, ws, B_XT_CHUNK), nchunks,
                     bufp<int32_t>(p, ws, B_XT_ROW), bufp<float>(p, ws, B_XT_VA), Y, l, ldy,
                     bufp<double>(p, ws, B_XT_CPART));
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_xcsc_colsum, dim3(ceil_div(static_cast<int64_t>(p.du) * (l + 1), 256)), dim3(256), 0, s,
                     bufp<int2>(p, ws, B_XT_CINFO), bufp<double>(p, ws, B_XT_CPART), p.du, l, P, ldp, colsum);
  TPO_LAUNCH_CHECK();
}

}  // namespace tpo
