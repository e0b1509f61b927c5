// Ingest (Section 2.1): the edge list becomes CSR(B_U) (rows U, columns V,
// columns ascending, duplicate pairs summed) and CSR(B_U^T) (rows V), the
// weighted degrees D_U and D_V, the scale vectors of the propagation and the
// hub-chunk work lists of the SpMM.
//
// Sorting is a stable LSD radix sort on packed (row, col) keys, 8 bits per
// pass, so the result is a deterministic function of the input.  The
// transpose is a stable sort of the deduplicated (row, col) list on its
// column bits only.
#include <algorithm>

#include "dev_common.hpp"
#include "tpo_internal.hpp"

namespace tpo {

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of uint32 (reduce-then-scan, three kernels).
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  // sh: kScanThreads/64 + 1 entries
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
      uint32_t c = sh[i];
      sh[i] = run;
      run += c;
    }
    sh[kScanThreads / 64] = run;
  }
  __syncthreads();
  uint32_t excl = x - v + sh[w];
  *total = sh[kScanThreads / 64];
  __syncthreads();
  return excl;
}

__global__ void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ bsum) {
  __shared__ uint32_t sh[kScanThreads / 64 + 1];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + static_cast<int64_t>(i) * kScanThreads + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  uint32_t tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_bsums(uint32_t* __restrict__ bsum, int nb, uint32_t* __restrict__ total_out) {
  __shared__ uint32_t sh[kScanThreads / 64 + 1];
  // each thread scans a contiguous run of entries sequentially
  const int per = (nb + kScanThreads - 1) / kScanThreads;
  const int beg = threadIdx.x * per;
  uint32_t s = 0;
  for (int i = 0; i < per; ++i)
    if (beg + i < nb) s += bsum[beg + i];
  uint32_t tot;
  uint32_t off = block_exclusive_scan(s, sh, &tot);
  for (int i = 0; i < per; ++i) {
    if (beg + i < nb) {
      uint32_t c = bsum[beg + i];
      bsum[beg + i] = off;
      off += c;
    }
  }
  if (threadIdx.x == 0 && total_out) *total_out = tot;
}

__global__ void k_scan_apply(const uint32_t* __restrict__ in, int64_t n, const uint32_t* __restrict__ bsum,
                             uint32_t* __restrict__ out) {
  __shared__ uint32_t sh[kScanThreads / 64 + 1];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  // blocked arrangement: thread t owns items [t*kScanItems, (t+1)*kScanItems)
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + static_cast<int64_t>(threadIdx.x) * kScanItems + i;
    v[i] = idx < n ? in[idx] : 0u;
    s += v[i];
  }
  uint32_t tot;
  uint32_t off = block_exclusive_scan(s, sh, &tot) + bsum[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + static_cast<int64_t>(threadIdx.x) * kScanItems + i;
    if (idx < n) out[idx] = off;
    off += v[i];
  }
}

// Exclusive scan of n entries; the grand total goes to *total (device) when
// given.  aux must hold ceil(n / kScanTile) entries.
static void scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* aux,
                           uint32_t* total, hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = ceil_div(n, kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, n, aux);
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kScanThreads), 0, s, aux, static_cast<int>(nb), total);
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, s, in, n, aux, out);
  TPO_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Keys and validation
// ---------------------------------------------------------------------------
__global__ void k_build_keys(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                             const float* __restrict__ ew, int64_t E, int n, int m, int colbits,
                             uint64_t* __restrict__ keys, float* __restrict__ wv,
                             int32_t* __restrict__ err_bits) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= E) return;
  int u = eu[i], v = ev[i];
  if (u < 0 || u >= n || v < 0 || v >= m) {
    atomicOr(err_bits, 1);
    u = 0;
    v = 0;
  }
  keys[i] = (static_cast<uint64_t>(u) << colbits) | static_cast<uint64_t>(v);
  if (ew) {
    float w = ew[i];
    if (!(w >= 0.0f) || !isfinite(w)) {
      atomicOr(err_bits, 2);
      w = 0.0f;
    }
    wv[i] = w;
  }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort pass (8-bit digit at `shift`)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t sort_count(int64_t n_static, const int32_t* n_dev) {
  return n_dev ? static_cast<int64_t>(*n_dev) : n_static;
}

__global__ void __launch_bounds__(kSortThreads)
k_radix_upsweep(const uint64_t* __restrict__ keys, int64_t n_static, const int32_t* n_dev, int shift,
                uint32_t* __restrict__ hist, int nb) {
  __shared__ uint32_t cnt[256];
  const int t = threadIdx.x;
  if (t < 256) cnt[t] = 0;
  __syncthreads();
  const int64_t n = sort_count(n_static, n_dev);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
  for (int r = 0; r < kSortItems; ++r) {
    int64_t idx = base + static_cast<int64_t>(r) * kSortThreads + t;
    if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (t < 256) hist[static_cast<int64_t>(t) * nb + blockIdx.x] = cnt[t];
}

// One tile's keys in digit order.  Wave w holds the tile's w-th eighth
// (keys w WK + 64 r + lane, r = 0..kSortItems-1), so the tile's order is
// (wave, r, lane).  Each wave ranks its own keys against a running count per
// digit in its own LDS row (eight ballots match a lane's digit; no barrier
// inside the loop), then one pass over the digits (thread t < 256 takes
// digit t) turns the eight waves' counts into their offsets and the tile's
// digit starts.  Equal digits keep
// the tile's order, so the sort is stable.  The keys are placed in LDS at
// their position in the tile's digit order and written out in that order:
// consecutive threads write consecutive addresses of one digit's run.
__global__ void __launch_bounds__(kSortThreads)
k_radix_downsweep(const uint64_t* __restrict__ keys, const float* __restrict__ vals, int64_t n_static,
                  const int32_t* n_dev, int shift, const uint32_t* __restrict__ hist_scan, int nb,
                  uint64_t* __restrict__ okeys, float* __restrict__ ovals) {
  constexpr int NW = kSortThreads / 64;
  constexpr int WK = kSortTile / NW;  // keys per wave
  __shared__ uint32_t goff[256];  // global start of each digit for this tile
  __shared__ uint32_t loff[256];  // start of each digit within the tile's order
  __shared__ uint32_t wcnt[NW][256];  // each wave's running digit counts, then its offsets
  __shared__ uint32_t wsum[NW];
  __shared__ uint64_t skeys[kSortTile];
  __shared__ float svals[kSortTile];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t n = sort_count(n_static, n_dev);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
  const int nvalid = static_cast<int>(max(static_cast<int64_t>(0), min(static_cast<int64_t>(kSortTile), n - base)));
  uint64_t key[kSortItems];
  float val[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int li = w * WK + r * 64 + lane;
    key[r] = li < nvalid ? keys[base + li] : 0ull;
    val[r] = (li < nvalid && vals) ? vals[base + li] : 0.0f;
  }
  static_assert(kSortThreads >= 256 && kSortThreads % 256 == 0, "one thread per digit");
  constexpr int DW = 256 / 64;  // waves that hold one digit per lane
  if (t < 256) {
    goff[t] = hist_scan[static_cast<int64_t>(t) * nb + blockIdx.x];
#pragma unroll
    for (int i = 0; i < NW; ++i) wcnt[i][t] = 0;
  }
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  uint32_t rk[kSortItems];  // rank among the wave's earlier keys of the same digit
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const bool valid = w * WK + r * 64 + lane < nvalid;
    const uint32_t d = static_cast<uint32_t>((key[r] >> shift) & 255u);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t before = wcnt[w][d];
    rk[r] = before + static_cast<uint32_t>(__popcll(peers & lt_mask));
    // the first lane of each digit advances the count (every lane of the wave
    // has read it above: a wave's LDS accesses complete in program order)
    if (valid && (peers & lt_mask) == 0) wcnt[w][d] = before + static_cast<uint32_t>(__popcll(peers));
  }
  __syncthreads();
  {
    // digit t: the waves' exclusive offsets, then the tile's exclusive scan
    // of the digit totals (waves 0..DW-1; the others only meet the barriers)
    uint32_t run = 0, v = 0;
    if (w < DW) {
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const uint32_t c = wcnt[i][t];
        wcnt[i][t] = run;
        run += c;
      }
      v = run;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
      }
      if (lane == 63) wsum[w] = v;
    }
    __syncthreads();
    if (w < DW) {
      uint32_t before = 0;
      for (int i = 0; i < w; ++i) before += wsum[i];
      loff[t] = before + v - run;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (w * WK + r * 64 + lane < nvalid) {
      const uint32_t d = static_cast<uint32_t>((key[r] >> shift) & 255u);
      const uint32_t lp = loff[d] + wcnt[w][d] + rk[r];
      skeys[lp] = key[r];
      if (vals) svals[lp] = val[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int j = r * kSortThreads + t;
    if (j < nvalid) {
      const uint64_t k = skeys[j];
      const uint32_t d = static_cast<uint32_t>((k >> shift) & 255u);
      const uint32_t pos = goff[d] + static_cast<uint32_t>(j) - loff[d];
      okeys[pos] = k;
      if (vals) ovals[pos] = svals[j];
    }
  }
}

// Sort keys[0..n) on bits [lo, hi) (stable), ping-pong through keys_alt;
// values follow when vals != nullptr.  The result ends in keys (copied back
// after an odd number of passes), or, with copy_back false, wherever the last
// pass left it: the return value says whether that is keys_alt / vals_alt.
// nb tiles of kSortTile keys; hist holds 256 nb counters, aux the scan's
// block sums.
static bool radix_sort_nb(int nb, uint32_t* hist, uint32_t* aux, uint64_t* keys, uint64_t* keys_alt, float* vals,
                          float* vals_alt, int64_t n_static, const int32_t* n_dev, int lo, int hi, hipStream_t s,
                          bool copy_back = true) {
  uint64_t* src = keys;
  uint64_t* dst = keys_alt;
  float* vsrc = vals;
  float* vdst = vals_alt;
  int passes = 0;
  for (int shift = lo; shift < hi; shift += 8) {
    hipLaunchKernelGGL(k_radix_upsweep, dim3(nb), dim3(kSortThreads), 0, s, src, n_static, n_dev, shift,
                       hist, nb);
    TPO_LAUNCH_CHECK();
    scan_exclusive(hist, hist, static_cast<int64_t>(nb) * 256, aux, nullptr, s);
    hipLaunchKernelGGL(k_radix_downsweep, dim3(nb), dim3(kSortThreads), 0, s, src, vsrc, n_static, n_dev,
                       shift, hist, nb, dst, vdst);
    TPO_LAUNCH_CHECK();
    std::swap(src, dst);
    std::swap(vsrc, vdst);
    ++passes;
  }
  if ((passes & 1) && !copy_back) return true;
  if (passes & 1) {
    TPO_HIP_CHECK(hipMemcpyAsync(keys, src, static_cast<size_t>(n_static) * sizeof(uint64_t),
                                 hipMemcpyDeviceToDevice, s));
    if (vals)
      TPO_HIP_CHECK(hipMemcpyAsync(vals, vsrc, static_cast<size_t>(n_static) * sizeof(float),
                                   hipMemcpyDeviceToDevice, s));
  }
  return false;
}

static bool radix_sort(const Plan& p, void* ws, uint64_t* keys, uint64_t* keys_alt, float* vals,
                       float* vals_alt, int64_t n_static, const int32_t* n_dev, int lo, int hi,
                       hipStream_t s, bool copy_back = true) {
  return radix_sort_nb(p.sort_blocks, bufp<uint32_t>(p, ws, B_HIST), bufp<uint32_t>(p, ws, B_SCAN_AUX), keys,
                       keys_alt, vals, vals_alt, n_static, n_dev, lo, hi, s, copy_back);
}

// ---------------------------------------------------------------------------
// Deduplication and CSR construction
// ---------------------------------------------------------------------------
__global__ void k_dedup_flags(const uint64_t* __restrict__ keys, int64_t E, uint32_t* __restrict__ flag) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= E) return;
  flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// For each first occurrence: write the unique (col) entry and its summed
// weight, and the transposed key (col << rowbits | row) for the second sort.
__global__ void k_dedup_write(const uint64_t* __restrict__ keys, const float* __restrict__ wv, int64_t E,
                              const uint32_t* __restrict__ upos, int colbits, int rowbits,
                              int32_t* __restrict__ col_u, float* __restrict__ val_u,
                              uint64_t* __restrict__ tkeys, float* __restrict__ tvals,
                              DevStatus* __restrict__ st) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= E) return;
  const uint64_t key = keys[i];
  if (i > 0 && keys[i - 1] == key) return;
  int64_t j = i;
  double w = 0.0;
  while (j < E && keys[j] == key) {
    w += wv ? static_cast<double>(wv[j]) : 1.0;
    ++j;
  }
  if (j - i > 1) atomicOr(&st->has_vals, 1);
  const uint32_t p = upos[i];
  const uint64_t colmask = (1ull << colbits) - 1ull;
  const uint32_t row = static_cast<uint32_t>(key >> colbits);
  const uint32_t col = static_cast<uint32_t>(key & colmask);
  col_u[p] = static_cast<int32_t>(col);
  val_u[p] = static_cast<float>(w);
  tkeys[p] = (static_cast<uint64_t>(col) << rowbits) | row;
  tvals[p] = static_cast<float>(w);
  if (j == E) st->n_unique = static_cast<int32_t>(p + 1);  // last run
}

// rowptr[r] = first position whose row is >= r, from sorted keys.
__global__ void k_rowptr(const uint64_t* __restrict__ keys, int64_t E_static, const int32_t* __restrict__ n_dev,
                         int shift, uint64_t mask, int nrows, int32_t* __restrict__ rowptr) {
  int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nu = n_dev ? *n_dev : E_static;
  if (p > nu) return;
  const int64_t row = (p < nu) ? static_cast<int64_t>((keys[p] >> shift) & mask) : nrows;
  const int64_t prev = (p == 0) ? -1 : static_cast<int64_t>((keys[p - 1] >> shift) & mask);
  for (int64_t r = prev + 1; r <= row && r <= nrows; ++r) rowptr[r] = static_cast<int32_t>(p);
}

__global__ void k_extract_cols(const uint64_t* __restrict__ tkeys, const float* __restrict__ tvals,
                               const int32_t* __restrict__ n_dev, int rowbits, int32_t* __restrict__ col_v,
                               float* __restrict__ val_v, int64_t E) {
  int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= E || p >= *n_dev) return;
  col_v[p] = static_cast<int32_t>(tkeys[p] & ((1ull << rowbits) - 1ull));
  val_v[p] = tvals[p];
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Weighted degree per row, the propagation scale and the hub chunk count.
// mode 0: U side, scale = D^-1/2; mode 1: V side, D^-1.  A wave owns 64
// consecutive rows at a time, one per lane, and a fixed grid walks the rows;
// summed edge weights (when present) are formed row by row by the whole wave
// in a fixed order.  Isolated rows are counted per workgroup and added to
// the total with one atomic per workgroup (a graph with many isolated rows
// would otherwise queue an atomic per wave on one address).
constexpr int kDegBlocks = 2048;

__global__ void __launch_bounds__(256)
k_degrees(const int32_t* __restrict__ rowptr, const float* __restrict__ val, int nrows,
          const DevStatus* __restrict__ st_ro, int mode, float* __restrict__ deg, float* __restrict__ scale,
          uint32_t* __restrict__ nchunk, uint32_t* __restrict__ ishub, int32_t* __restrict__ iso_count) {
  __shared__ int iso_blk;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) iso_blk = 0;
  __syncthreads();
  const bool has_vals = st_ro->has_vals != 0;
  int iso_w = 0;  // isolated rows seen by this wave (lane 0's count)
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x - lane; base < nrows;
       base += static_cast<int64_t>(gridDim.x) * 256) {
    const int r = static_cast<int>(base) + lane;
    const bool live = r < nrows;
    int b = 0, e = 0;
    if (live) {
      b = rowptr[r];
      e = rowptr[r + 1];
    }
    double s = static_cast<double>(e - b);
    if (has_vals) {
      // a row of at most 64 entries is summed by its own lane in stored order;
      // a longer one by the whole wave (strided partial sums, then a tree)
      double mine = 0.0;
      const bool serial = live && e - b <= 64;
      if (serial)
        for (int i = b; i < e; ++i) mine += static_cast<double>(val[i]);
      uint64_t longs = __ballot(live && !serial);
      while (longs) {
        const int j = __ffsll(static_cast<unsigned long long>(longs)) - 1;
        longs &= longs - 1;
        const int bj = __shfl(b, j, 64), ej = __shfl(e, j, 64);
        double t = 0.0;
        for (int i = bj + lane; i < ej; i += 64) t += static_cast<double>(val[i]);
        t = wave_sum(t);
        if (lane == j) mine = t;
      }
      s = mine;
    }
    if (live) {
      deg[r] = static_cast<float>(s);
      double sc = 0.0;
      if (s > 0.0) sc = (mode == 0) ? 1.0 / sqrt(s) : 1.0 / s;
      scale[r] = static_cast<float>(sc);
      const int cnt = e - b;
      const uint32_t nc = cnt > kHubChunk ? static_cast<uint32_t>((cnt + kHubChunk - 1) / kHubChunk) : 0u;
      nchunk[r] = nc;
      ishub[r] = nc > 0 ? 1u : 0u;
    }
    iso_w += __popcll(__ballot(live && !(s > 0.0)));
  }
  if (lane == 0 && iso_w != 0) atomicAdd(&iso_blk, iso_w);
  __syncthreads();
  if (threadIdx.x == 0 && iso_blk != 0) atomicAdd(iso_count, iso_blk);
}

__global__ void k_hub_lists(const int32_t* __restrict__ rowptr, int nrows, const uint32_t* __restrict__ nchunk_raw,
                            const uint32_t* __restrict__ chunk_off, const uint32_t* __restrict__ hub_idx,
                            int4* __restrict__ chunks, int4* __restrict__ hubs) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int b = rowptr[r], e = rowptr[r + 1];
  const int cnt = e - b;
  if (cnt <= kHubChunk) return;
  const int nc = (cnt + kHubChunk - 1) / kHubChunk;
  const int off = static_cast<int>(chunk_off[r]);
  hubs[hub_idx[r]] = make_int4(r, off, nc, 0);
  for (int c = 0; c < nc; ++c) {
    const int cb = b + c * kHubChunk;
    const int ce = min(cb + kHubChunk, e);
    chunks[off + c] = make_int4(r, cb, ce, off + c);
  }
  (void)nchunk_raw;
}

static void side_lists(const Plan& p, void* ws, int nrows, const int32_t* rowptr, const float* val, int mode,
                       Buf deg_b, Buf scale_b, Buf cnt_b, Buf hub_b, Buf chunk_b, Buf hublist_b,
                       int32_t* iso, int32_t* n_chunks, int32_t* n_hubs, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  uint32_t* nchunk = bufp<uint32_t>(p, ws, cnt_b);
  uint32_t* ishub = bufp<uint32_t>(p, ws, hub_b);
  uint32_t* aux = bufp<uint32_t>(p, ws, B_SCAN_AUX);
  hipLaunchKernelGGL(k_degrees, dim3(std::max<int64_t>(1, std::min<int64_t>(ceil_div(static_cast<int64_t>(nrows), 256), kDegBlocks))), dim3(256), 0, s, rowptr,
                     val, nrows, st, mode, bufp<float>(p, ws, deg_b), bufp<float>(p, ws, scale_b), nchunk, ishub,
                     iso);
  TPO_LAUNCH_CHECK();
  scan_exclusive(nchunk, nchunk, nrows, aux, reinterpret_cast<uint32_t*>(n_chunks), s);
  scan_exclusive(ishub, ishub, nrows, aux, reinterpret_cast<uint32_t*>(n_hubs), s);
  hipLaunchKernelGGL(k_hub_lists, dim3(ceil_div(nrows, 256)), dim3(256), 0, s, rowptr, nrows, nchunk, nchunk,
                     ishub, bufp<int4>(p, ws, chunk_b), bufp<int4>(p, ws, hublist_b));
  TPO_LAUNCH_CHECK();
}

void launch_ingest(const Plan& p, void* ws, const tpo_inputs* in, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  const int64_t E = p.E;
  uint64_t* ka = bufp<uint64_t>(p, ws, B_KEYS_A);
  uint64_t* kb = bufp<uint64_t>(p, ws, B_KEYS_B);
  float* wa = bufp<float>(p, ws, B_WV_A);
  float* wb = bufp<float>(p, ws, B_WV_B);
  int32_t* rowptr_u = bufp<int32_t>(p, ws, B_ROWPTR_U);
  int32_t* rowptr_v = bufp<int32_t>(p, ws, B_ROWPTR_V);
  int32_t* col_u = bufp<int32_t>(p, ws, B_COL_U);
  int32_t* col_v = bufp<int32_t>(p, ws, B_COL_V);
  float* val_u = bufp<float>(p, ws, B_VAL_U);
  float* val_v = bufp<float>(p, ws, B_VAL_V);
  uint32_t* upos = bufp<uint32_t>(p, ws, B_UPOS);
  uint32_t* aux = bufp<uint32_t>(p, ws, B_SCAN_AUX);
  const uint64_t rowmask = (1ull << p.rowbits) - 1ull;
  const uint64_t colmask = (1ull << p.colbits) - 1ull;

  if (E > 0) {
    float* win = p.prob.weighted ? wa : nullptr;
    hipLaunchKernelGGL(k_build_keys, dim3(ceil_div(E, 256)), dim3(256), 0, s, in->edge_u, in->edge_v,
                       p.prob.weighted ? in->edge_w : nullptr, E, p.n, p.m, p.colbits, ka, win, &st->err_bits);
    TPO_LAUNCH_CHECK();
    // (row, col) order: all bits of the packed key; weights follow
    radix_sort(p, ws, ka, kb, win, p.prob.weighted ? wb : nullptr, E, nullptr, 0, p.rowbits + p.colbits, s);
    hipLaunchKernelGGL(k_dedup_flags, dim3(ceil_div(E, 256)), dim3(256), 0, s, ka, E, upos);
    TPO_LAUNCH_CHECK();
    scan_exclusive(upos, upos, E, aux, nullptr, s);
    // unique entries of B_U; transposed keys (col << rowbits | row) to kb and
    // their summed weights to wb
    hipLaunchKernelGGL(k_dedup_write, dim3(ceil_div(E, 256)), dim3(256), 0, s, ka, win, E, upos, p.colbits,
                       p.rowbits, col_u, val_u, kb, wb, st);
    TPO_LAUNCH_CHECK();
    // kb is in (row, col) order here: its low rowbits are the rows of B_U
    hipLaunchKernelGGL(k_rowptr, dim3(ceil_div(E + 1, 256)), dim3(256), 0, s, kb, E, &st->n_unique, 0, rowmask,
                       p.n, rowptr_u);
    TPO_LAUNCH_CHECK();
    // B_U^T: stable sort on the column bits only keeps rows ascending per
    // column; read from whichever buffers the last pass wrote
    const bool alt = radix_sort(p, ws, kb, ka, wb, wa, E, &st->n_unique, p.rowbits, p.rowbits + p.colbits, s,
                                false);
    const uint64_t* tk = alt ? ka : kb;
    const float* tw = alt ? wa : wb;
    hipLaunchKernelGGL(k_rowptr, dim3(ceil_div(E + 1, 256)), dim3(256), 0, s, tk, E, &st->n_unique, p.rowbits,
                       colmask, p.m, rowptr_v);
    TPO_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_extract_cols, dim3(ceil_div(E, 256)), dim3(256), 0, s, tk, tw, &st->n_unique, p.rowbits,
                       col_v, val_v, E);
    TPO_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div(p.n + 1, 256)), dim3(256), 0, s, rowptr_u,
                       static_cast<int64_t>(p.n + 1), 0);
    TPO_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div(p.m + 1, 256)), dim3(256), 0, s, rowptr_v,
                       static_cast<int64_t>(p.m + 1), 0);
    TPO_LAUNCH_CHECK();
  }
  side_lists(p, ws, p.n, rowptr_u, val_u, 0, B_DEG_U, B_ISQ_U, B_HUBCNT_U, B_HUBROW_U, B_CHUNK_U, B_HUBLIST_U,
             &st->iso_u, &st->hub_chunks_u, &st->hub_rows_u, s);
  side_lists(p, ws, p.m, rowptr_v, val_v, 1, B_DEG_V, B_INV_V, B_HUBCNT_V, B_HUBROW_V, B_CHUNK_V, B_HUBLIST_V,
             &st->iso_v, &st->hub_chunks_v, &st->hub_rows_v, s);
  save_graph_status(p, ws, s);
}

// ---------------------------------------------------------------------------
// The ingested graph's status, kept for resident jobs
// ---------------------------------------------------------------------------
__global__ void k_save_graph_status(const DevStatus* __restrict__ st, int n, int m, int64_t E,
                                    GraphStatus* __restrict__ g) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  g->n = n;
  g->m = m;
  g->n_edges = static_cast<int32_t>(E);
  g->has_vals = st->has_vals;
  g->n_unique = st->n_unique;
  g->iso_u = st->iso_u;
  g->iso_v = st->iso_v;
  g->hub_chunks_u = st->hub_chunks_u;
  g->hub_rows_u = st->hub_rows_u;
  g->hub_chunks_v = st->hub_chunks_v;
  g->hub_rows_v = st->hub_rows_v;
  g->err_bits = st->err_bits & 3;
  g->magic = kGraphMagic;
}

__global__ void k_restore_graph_status(const GraphStatus* __restrict__ g, DevStatus* __restrict__ st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->has_vals = g->has_vals;
  st->n_unique = g->n_unique;
  st->iso_u = g->iso_u;
  st->iso_v = g->iso_v;
  st->hub_chunks_u = g->hub_chunks_u;
  st->hub_rows_u = g->hub_rows_u;
  st->hub_chunks_v = g->hub_chunks_v;
  st->hub_rows_v = g->hub_rows_v;
  st->err_bits |= g->err_bits;
}

void save_graph_status(const Plan& p, void* ws, hipStream_t s) {
  hipLaunchKernelGGL(k_save_graph_status, dim3(1), dim3(64), 0, s, bufp<DevStatus>(p, ws, B_STATUS), p.n, p.m, p.E,
                     bufp<GraphStatus>(p, ws, B_GSTATUS));
  TPO_LAUNCH_CHECK();
}

void restore_graph_status(const Plan& p, void* ws, hipStream_t s) {
  hipLaunchKernelGGL(k_restore_graph_status, dim3(1), dim3(64), 0, s, bufp<GraphStatus>(p, ws, B_GSTATUS),
                     bufp<DevStatus>(p, ws, B_STATUS));
  TPO_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Sparse attributes (TPO_X_CSR): the transpose of X_U (CSC), for the column
// products of the reduction's refinement step
// ---------------------------------------------------------------------------
// Keys (col << rowbits | row) and values of the stored entries in CSR order,
// one wave per row.  Row starts are clamped to [0, nnz] and an entry whose
// column is out of range keeps column 0 with value 0 (the status word then
// holds bit 7, reported as TPO_ERANGE), so every later access stays in bounds.
__global__ void __launch_bounds__(256)
k_xcsr_keys(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col, const float* __restrict__ val,
            int n, int64_t nnz, int du, int rowbits, uint64_t* __restrict__ keys, float* __restrict__ vals,
            int32_t* __restrict__ err_bits) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (r >= n) return;
  int64_t b = rowptr[r], e = rowptr[r + 1];
  const bool bad_row = b < 0 || e > nnz || b > e || (r == 0 && b != 0) || (r == n - 1 && e != nnz);
  b = min(max(b, static_cast<int64_t>(0)), nnz);
  e = min(max(e, b), nnz);
  if (bad_row && lane == 0) atomicOr(err_bits, 128);
  for (int64_t i = b + lane; i < e; i += 64) {
    int c = col[i];
    float v = val[i];
    if (c < 0 || c >= du) {
      atomicOr(err_bits, 128);
      c = 0;
      v = 0.0f;
    }
    if (!isfinite(v)) {
      atomicOr(err_bits, 4);
      v = 0.0f;
    }
    keys[i] = (static_cast<uint64_t>(c) << rowbits) | static_cast<uint64_t>(r);
    vals[i] = v;
  }
}

static int key_bits(int64_t n) {
  int b = 1;
  while ((int64_t{1} << b) < n) ++b;
  return b;
}

__global__ void k_split_keys(const uint64_t* __restrict__ keys, int64_t nnz, int rowbits, int32_t* __restrict__ rows) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < nnz) rows[i] = static_cast<int32_t>(keys[i] & ((1ull << rowbits) - 1ull));
}

void xcsr_transpose(const Plan& p, void* ws, const int64_t* rowptr, const int32_t* col, const float* val,
                    hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  uint64_t* ka = bufp<uint64_t>(p, ws, B_XT_KA);
  uint64_t* kb = bufp<uint64_t>(p, ws, B_XT_KB);
  float* va = bufp<float>(p, ws, B_XT_VA);
  float* vb = bufp<float>(p, ws, B_XT_VB);
  int32_t* colptr = bufp<int32_t>(p, ws, B_XT_COLPTR);
  const int64_t nnz = p.xnnz;
  const int rowbits = key_bits(p.n);
  const int colbits = key_bits(p.du);
  if (nnz > 0) {
    hipLaunchKernelGGL(k_xcsr_keys, dim3(ceil_div(static_cast<int64_t>(p.n) * 64, 256)), dim3(256), 0, s, rowptr,
                       col, val, p.n, nnz, p.du, rowbits, ka, va, &st->err_bits);
    TPO_LAUNCH_CHECK();
    // stable sort on the column bits: rows stay ascending within a column
    radix_sort_nb(p.xsort_blocks, bufp<uint32_t>(p, ws, B_XT_HIST), bufp<uint32_t>(p, ws, B_XT_AUX), ka, kb, va,
                  vb, nnz, nullptr, rowbits, rowbits + colbits, s);
    hipLaunchKernelGGL(k_rowptr, dim3(ceil_div(nnz + 1, 256)), dim3(256), 0, s, ka, nnz, nullptr, rowbits,
                       (1ull << colbits) - 1ull, p.du, colptr);
    TPO_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_split_keys, dim3(ceil_div(nnz, 256)), dim3(256), 0, s, ka, nnz, rowbits,
                       bufp<int32_t>(p, ws, B_XT_ROW));
    TPO_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div(p.du + 1, 256)), dim3(256), 0, s, colptr,
                       static_cast<int64_t>(p.du + 1), 0);
    TPO_LAUNCH_CHECK();
  }
}

}  // namespace tpo
