// Dense stages: the attribute reduction (Section 3.2.1), the random features
// (Algorithm 1) and RandomizedSVD(R, k) (Algorithm 2).
//
// Both randomized SVDs run the subspace iteration on a Gram matrix that is
// formed once in FP64 (C = X^T X for the reduction, K = R^T R for the
// embedding).  For the embedding this is the same iteration as
// Y <- orth(R orth(R^T Y)) re-associated through K: the basis of R's column
// space is R M L^{-T}, with M the 2d x k' right factor and L the Cholesky
// factor of M^T K M, so no n x k' block is ever materialised; Gamma = R S is
// formed by one final pass (k_cluster.hip).
#include "blk_chol16.hpp"
#include "blk_linalg.hpp"
#include "dev_common.hpp"
#include "tpo_internal.hpp"

namespace tpo {

// ---------------------------------------------------------------------------
// FP64 Gram of a tall FP32 matrix: G = X^T X and the column sums of X.
// Grid: (upper-triangular 64x64 tile pairs, row chunks).  Each workgroup
// accumulates its tile over its chunk of rows in FP64 (products of FP32
// values are exact in FP64) and writes a partial; k_gram_reduce adds the
// partials in chunk order.
// ---------------------------------------------------------------------------
constexpr int kGT = 64;
constexpr int kGSub = 64;
constexpr int kGLd = kGT + 4;

// One 64 x 64 tile pair (ti <= tj) of the Gram over one chunk of rows, on
// FP64 MFMA 16x16x4: 64-row slabs of both column tiles are staged in LDS (as
// FP32; converted exactly to FP64 at the operand read), with the next slab's
// global loads in flight during the current slab's MFMAs.  Wave w owns the
// 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 MFMA tiles.  Operand layout: lane
// l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; result v of lane l is
// D[4 v + l / 16][l % 16].  part: [chunk][pair][64 x 64].
__global__ void __launch_bounds__(256)
k_gram_part(const float* __restrict__ X, int64_t n, int c, int64_t ldx, int ntiles, int rows_per_chunk,
            double* __restrict__ part, double* __restrict__ colsum_part) {
  constexpr int PER = kGSub * kGT / 256;  // slab elements per thread
  __shared__ float As[kGSub * kGLd];
  __shared__ float Bs[kGSub * kGLd];
  __shared__ double csum[4][kGT];
  int pi = blockIdx.x, ti = 0;
  while (pi >= ntiles - ti) {
    pi -= ntiles - ti;
    ++ti;
  }
  const int tj = ti + pi;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int qa = w >> 1, qb = w & 1;
  const int64_t r_beg = static_cast<int64_t>(blockIdx.y) * rows_per_chunk;
  const int64_t r_end = min(n, r_beg + rows_per_chunk);
  const bool diag = ti == tj;
  const float* Bp = diag ? As : Bs;
  v4d_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d_t{0.0, 0.0, 0.0, 0.0};
  double cs = 0.0;
  float ra[PER], rb[PER];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      const int rr = e >> 6, jj = e & 63;
      const int64_t row = r0 + rr;
      const int ca = ti * kGT + jj, cb = tj * kGT + jj;
      ra[u] = (row < r_end && ca < c) ? X[row * ldx + ca] : 0.0f;
      rb[u] = (!diag && row < r_end && cb < c) ? X[row * ldx + cb] : 0.0f;
    }
  };
  if (r_beg < r_end) fetch(r_beg);
  for (int64_t r0 = r_beg; r0 < r_end; r0 += kGSub) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      As[(e >> 6) * kGLd + (e & 63)] = ra[u];
      if (!diag) Bs[(e >> 6) * kGLd + (e & 63)] = rb[u];
    }
    __syncthreads();
    if (r0 + kGSub < r_end) fetch(r0 + kGSub);
#pragma unroll
    for (int st = 0; st < kGSub / 4; ++st) {
      const int k = 4 * st + kq;
      const double a0 = As[k * kGLd + 32 * qa + i16], a1 = As[k * kGLd + 32 * qa + 16 + i16];
      const double b0 = Bp[k * kGLd + 32 * qb + i16], b1 = Bp[k * kGLd + 32 * qb + 16 + i16];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (diag && colsum_part) {
      for (int rr = w; rr < kGSub; rr += 4) cs += static_cast<double>(As[rr * kGLd + lane]);
    }
    __syncthreads();
  }
  const int npairs = ntiles * (ntiles + 1) / 2;
  double* out = part + (static_cast<int64_t>(blockIdx.y) * npairs + blockIdx.x) * kGT * kGT;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(32 * qa + 16 * a + 4 * v + kq) * kGT + 32 * qb + 16 * b + i16] = acc[a][b][v];
  if (diag && colsum_part) {
    csum[w][lane] = cs;
    __syncthreads();
    if (tid < kGT) {
      const double v = ((csum[0][tid] + csum[1][tid]) + csum[2][tid]) + csum[3][tid];
      const int j = ti * kGT + tid;
      if (j < c) colsum_part[static_cast<int64_t>(blockIdx.y) * c + j] = v;
    }
  }
}

// G (c x c, both triangles) = sum over chunks of the tile partials, in chunk
// order; every load of a batch is issued before its sums.
constexpr int kGramBatch = 16;

__global__ void __launch_bounds__(256)
k_gram_reduce(const double* __restrict__ part, const double* __restrict__ colsum_part, int nchunks, int c,
              int ntiles, const float* __restrict__ scale, double* __restrict__ G, double* __restrict__ colsum) {
  const int npairs = ntiles * (ntiles + 1) / 2;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx < static_cast<int64_t>(npairs) * kGT * kGT) {
    const int pr = static_cast<int>(idx / (kGT * kGT)), e = static_cast<int>(idx % (kGT * kGT));
    int pi = pr, ti = 0;
    while (pi >= ntiles - ti) {
      pi -= ntiles - ti;
      ++ti;
    }
    const int tj = ti + pi;
    const int i = ti * kGT + e / kGT, j = tj * kGT + e % kGT;
    const double* src = part + idx;
    const int64_t stride = static_cast<int64_t>(npairs) * kGT * kGT;
    double s = 0.0;
    for (int ch0 = 0; ch0 < nchunks; ch0 += kGramBatch) {
      double v[kGramBatch];
#pragma unroll
      for (int u = 0; u < kGramBatch; ++u) v[u] = ch0 + u < nchunks ? src[(ch0 + u) * stride] : 0.0;
#pragma unroll
      for (int u = 0; u < kGramBatch; ++u) s += v[u];
    }
    if (i < c && j < c) {
      // column scales of an FP8 X: C_ij = s_i s_j (sum of the raw products);
      // s_i s_j is exact in FP64
      if (scale) s *= static_cast<double>(scale[i]) * static_cast<double>(scale[j]);
      G[static_cast<int64_t>(i) * c + j] = s;
      G[static_cast<int64_t>(j) * c + i] = s;
    }
  }
  if (colsum && idx < c) {
    double s = 0.0;
    for (int ch0 = 0; ch0 < nchunks; ch0 += kGramBatch) {
      double v[kGramBatch];
#pragma unroll
      for (int u = 0; u < kGramBatch; ++u)
        v[u] = ch0 + u < nchunks ? colsum_part[static_cast<int64_t>(ch0 + u) * c + idx] : 0.0;
#pragma unroll
      for (int u = 0; u < kGramBatch; ++u) s += v[u];
    }
    colsum[idx] = scale ? s * static_cast<double>(scale[idx]) : s;
  }
}

typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));
typedef unsigned int v4u_t __attribute__((ext_vector_type(4)));

// The same partials for a narrow-type X (the attribute precision forms):
// FMT 1 = bfloat16 on BF16 MFMA 16x16x32, FMT 2 = FP8 E4M3 (raw codes; the
// column scales are applied when the partials are summed) on the gfx950 FP8
// MFMA 16x16x128 with unit block scales.  Products of two BF16 or two E4M3
// values are exact in FP32; each output's FP32 sums over a block of kNFlush
// rows are added into FP64 registers, so an entry's error is at most
// kNFlush u times the sum of its products' magnitudes (u = 2^-24).
//
// A workgroup of 8 waves owns one 128 x 128 tile pair (ti <= tj) of the Gram
// over one row chunk.  Each slab (256 bytes of every column: 128 BF16 rows or
// 256 FP8 rows) of both column tiles is staged row-major in LDS as it is read
// (16-byte pieces of a row, row stride kNRowLd bytes), double-buffered, with
// the next slab's global loads in flight in registers.  The MFMA operands,
// which run down columns, come out of the row-major slab through gfx950's
// transposing LDS reads: within each group of 16 lanes, ds_read_b64_tr_b16
// gives lane j element j mod 4 of the 8-byte pieces read by lanes
// 4 r + j / 4 (r = 0..3), and ds_read_b64_tr_b8 byte j mod 8 of those of
// lanes 2 r + j / 8 (r = 0..7).  So when lane 4 r + q (2 r + q) points at row
// r of a 4- (8-) row block, columns 4 q (8 q) on, lane j receives column j of
// the block: two reads give a BF16 operand's 8 rows, four an FP8 operand's
// 32.  Wave w computes the 64 x 32 block (rows 64 (w / 4) .., columns
// 32 (w % 4) ..) as 4 x 2 MFMA tiles.  On a diagonal tile the two waves below
// the diagonal (w = 4, 5) form the tile's column sums instead.  Operand
// layout: lane l supplies the rows of k-group l / 16 of its column l % 16 for
// both operands (the same rows for A and B, so the contraction does not
// depend on the order inside the instruction); result v of lane l is
// D[4 (l / 16) + v][l % 16].
//
// Workgroups are dispatched to the eight XCDs in turn (workgroup b runs on
// XCD b % 8); every tile pair of one row chunk goes to the same XCD, so the
// chunk's rows are fetched from memory about once per XCD and served to the
// other pairs from its L2.  vec: X 16-byte aligned and the row stride a
// multiple of 16 bytes (16-byte loads); otherwise element loads.
constexpr int kNT = 128;       // column tile
constexpr int kNColB = 256;    // staged bytes of one column per slab
constexpr int kNFlush = 256;   // rows per FP32 block
typedef int v8i_t __attribute__((ext_vector_type(8)));
typedef int v2i_t __attribute__((ext_vector_type(2)));
typedef short v4s_t __attribute__((ext_vector_type(4)));
typedef short v8s_t __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) v2i_t lds_v2i_t;
typedef __attribute__((address_space(3))) v4s_t lds_v4s_t;

// LDS row stride of a staged slab (bytes): 128 columns, then padding that
// puts the rows one transposing read touches (4 of 32 bytes for BF16, 8 of
// 16 bytes for FP8) in distinct banks
template <int ES>
__host__ __device__ constexpr int narrow_row_ld() { return ES == 2 ? 2 * kNT + 32 : kNT + 16; }
// bytes of one staged operand (a slab of one column tile)
template <int ES>
__host__ __device__ constexpr int narrow_op_bytes() { return (kNColB / ES) * narrow_row_ld<ES>(); }

// the transposing LDS reads at a byte offset of an LDS array
__device__ __forceinline__ v2i_t lds_tr8(const uint8_t* lds_base, int off) {
  return __builtin_amdgcn_ds_read_tr8_b64_v2i32(
      (lds_v2i_t*)((__attribute__((address_space(3))) uint8_t*)(lds_base) + off));
}
__device__ __forceinline__ v4s_t lds_tr16(const uint8_t* lds_base, int off) {
  return __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (lds_v4s_t*)((__attribute__((address_space(3))) uint8_t*)(lds_base) + off));
}

// An FP8 E4M3 attribute (raw byte) as FP32, exactly.
__device__ __forceinline__ float fp8_to_f32(uint32_t byte) {
  return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(byte), 0);
}

template <int FMT>
__global__ void __launch_bounds__(512)
k_gram_narrow(const uint8_t* __restrict__ X, int64_t n, int c, int64_t ldx, int ntiles, int rows_per_chunk,
              int nchunks, int vec, double* __restrict__ part, double* __restrict__ colsum_part, int accumulate) {
  constexpr int ES = FMT == 1 ? 2 : 1;  // bytes per element
  constexpr int SR = kNColB / ES;       // rows per slab
  constexpr int EPG = 16 / ES;          // elements per 16-byte piece
  constexpr int CPR = kNT / EPG;        // 16-byte pieces per row of a column tile
  constexpr int HR = SR * CPR / 256;    // pieces a staging thread moves (8)
  constexpr int KS = FMT == 1 ? SR / 32 : SR / 128;  // MFMA k steps per slab
  constexpr int FLUSH_SLABS = kNFlush / SR;
  constexpr int RLD = narrow_row_ld<ES>(), OPB = narrow_op_bytes<ES>();
  __shared__ __align__(16) uint8_t lds[2 * 2 * OPB];  // [buffer][operand]
  const int npairs = ntiles * (ntiles + 1) / 2;
  const int b = blockIdx.x;
  const int xcd = b % 8, slot = b / 8;
  const int per_xcd = (nchunks + 7) / 8;
  const int chunk = slot / npairs + per_xcd * xcd;
  if (chunk >= nchunks) return;  // uniform: the padding of the grid
  const int pair = slot % npairs;
  int pi = pair, ti = 0;
  while (pi >= ntiles - ti) {
    pi -= ntiles - ti;
    ++ti;
  }
  const int tj = ti + pi;
  const bool diag = ti == tj;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int qa = w >> 2, qb = w & 3;
  const bool colsum_wave = diag && qa == 1 && qb < 2;  // wave-uniform
  const int64_t r_beg = static_cast<int64_t>(chunk) * rows_per_chunk;
  const int64_t r_end = min(n, r_beg + rows_per_chunk);
  const int nslabs = r_end > r_beg ? static_cast<int>((r_end - r_beg + SR - 1) / SR) : 0;

  // staging: threads 0..255 stage column tile ti, 256..511 tile tj (idle on a
  // diagonal tile); piece e = sb + 256 h of the slab is 16-byte piece e % CPR
  // of row e / CPR (consecutive threads read consecutive pieces of a row)
  const int op = tid >> 8, sb = tid & 255;
  const bool loader = !(diag && op == 1);
  const int tcol0 = (op ? tj : ti) * kNT;  // first column of the staged tile
  uint32_t pre[HR][4];
  auto fetch = [&](int64_t r0, uint32_t (&pf)[HR][4]) {
#pragma unroll
    for (int h = 0; h < HR; ++h) {
      const int e = sb + 256 * h;
      const int64_t row = r0 + e / CPR;
      const int gcol = tcol0 + (e % CPR) * EPG;
#pragma unroll
      for (int d = 0; d < 4; ++d) pf[h][d] = 0u;
      if (!loader || row >= r_end || gcol >= c) continue;
      const uint8_t* src = X + (row * ldx + gcol) * ES;
      if (vec && gcol + EPG <= c) {
        const v4u_t v = *reinterpret_cast<const v4u_t*>(src);
#pragma unroll
        for (int d = 0; d < 4; ++d) pf[h][d] = v[d];
      } else {
#pragma unroll
        for (int el = 0; el < EPG; ++el) {
          if (gcol + el >= c) break;
          const uint32_t val = ES == 2 ? static_cast<uint32_t>(reinterpret_cast<const uint16_t*>(src)[el])
                                       : static_cast<uint32_t>(src[el]);
          pf[h][(el * ES) / 4] |= val << (8 * ((el * ES) % 4));
        }
      }
    }
  };
  auto store = [&](int buf, const uint32_t (&ps)[HR][4]) {
    if (!loader) return;
    uint8_t* base = lds + (2 * buf + op) * OPB;
#pragma unroll
    for (int h = 0; h < HR; ++h) {
      const int e = sb + 256 * h;
      *reinterpret_cast<v4u_t*>(base + (e / CPR) * RLD + (e % CPR) * 16) =
          v4u_t{ps[h][0], ps[h][1], ps[h][2], ps[h][3]};
    }
  };
  // lane offsets of the transposing reads inside a 16-lane group: the row
  // within the block and the byte offset of the lane's 8-byte piece
  const int tr_row = ES == 2 ? (i16 >> 2) : (i16 >> 1);
  const int tr_col = ES == 2 ? 8 * (i16 & 3) : 8 * (i16 & 1);
  v4f_t s32[4][2];
  v4d_t acc[4][2];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      s32[m][mb] = v4f_t{0.f, 0.f, 0.f, 0.f};
      acc[m][mb] = v4d_t{0.0, 0.0, 0.0, 0.0};
    }
  double cs = 0.0;  // column sum of column 64 qb + lane (colsum waves)

  auto mma = [&](int buf) {
    const uint8_t* la = lds + (2 * buf) * OPB;
    const uint8_t* lb = diag ? la : la + OPB;
    if constexpr (FMT == 1) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        // rows 32 ks + 8 kq + (0..3), then + 4
        const int roff = (32 * ks + 8 * kq + tr_row) * RLD + tr_col;
        v8bf_t av[4], bv[2];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int off = roff + 2 * (64 * qa + 16 * m);
          const v4s_t lo = lds_tr16(la, off), hi = lds_tr16(la, off + 4 * RLD);
          av[m] = __builtin_bit_cast(v8bf_t, v8s_t{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]});
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          const int off = roff + 2 * (32 * qb + 16 * mb);
          const v4s_t lo = lds_tr16(lb, off), hi = lds_tr16(lb, off + 4 * RLD);
          bv[mb] = __builtin_bit_cast(v8bf_t, v8s_t{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]});
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int mb = 0; mb < 2; ++mb)
            s32[m][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv[mb], s32[m][mb], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        // rows 128 ks + 32 kq + 8 h + (0..7), h = 0..3
        const int roff = (128 * ks + 32 * kq + tr_row) * RLD + tr_col;
        v8i_t av[4], bv[2];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int off = roff + 64 * qa + 16 * m;
          const v2i_t x0 = lds_tr8(la, off), x1 = lds_tr8(la, off + 8 * RLD);
          const v2i_t x2 = lds_tr8(la, off + 16 * RLD), x3 = lds_tr8(la, off + 24 * RLD);
          av[m] = v8i_t{x0[0], x0[1], x1[0], x1[1], x2[0], x2[1], x3[0], x3[1]};
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          const int off = roff + 32 * qb + 16 * mb;
          const v2i_t x0 = lds_tr8(lb, off), x1 = lds_tr8(lb, off + 8 * RLD);
          const v2i_t x2 = lds_tr8(lb, off + 16 * RLD), x3 = lds_tr8(lb, off + 24 * RLD);
          bv[mb] = v8i_t{x0[0], x0[1], x1[0], x1[1], x2[0], x2[1], x3[0], x3[1]};
        }
        // formats 0 (E4M3) for both operands; block scales 127 (2^0)
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int mb = 0; mb < 2; ++mb)
            s32[m][mb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av[m], bv[mb], s32[m][mb], 0, 0, 0, 127,
                                                                          0, 127);
      }
    }
  };
  // column sums of the staged slab (column 64 qb + lane of tile ti, read
  // down the column with the same transposing reads): BF16 in FP32 groups of
  // 8 rows, E4M3 in FP32 groups of 64 rows (exact: E4M3 values are multiples
  // of 2^-9 below 2^9, so 64 of them sum below 2^24 units), each group added
  // into FP64
  auto colsum = [&](int buf) {
    const uint8_t* la = lds + (2 * buf) * OPB;
    const int coff = tr_row * RLD + tr_col + ES * (64 * qb + 16 * kq);  // this lane's column: 64 qb + lane
    if constexpr (FMT == 1) {
#pragma unroll
      for (int g = 0; g < SR / 8; ++g) {
        const v4s_t lo = lds_tr16(la, coff + 8 * g * RLD), hi = lds_tr16(la, coff + (8 * g + 4) * RLD);
        const short x[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        float sg = 0.0f;
#pragma unroll
        for (int d = 0; d < 4; ++d)
          sg += __uint_as_float(static_cast<uint32_t>(static_cast<uint16_t>(x[2 * d])) << 16) +
                __uint_as_float(static_cast<uint32_t>(static_cast<uint16_t>(x[2 * d + 1])) << 16);
        cs += static_cast<double>(sg);
      }
    } else {
#pragma unroll
      for (int hgrp = 0; hgrp < SR / 64; ++hgrp) {
        float sg = 0.0f;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          const v2i_t x = lds_tr8(la, coff + (64 * hgrp + 8 * g) * RLD);
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(x[d], false);
            const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(x[d], true);
            sg += (lo[0] + lo[1]) + (hi[0] + hi[1]);
          }
        }
        cs += static_cast<double>(sg);
      }
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[m][mb][v] += static_cast<double>(s32[m][mb][v]);
        s32[m][mb] = v4f_t{0.f, 0.f, 0.f, 0.f};
      }
  };

  // slab s is read from LDS buffer s & 1 while slab s + 1 waits in
  // registers; after the products it is staged into the other buffer (last
  // read one slab earlier, before the barrier) and slab s + 2 is fetched
  if (nslabs > 0) {
    fetch(r_beg, pre);
    store(0, pre);
    if (nslabs > 1) fetch(r_beg + SR, pre);
  }
  __syncthreads();
  for (int s = 0; s < nslabs; ++s) {
    const int cur = s & 1;
    if (colsum_wave) {
      if (colsum_part) colsum(cur);
    } else {
      mma(cur);
    }
    if (s + 1 < nslabs) {
      store(cur ^ 1, pre);
      if (s + 2 < nslabs) fetch(r_beg + static_cast<int64_t>(s + 2) * SR, pre);
    }
    if (!colsum_wave && ((s + 1) % FLUSH_SLABS == 0 || s + 1 == nslabs)) flush();
    __syncthreads();
  }

  double* out = part + (static_cast<int64_t>(chunk) * npairs + pair) * kNT * kNT;
  if (!colsum_wave) {
    // accumulate: add to the partial of an earlier launch over other rows (the
    // row groups of a sparse X_U, staged one after another)
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double* o = out + (64 * qa + 16 * m + 4 * kq + v) * kNT + 32 * qb + 16 * mb + i16;
          *o = accumulate ? *o + acc[m][mb][v] : acc[m][mb][v];
        }
  } else if (colsum_part) {
    const int j = ti * kNT + 64 * qb + lane;
    if (j < c) colsum_part[static_cast<int64_t>(chunk) * c + j] = cs;
  }
}

// G (c x c, both triangles) from the 128 x 128 tile partials of the narrow
// kernel, summed in chunk order; on a diagonal tile only the entries on and
// above its diagonal are read (the block below it is not formed).
__global__ void __launch_bounds__(256)
k_gram_reduce_n(const double* __restrict__ part, const double* __restrict__ colsum_part, int nchunks, int c,
                int ntiles, const float* __restrict__ scale, double* __restrict__ G, double* __restrict__ colsum) {
  const int npairs = ntiles * (ntiles + 1) / 2;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx < static_cast<int64_t>(npairs) * kNT * kNT) {
    const int pr = static_cast<int>(idx / (kNT * kNT)), e = static_cast<int>(idx % (kNT * kNT));
    int pi = pr, ti = 0;
    while (pi >= ntiles - ti) {
      pi -= ntiles - ti;
      ++ti;
    }
    const int tj = ti + pi;
    const int a = e / kNT, bcol = e % kNT;
    const int i = ti * kNT + a, j = tj * kNT + bcol;
    if (i < c && j < c && !(ti == tj && a > bcol)) {
      const double* src = part + idx;
      const int64_t stride = static_cast<int64_t>(npairs) * kNT * kNT;
      double s = 0.0;
      for (int ch0 = 0; ch0 < nchunks; ch0 += kGramBatch) {
        double v[kGramBatch];
#pragma unroll
        for (int u = 0; u < kGramBatch; ++u) v[u] = ch0 + u < nchunks ? src[(ch0 + u) * stride] : 0.0;
#pragma unroll
        for (int u = 0; u < kGramBatch; ++u) s += v[u];
      }
      // column scales of an FP8 X: C_ij = s_i s_j (sum of the raw products);
      // s_i s_j is exact in FP64
      if (scale) s *= static_cast<double>(scale[i]) * static_cast<double>(scale[j]);
      G[static_cast<int64_t>(i) * c + j] = s;
      G[static_cast<int64_t>(j) * c + i] = s;
    }
  }
  if (colsum && idx < c) {
    double s = 0.0;
    for (int ch0 = 0; ch0 < nchunks; ch0 += kGramBatch) {
      double v[kGramBatch];
#pragma unroll
      for (int u = 0; u < kGramBatch; ++u)
        v[u] = ch0 + u < nchunks ? colsum_part[static_cast<int64_t>(ch0 + u) * c + idx] : 0.0;
#pragma unroll
      for (int u = 0; u < kGramBatch; ++u) s += v[u];
    }
    colsum[idx] = scale ? s * static_cast<double>(scale[idx]) : s;
  }
}

// xdt: 0 FP32, 1 bfloat16, 2 FP8 E4M3 with column scales `scale`
static void gram(const void* X, int xdt, const float* scale, int64_t n, int c, int64_t ldx, int nchunks, double* part,
                 double* colsum_part, double* G, double* colsum, hipStream_t s) {
  const int rows_per_chunk = static_cast<int>((n + nchunks - 1) / nchunks);
  if (xdt == 1 || xdt == 2) {
    const int ntiles = (c + kNT - 1) / kNT;
    const int npairs = ntiles * (ntiles + 1) / 2;
    const int es = xdt == 1 ? 2 : 1;
    const int vec = (reinterpret_cast<uintptr_t>(X) % 16 == 0 && (ldx * es) % 16 == 0) ? 1 : 0;
    const int per_xcd = (nchunks + 7) / 8;
    if (xdt == 1)
      hipLaunchKernelGGL(k_gram_narrow<1>, dim3(8 * per_xcd * npairs), dim3(512), 0, s,
                         static_cast<const uint8_t*>(X), n, c, ldx, ntiles, rows_per_chunk, nchunks, vec, part,
                         colsum_part, 0);
    else
      hipLaunchKernelGGL(k_gram_narrow<2>, dim3(8 * per_xcd * npairs), dim3(512), 0, s,
                         static_cast<const uint8_t*>(X), n, c, ldx, ntiles, rows_per_chunk, nchunks, vec, part,
                         colsum_part, 0);
    TPO_LAUNCH_CHECK();
    const int64_t outs = std::max<int64_t>(static_cast<int64_t>(npairs) * kNT * kNT, c);
    hipLaunchKernelGGL(k_gram_reduce_n, dim3(ceil_div(outs, 256)), dim3(256), 0, s, part, colsum_part, nchunks, c,
                       ntiles, xdt == 2 ? scale : nullptr, G, colsum);
    TPO_LAUNCH_CHECK();
    return;
  }
  const int ntiles = (c + kGT - 1) / kGT;
  const int npairs = ntiles * (ntiles + 1) / 2;
  hipLaunchKernelGGL(k_gram_part, dim3(npairs, nchunks), dim3(256), 0, s, static_cast<const float*>(X), n, c, ldx,
                     ntiles, rows_per_chunk, part, colsum_part);
  TPO_LAUNCH_CHECK();
  const int64_t outs = std::max<int64_t>(static_cast<int64_t>(npairs) * kGT * kGT, c);
  hipLaunchKernelGGL(k_gram_reduce, dim3(ceil_div(outs, 256)), dim3(256), 0, s, part, colsum_part, nchunks, c,
                     ntiles, nullptr, G, colsum);
  TPO_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Multi-workgroup FP64 GEMM C = A B (row-major), 16x16 tile per workgroup.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_gemm_f64(int m, int n, int k, const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
           double* __restrict__ C, int ldc) {
  __shared__ double As[16][17];
  __shared__ double Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < k; k0 += 16) {
    As[ty][tx] = (row < m && k0 + tx < k) ? A[static_cast<int64_t>(row) * lda + k0 + tx] : 0.0;
    Bs[ty][tx] = (k0 + ty < k && col < n) ? B[static_cast<int64_t>(k0 + ty) * ldb + col] : 0.0;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 16; ++t) acc = fma(As[ty][t], Bs[t][tx], acc);
    __syncthreads();
  }
  if (row < m && col < n) C[static_cast<int64_t>(row) * ldc + col] = acc;
}

static void gemm_f64(int m, int n, int k, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_gemm_f64, dim3(ceil_div(n, 16), ceil_div(m, 16)), dim3(256), 0, s, m, n, k, A, lda, B, ldb,
                     C, ldc);
  TPO_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Single-workgroup kernels
// ---------------------------------------------------------------------------
constexpr int kSmallThreads = 1024;

// In-place Cholesky QR of A (m x n); G is n x n global scratch.
__global__ void __launch_bounds__(kSmallThreads)
k_cholqr(double* __restrict__ A, int m, int n, int lda, double* __restrict__ G, int32_t* __restrict__ err_bits) {
  __shared__ int flag;
  if (!blk_cholqr(A, m, n, lda, G, n, &flag)) {
    if (threadIdx.x == 0) atomicOr(err_bits, 16);
  }
}

// Q of Algorithm 1 from G by Cholesky QR done twice (the unique QR
// factor with positive diagonal of R, re-orthogonalised), plus Q^T in FP32.
__global__ void __launch_bounds__(kSmallThreads)
k_q_from_g(const double* __restrict__ Gm, int d, double* __restrict__ Q, double* __restrict__ scratch,
           float* __restrict__ Qt32, int32_t* __restrict__ err_bits) {
  __shared__ int flag;
  blk_copy(d, d, Gm, d, Q, d);
  bool ok = blk_cholqr(Q, d, d, d, scratch, d, &flag);
  if (ok) ok = blk_cholqr(Q, d, d, d, scratch, d, &flag);
  if (!ok) {
    if (threadIdx.x == 0) atomicOr(err_bits, 16);
    return;
  }
  for (int idx = threadIdx.x; idx < d * d; idx += blockDim.x) {
    const int j = idx / d, l = idx % d;
    Qt32[idx] = static_cast<float>(Q[l * d + j]);  // Qt[j][l] = Q[l][j]
  }
}

// Column sign convention: flip column c of the left factor L = Y * Sm (given
// through its column sums colsum^T Sm[:, c] and norms) and of the right vector
// Rv[:, c] so that the sum of L's column is positive; a sum within
// 1e-9 * sqrt(nrows) * ||L[:, c]|| of zero defers to the sign of Rv's entry of
// largest magnitude (lowest index on ties).
__device__ void blk_sign_convention(int rows_s, int ncol, const double* colsum, double* Sm, int lds, double* Rv,
                                    int rows_r, int ldr, const double* norms, double nrows_sqrt, double* sh) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < rows_s; ++i) s += colsum[i] * Sm[i * lds + c];
    if (fabs(s) <= 1e-9 * nrows_sqrt * norms[c]) {
      double best = -1.0;
      s = 0.0;
      for (int i = 0; i < rows_r; ++i) {
        const double v = Rv[i * ldr + c];
        if (fabs(v) > best) {
          best = fabs(v);
          s = v;
        }
      }
    }
    sh[c] = s < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < rows_s * ncol; idx += blockDim.x) {
    const int i = idx / ncol, c = idx % ncol;
    Sm[i * lds + c] *= sh[c];
  }
  if (Rv != Sm) {
    for (int idx = threadIdx.x; idx < rows_r * ncol; idx += blockDim.x) {
      const int i = idx / ncol, c = idx % ncol;
      Rv[i * ldr + c] *= sh[c];
    }
  }
  __syncthreads();
}

// Rayleigh-Ritz step of the reduction: T = M^T (C M), eigenpairs of T, the top
// d kept: Psi_d = M V_d, sigma = sqrt(lambda); sign convention on X' = X Psi_d.
__global__ void __launch_bounds__(kSmallThreads)
k_reduce_rr(const double* __restrict__ M, const double* __restrict__ P, int du, int l, int d, int dp,
            const double* __restrict__ colsum_x, int64_t n, double* __restrict__ T, double* __restrict__ V,
            double* __restrict__ evals, double* __restrict__ psi, float* __restrict__ psi32) {
  __shared__ double red[kSmallThreads];
  __shared__ __align__(16) double sh[3 * 64 + 8 + 256];
  __shared__ int perm[256];
  __shared__ double ev[256];
  __shared__ double nrm[256];
  blk_gemm(l, l, du, M, l, true, P, l, false, T, l, 1.0, 0.0);
  for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
    const int i = idx / l, j = idx % l;
    if (i < j) {
      const double a = 0.5 * (T[i * l + j] + T[j * l + i]);
      T[i * l + j] = a;
      T[j * l + i] = a;
    }
  }
  __syncthreads();
  blk_jacobi<4>(T, l, V, l, l, sh, red, 40);
  blk_sort_desc(T, l, l, ev, perm);
  // psi = M V[:, perm[:d]]
  for (int idx = threadIdx.x; idx < du * d; idx += blockDim.x) {
    const int i = idx / d, c = idx % d;
    const int pc = perm[c];
    double acc = 0.0;
    for (int t = 0; t < l; ++t) acc = fma(M[i * l + t], V[t * l + pc], acc);
    psi[i * d + c] = acc;
  }
  for (int c = threadIdx.x; c < d; c += blockDim.x) {
    const double lam = ev[c] > 0.0 ? ev[c] : 0.0;
    evals[c] = sqrt(lam);
    nrm[c] = sqrt(lam);
  }
  __syncthreads();
  blk_sign_convention(du, d, colsum_x, psi, d, psi, du, d, nrm, sqrt(static_cast<double>(n)), sh);
  for (int idx = threadIdx.x; idx < du * dp; idx += blockDim.x) {
    const int i = idx / dp, c = idx % dp;
    psi32[idx] = c < d ? static_cast<float>(psi[i * d + c]) : 0.0f;
  }
}

// RandomizedSVD(R, k) on K = R^T R (2d x 2d):
//   M <- Omega;  q times: M <- orth(K M)
//   L = chol(M^T K M);  B^T = K M L^{-T};  B B^T = U diag(lambda) U^T
//   S = M L^{-T} U_k (Gamma = R S), sigma = sqrt(lambda_k), Psi = B^T U_k / sigma
// then the column sign convention, H = Psi Sigma (Eq. init-HY).
__global__ void __launch_bounds__(kSmallThreads)
k_embed_small(const double* __restrict__ K, const double* __restrict__ Omega, int twod, int kp, int k, int q,
              const double* __restrict__ colsum_r, int64_t n, double* __restrict__ M, double* __restrict__ P,
              double* __restrict__ G, double* __restrict__ BBt, double* __restrict__ V, double* __restrict__ S,
              float* __restrict__ S32, double* __restrict__ sigma, double* __restrict__ psi,
              double* __restrict__ H, float* __restrict__ H32, int32_t* __restrict__ err_bits) {
  __shared__ double red[kSmallThreads];
  __shared__ __align__(16) double sh[3 * 64 + 8 + 256];
  __shared__ int perm[128];
  __shared__ double ev[128];
  __shared__ double nrm[128];
  __shared__ int flag;
  blk_copy(twod, kp, Omega, kp, M, kp);
  for (int it = 0; it < q; ++it) {
    blk_gemm(twod, kp, twod, K, twod, false, M, kp, false, P, kp, 1.0, 0.0);
    if (!blk_cholqr(P, twod, kp, kp, G, kp, &flag)) {
      if (threadIdx.x == 0) atomicOr(err_bits, 16);
      return;
    }
    blk_copy(twod, kp, P, kp, M, kp);
  }
  blk_gemm(twod, kp, twod, K, twod, false, M, kp, false, P, kp, 1.0, 0.0);       // P = K M
  blk_gemm(kp, kp, twod, M, kp, true, P, kp, false, G, kp, 1.0, 0.0);            // G = M^T K M
  if (!blk_chol(G, kp, kp, &flag)) {
    if (threadIdx.x == 0) atomicOr(err_bits, 16);
    return;
  }
  blk_trsm_right_lt(P, twod, kp, kp, G, kp);                                      // P = B^T
  blk_trsm_right_lt(M, twod, kp, kp, G, kp);                                      // M = M L^-T
  blk_gemm(kp, kp, twod, P, kp, true, P, kp, false, BBt, kp, 1.0, 0.0);          // B B^T
  for (int idx = threadIdx.x; idx < kp * kp; idx += blockDim.x) {
    const int i = idx / kp, j = idx % kp;
    if (i < j) {
      const double a = 0.5 * (BBt[i * kp + j] + BBt[j * kp + i]);
      BBt[i * kp + j] = a;
      BBt[j * kp + i] = a;
    }
  }
  __syncthreads();
  blk_jacobi<4>(BBt, kp, V, kp, kp, sh, red, 40);
  blk_sort_desc(BBt, kp, kp, ev, perm);
  for (int c = threadIdx.x; c < k; c += blockDim.x) sigma[c] = sqrt(ev[c] > 0.0 ? ev[c] : 0.0);
  __syncthreads();
  // S = (M L^-T) U_k ; Psi = B^T U_k / sigma
  for (int idx = threadIdx.x; idx < twod * k; idx += blockDim.x) {
    const int i = idx / k, c = idx % k;
    const int pc = perm[c];
    double a = 0.0, b = 0.0;
    for (int t = 0; t < kp; ++t) {
      a = fma(M[i * kp + t], V[t * kp + pc], a);
      b = fma(P[i * kp + t], V[t * kp + pc], b);
    }
    S[i * k + c] = a;
    psi[i * k + c] = sigma[c] > 0.0 ? b / sigma[c] : 0.0;
  }
  __syncthreads();
  // ||Gamma[:, c]|| = sqrt(S_c^T K S_c)
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < twod; ++i) {
      double ki = 0.0;
      for (int j = 0; j < twod; ++j) ki = fma(K[i * twod + j], S[j * k + c], ki);
      acc = fma(S[i * k + c], ki, acc);
    }
    nrm[c] = sqrt(acc > 0.0 ? acc : 0.0);
  }
  __syncthreads();
  blk_sign_convention(twod, k, colsum_r, S, k, psi, twod, k, nrm, sqrt(static_cast<double>(n)), sh);
  for (int idx = threadIdx.x; idx < twod * k; idx += blockDim.x) {
    const int c = idx % k;
    S32[idx] = static_cast<float>(S[idx]);
    H[idx] = psi[idx] * sigma[c];
    H32[idx] = static_cast<float>(H[idx]);
  }
}

// ---------------------------------------------------------------------------
// Attribute projection X' = X Psi_d (FP32), rows padded to dp columns, or a
// padded copy of X when there is no reduction.  Also flags non-finite input.
// ---------------------------------------------------------------------------
// X' = X Psi_d on FP32 MFMA 16x16x4 (lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; its v-th result is D[4 (l / 16) + v][l % 16]).  A
// workgroup takes 64 rows; wave w owns rows 16 w.. and all CT column tiles.
// 32-column slabs of X and the matching rows of Psi_d are staged in LDS.
constexpr int kPjRows = 64;
constexpr int kPjK = 32;
constexpr int kPjXLd = kPjK + 1;

// An attribute as FP32: FP32 X as is, bfloat16 X (raw 16 bits) widened
// exactly, FP8 X (raw byte) decoded exactly (its column scale is applied by
// the caller).
__device__ __forceinline__ float x_at(const float* X, int64_t i) { return X[i]; }
__device__ __forceinline__ float x_at(const uint16_t* X, int64_t i) {
  return __uint_as_float(static_cast<uint32_t>(X[i]) << 16);
}
__device__ __forceinline__ float x_at(const uint8_t* X, int64_t i) { return fp8_to_f32(X[i]); }

template <int CT, typename XT>
__global__ void __launch_bounds__(256)
k_project_mfma(const XT* __restrict__ X, int64_t n, int du, int64_t ldx, const float* __restrict__ scale,
               const float* __restrict__ psi32, int dp, float* __restrict__ out, int32_t* __restrict__ err_bits) {
  constexpr int PLD = 16 * CT + 4;
  __shared__ float xs[kPjRows * kPjXLd];
  __shared__ float ps[kPjK * PLD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kPjRows;
  v4f_t acc[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = v4f_t{0.f, 0.f, 0.f, 0.f};
  bool bad = false;
  for (int k0 = 0; k0 < du; k0 += kPjK) {
#pragma unroll
    for (int u = 0; u < kPjRows * kPjK / 256; ++u) {
      const int e = tid + 256 * u;
      const int rr = e / kPjK, kk = e % kPjK;
      const int64_t row = row0 + rr;
      float v = (row < n && k0 + kk < du) ? x_at(X, row * ldx + k0 + kk) : 0.0f;
      if (scale && k0 + kk < du) v *= scale[k0 + kk];
      if (!isfinite(v)) {
        bad = true;
        v = 0.0f;
      }
      xs[rr * kPjXLd + kk] = v;
    }
    for (int e = tid; e < kPjK * 16 * CT; e += 256) {
      const int kk = e / (16 * CT), cc = e % (16 * CT);
      ps[kk * PLD + cc] = (k0 + kk < du && cc < dp) ? psi32[static_cast<int64_t>(k0 + kk) * dp + cc] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < kPjK / 4; ++st) {
      const float av = xs[(16 * w + i16) * kPjXLd + 4 * st + kq];
#pragma unroll
      for (int t = 0; t < CT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, ps[(4 * st + kq) * PLD + 16 * t + i16], acc[t], 0, 0, 0);
    }
    __syncthreads();
  }
  if (bad) atomicOr(err_bits, 4);
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const int col = 16 * t + i16;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = row0 + 16 * w + 4 * kq + v;
      if (row < n && col < dp) out[row * dp + col] = acc[t][v];
    }
  }
}

template <typename XT>
__global__ void k_pad_copy(const XT* __restrict__ X, int64_t n, int du, int64_t ldx, const float* __restrict__ scale,
                           int dp, float* __restrict__ out, int32_t* __restrict__ err_bits) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n * dp) return;
  const int64_t r = i / dp;
  const int c = static_cast<int>(i % dp);
  float v = c < du ? x_at(X, r * ldx + c) : 0.0f;
  if (scale && c < du) v *= scale[c];
  if (!isfinite(v)) {
    atomicOr(err_bits, 4);
    v = 0.0f;
  }
  out[i] = v;
}

// Narrow attributes (bfloat16, or FP8 E4M3, both exact in bfloat16): X' =
// X diag(s) Psi_d on BF16 MFMA 16x16x32.  Psi~ = diag(s) Psi_d is split once
// into three bfloat16 parts hi + mid + lo (each the round-to-nearest of what
// the previous parts leave, in FP64: 24 significant bits in all), stored
// transposed (part, column n, k) so that the B operand's eight consecutive k
// are one 16-byte read.  Products of two bfloat16 values are exact in FP32;
// hi goes to one set of FP32 accumulators, mid and lo to another, added at
// the end.  The A operand (eight consecutive columns of one row) is read
// straight from row-major X staged in LDS, no transpose.
__device__ __forceinline__ uint16_t f32_to_bf16_rn(float f) {
  const uint32_t u = __float_as_uint(f);
  return static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__global__ void k_psi_split(const double* __restrict__ psi, const float* __restrict__ scale, int du, int d, int dp,
                            int dup, uint16_t* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(dp) * dup) return;
  const int n = static_cast<int>(i / dup), k = static_cast<int>(i % dup);
  double v = (n < d && k < du) ? psi[static_cast<int64_t>(k) * d + n] : 0.0;
  if (scale && k < du) v *= static_cast<double>(scale[k]);
  const uint16_t hi = f32_to_bf16_rn(static_cast<float>(v));
  const double r1 = v - static_cast<double>(__uint_as_float(static_cast<uint32_t>(hi) << 16));
  const uint16_t mid = f32_to_bf16_rn(static_cast<float>(r1));
  const double r2 = r1 - static_cast<double>(__uint_as_float(static_cast<uint32_t>(mid) << 16));
  const uint16_t lo = f32_to_bf16_rn(static_cast<float>(r2));
  const int64_t plane = static_cast<int64_t>(dp) * dup;
  out[i] = hi;
  out[plane + i] = mid;
  out[2 * plane + i] = lo;
}

constexpr int kPsK = 32;         // columns of X per slab
constexpr int kPsLd = kPsK + 8;  // LDS row stride (bfloat16 elements; 80 bytes)

// A narrow attribute as bfloat16 (raw bits).
__device__ __forceinline__ uint16_t narrow_to_bf16(uint16_t v) { return v; }
__device__ __forceinline__ uint16_t narrow_to_bf16(uint8_t v) {
  return static_cast<uint16_t>(__float_as_uint(fp8_to_f32(v)) >> 16);  // exact: E4M3 is a subset of bfloat16
}
__device__ __forceinline__ bool bf16_finite(uint16_t b) { return (b & 0x7f80u) != 0x7f80u; }

// Rows per workgroup of the split projection: each wave takes RT row tiles
// against the same staged slab of the three parts of Psi~ (four for up to 32
// output columns, two for 64, one for 128, as the accumulators allow).
__host__ __device__ constexpr int ps_row_tiles(int ct) { return ct <= 2 ? 4 : (ct == 4 ? 2 : 1); }

template <int CT, typename XT>
__global__ void __launch_bounds__(256)
k_project_split(const XT* __restrict__ X, int64_t n, int du, int64_t ldx, const uint16_t* __restrict__ psit, int dp,
                int dup, float* __restrict__ out, int32_t* __restrict__ err_bits, int vec) {
  constexpr int NC = 16 * CT;
  constexpr int RT = ps_row_tiles(CT), ROWS = 64 * RT;
  __shared__ __align__(16) uint16_t xs[ROWS * kPsLd];
  __shared__ __align__(16) uint16_t ps[3 * NC * kPsLd];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * ROWS;
  const int64_t plane = static_cast<int64_t>(dp) * dup;
  v4f_t acc_hi[RT][CT], acc_lo[RT][CT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int t = 0; t < CT; ++t) acc_hi[r][t] = acc_lo[r][t] = v4f_t{0.f, 0.f, 0.f, 0.f};
  bool bad = false;
  for (int k0 = 0; k0 < du; k0 += kPsK) {
    constexpr int PPR = kPsK / 8, RPP = 256 / PPR;  // 16-byte pieces per row, rows per pass
#pragma unroll
    for (int u = 0; u < ROWS / RPP; ++u) {  // X: thread tid stages row tid / PPR + RPP u, piece tid % PPR
      const int rr = tid / PPR + RPP * u, c0 = 8 * (tid % PPR);
      const int64_t row = row0 + rr;
      uint16_t v[8];
      if (vec) {  // one 16-byte (bfloat16) or 8-byte (FP8) load; d_u is a multiple of 8
        const bool in = row < n && k0 + c0 < du;
        if constexpr (sizeof(XT) == 2) {
          v4u_t raw = {0u, 0u, 0u, 0u};
          if (in) raw = *reinterpret_cast<const v4u_t*>(X + row * ldx + k0 + c0);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            v[2 * j] = static_cast<uint16_t>(raw[j] & 0xffffu);
            v[2 * j + 1] = static_cast<uint16_t>(raw[j] >> 16);
          }
        } else {
          uint2 raw = make_uint2(0u, 0u);
          if (in) raw = *reinterpret_cast<const uint2*>(X + row * ldx + k0 + c0);
          const uint32_t wd[2] = {raw.x, raw.y};
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            // exact decodes, two bytes at a time (E4M3 is a subset of bfloat16)
            const auto lo2 = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(wd[h]), false);
            const auto hi2 = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(wd[h]), true);
            v[4 * h + 0] = static_cast<uint16_t>(__float_as_uint(lo2[0]) >> 16);
            v[4 * h + 1] = static_cast<uint16_t>(__float_as_uint(lo2[1]) >> 16);
            v[4 * h + 2] = static_cast<uint16_t>(__float_as_uint(hi2[0]) >> 16);
            v[4 * h + 3] = static_cast<uint16_t>(__float_as_uint(hi2[1]) >> 16);
          }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (!bf16_finite(v[j])) {
            bad = true;
            v[j] = 0;
          }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int c = k0 + c0 + j;
          uint16_t b = (row < n && c < du) ? narrow_to_bf16(X[row * ldx + c]) : uint16_t{0};
          if (!bf16_finite(b)) {
            bad = true;
            b = 0;
          }
          v[j] = b;
        }
      }
      v4u_t wv;
#pragma unroll
      for (int j = 0; j < 4; ++j) wv[j] = static_cast<uint32_t>(v[2 * j]) | (static_cast<uint32_t>(v[2 * j + 1]) << 16);
      *reinterpret_cast<v4u_t*>(xs + rr * kPsLd + c0) = wv;
    }
    // the three parts of Psi~ for columns k0 .. k0 + 31 (dup is a multiple of
    // 8, zero beyond d_u), 16-byte pieces
    for (int e = tid; e < 3 * NC * (kPsK / 8); e += 256) {
      const int part = e / (NC * (kPsK / 8)), rem = e - part * (NC * (kPsK / 8));
      const int nn = rem / (kPsK / 8), q = rem - nn * (kPsK / 8);
      const int kk = k0 + 8 * q;
      v4u_t wv = {0u, 0u, 0u, 0u};
      if (nn < dp && kk < dup)
        wv = *reinterpret_cast<const v4u_t*>(psit + part * plane + static_cast<int64_t>(nn) * dup + kk);
      *reinterpret_cast<v4u_t*>(ps + (part * NC + nn) * kPsLd + 8 * q) = wv;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kPsK / 32; ++ks) {
      v8bf_t a[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r)
        a[r] = __builtin_bit_cast(
            v8bf_t, *reinterpret_cast<const v4u_t*>(xs + (16 * (w + 4 * r) + i16) * kPsLd + 32 * ks + 8 * kq));
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        const int nn = 16 * t + i16, kc = 32 * ks + 8 * kq;
        const v8bf_t bh = __builtin_bit_cast(v8bf_t, *reinterpret_cast<const v4u_t*>(ps + nn * kPsLd + kc));
        const v8bf_t bm = __builtin_bit_cast(v8bf_t, *reinterpret_cast<const v4u_t*>(ps + (NC + nn) * kPsLd + kc));
        const v8bf_t bl =
            __builtin_bit_cast(v8bf_t, *reinterpret_cast<const v4u_t*>(ps + (2 * NC + nn) * kPsLd + kc));
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          acc_hi[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], bh, acc_hi[r][t], 0, 0, 0);
          acc_lo[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], bl, acc_lo[r][t], 0, 0, 0);
          acc_lo[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], bm, acc_lo[r][t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(err_bits, 4);
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int col = 16 * t + i16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + 16 * (w + 4 * r) + 4 * kq + v;
        if (row < n && col < dp) out[row * dp + col] = acc_hi[r][t][v] + acc_lo[r][t][v];
      }
    }
}

template <typename XT>
static void project_split(const Plan& p, void* ws, const XT* x, int64_t ldx, const float* sc, float* xp, int32_t* err,
                          hipStream_t s) {
  if (p.dp > 128) throw std::runtime_error("narrow-attribute projection: padded width above 128");
  const int dup = (p.du + 7) / 8 * 8;
  uint16_t* pst = bufp<uint16_t>(p, ws, B_PSI_SPLIT);
  const int64_t cnt = static_cast<int64_t>(p.dp) * dup;
  hipLaunchKernelGGL(k_psi_split, dim3(ceil_div(cnt, 256)), dim3(256), 0, s, bufp<double>(p, ws, B_PSI_D), sc, p.du,
                     p.d, p.dp, dup, pst);
  TPO_LAUNCH_CHECK();
  const int64_t n = p.n;
  const int ct = (p.dp + 15) / 16;
  const dim3 grid(ceil_div(p.n, 64 * ps_row_tiles(ct == 1 || ct == 2 || ct == 4 ? ct : 8)));
  // word loads: eight elements (16 or 8 bytes) aligned to their size
  const int vec = (reinterpret_cast<uintptr_t>(x) % (8 * sizeof(XT)) == 0 && ldx % 8 == 0 && p.du % 8 == 0) ? 1 : 0;
  switch ((p.dp + 15) / 16) {
    case 1: hipLaunchKernelGGL((k_project_split<1, XT>), grid, dim3(256), 0, s, x, n, p.du, ldx, pst, p.dp, dup, xp, err, vec); break;
    case 2: hipLaunchKernelGGL((k_project_split<2, XT>), grid, dim3(256), 0, s, x, n, p.du, ldx, pst, p.dp, dup, xp, err, vec); break;
    case 4: hipLaunchKernelGGL((k_project_split<4, XT>), grid, dim3(256), 0, s, x, n, p.du, ldx, pst, p.dp, dup, xp, err, vec); break;
    default: hipLaunchKernelGGL((k_project_split<8, XT>), grid, dim3(256), 0, s, x, n, p.du, ldx, pst, p.dp, dup, xp, err, vec); break;
  }
  TPO_LAUNCH_CHECK();
}

template <typename XT>
static void project(const Plan& p, const XT* x, int64_t ldx, const float* sc, const float* psi32, float* xp,
                    int32_t* err, hipStream_t s) {
  const dim3 grid(ceil_div(p.n, kPjRows));
  const int64_t n = p.n;
  switch ((p.dp + 15) / 16) {
    case 1: hipLaunchKernelGGL((k_project_mfma<1, XT>), grid, dim3(256), 0, s, x, n, p.du, ldx, sc, psi32, p.dp, xp, err); break;
    case 2: hipLaunchKernelGGL((k_project_mfma<2, XT>), grid, dim3(256), 0, s, x, n, p.du, ldx, sc, psi32, p.dp, xp, err); break;
    case 4: hipLaunchKernelGGL((k_project_mfma<4, XT>), grid, dim3(256), 0, s, x, n, p.du, ldx, sc, psi32, p.dp, xp, err); break;
    case 8: hipLaunchKernelGGL((k_project_mfma<8, XT>), grid, dim3(256), 0, s, x, n, p.du, ldx, sc, psi32, p.dp, xp, err); break;
    default: hipLaunchKernelGGL((k_project_mfma<16, XT>), grid, dim3(256), 0, s, x, n, p.du, ldx, sc, psi32, p.dp, xp, err); break;
  }
  TPO_LAUNCH_CHECK();
}

// The FP8 Gram of a sparse X_U: row groups of p.xstage_rows rows staged as
// E4M3 codes one after another, each group's tile-pair partials added to the
// previous groups' (group order fixed), then the chunk partials summed with
// the column scales.
static void gram_xcsr(const Plan& p, void* ws, const tpo_inputs* in, hipStream_t s) {
  const int c = p.du;
  const int ld = xcsr_stage_ld(c);
  const int ntiles = (c + kNT - 1) / kNT;
  const int npairs = ntiles * (ntiles + 1) / 2;
  const int nchunks = p.gram_chunks_x;
  const int per_xcd = (nchunks + 7) / 8;
  double* part = bufp<double>(p, ws, B_GRAM_PART);
  const uint8_t* stage = bufp<uint8_t>(p, ws, B_XS_STAGE);
  for (int64_t r0 = 0; r0 < p.n; r0 += p.xstage_rows) {
    const int rows = static_cast<int>(std::min<int64_t>(p.xstage_rows, p.n - r0));
    xcsr_stage_fp8(p, ws, r0, rows, ld, s);
    const int rows_per_chunk = (rows + nchunks - 1) / nchunks;
    hipLaunchKernelGGL(k_gram_narrow<2>, dim3(8 * per_xcd * npairs), dim3(512), 0, s, stage,
                       static_cast<int64_t>(rows), c, static_cast<int64_t>(ld), ntiles, rows_per_chunk, nchunks, 1,
                       part, nullptr, r0 > 0 ? 1 : 0);
    TPO_LAUNCH_CHECK();
  }
  const int64_t outs = static_cast<int64_t>(npairs) * kNT * kNT;
  hipLaunchKernelGGL(k_gram_reduce_n, dim3(ceil_div(outs, 256)), dim3(256), 0, s, part, nullptr, nchunks, c, ntiles,
                     bufp<float>(p, ws, B_XS_SCALE), bufp<double>(p, ws, B_C), nullptr);
  TPO_LAUNCH_CHECK();
}

// Reduction of a sparse X_U (TPO_X_CSR): scales, transpose and column sums,
// the FP8 Gram, subspace iteration on it, x_refine refinement steps with the
// exact FP32 values (P = X^T (X M): power steps, the last one the
// Rayleigh-Ritz product), Rayleigh-Ritz, and X' = X Psi_d from the exact
// values.
static void reduce_xcsr(const Plan& p, void* ws, const tpo_inputs* in, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  const float* val = static_cast<const float*>(in->x_u);
  float* xp = bufp<float>(p, ws, B_XPRIME);
  double* colsum = bufp<double>(p, ws, B_COLSUM_X);
  xcsr_transpose(p, ws, in->x_rowptr, in->x_col, val, s);
  xcsc_make_chunks(p, ws, s);
  xcsr_scales(p, ws, s);
  gram_xcsr(p, ws, in, s);
  double* ma = bufp<double>(p, ws, B_MR_A);
  double* mb = bufp<double>(p, ws, B_MR_B);
  const double* C = bufp<double>(p, ws, B_C);
  double* m;   // the basis after q + 1 products with C
  double* pm;  // C m, replaced by X^T (X m) in the refinement step
  if (p.lr <= kLdsMaxN) {
    m = bufp<double>(p, ws, B_SI_M);
    pm = bufp<double>(p, ws, B_SI_P);
    subspace_iterate(C, p.du, bufp<double>(p, ws, B_OMR), p.lr, p.par.q + 1, ma, mb, bufp<double>(p, ws, B_SI_GRAM),
                     bufp<double>(p, ws, B_SI_PART), bufp<unsigned>(p, ws, B_SI_BAR), m, pm, &st->err_bits, s);
  } else {
    double* gs = bufp<double>(p, ws, B_SMALL_A);
    TPO_HIP_CHECK(hipMemcpyAsync(ma, bufp<double>(p, ws, B_OMR), sizeof(double) * p.du * p.lr,
                                 hipMemcpyDeviceToDevice, s));
    for (int it = 0; it <= p.par.q; ++it) {
      gemm_f64(p.du, p.lr, p.du, C, p.du, ma, p.lr, mb, p.lr, s);
      hipLaunchKernelGGL(k_cholqr, dim3(1), dim3(kSmallThreads), 0, s, mb, p.du, p.lr, p.lr, gs, &st->err_bits);
      TPO_LAUNCH_CHECK();
      std::swap(ma, mb);
    }
    gemm_f64(p.du, p.lr, p.du, C, p.du, ma, p.lr, mb, p.lr, s);
    m = ma;
    pm = mb;
  }
  // refinement: Y = X M (FP32 from FP64 sums), P = X^T Y with the exact
  // values (and the column sums of X); all but the last step re-orthonormalise
  // P into M as further power steps
  float* y = bufp<float>(p, ws, B_XT_Y);
  const int steps = p.par.x_refine;
  for (int step = 0; step < std::max(steps, 1); ++step) {
    xcsr_rowgather(p, in->x_rowptr, in->x_col, val, m, p.lr, p.lr, y, p.lr, p.lr, s);
    xcsc_colgather(p, ws, y, p.lr, p.lr, steps > 0 ? pm : nullptr, p.lr, colsum, s);
    if (step + 1 < steps) {
      TPO_HIP_CHECK(hipMemcpyAsync(m, pm, sizeof(double) * p.du * p.lr, hipMemcpyDeviceToDevice, s));
      if (p.lr <= kLdsMaxN) {
        cholqr_lds(m, p.du, p.lr, p.lr, &st->err_bits, s);
      } else {
        hipLaunchKernelGGL(k_cholqr, dim3(1), dim3(kSmallThreads), 0, s, m, p.du, p.lr, p.lr,
                           bufp<double>(p, ws, B_SMALL_A), &st->err_bits);
        TPO_LAUNCH_CHECK();
      }
    }
  }
  if (p.lr <= kLdsMaxN) {
    rr_reduce_lds(m, pm, p.du, p.lr, p.d, p.dp, colsum, static_cast<int64_t>(p.n), bufp<double>(p, ws, B_EVAL),
                  bufp<double>(p, ws, B_PSI_D), bufp<float>(p, ws, B_PSI_D32), jacobi_log(p, ws), s);
  } else {
    hipLaunchKernelGGL(k_reduce_rr, dim3(1), dim3(kSmallThreads), 0, s, m, pm, p.du, p.lr, p.d, p.dp, colsum,
                       static_cast<int64_t>(p.n), bufp<double>(p, ws, B_SMALL_B), bufp<double>(p, ws, B_SMALL_C),
                       bufp<double>(p, ws, B_EVAL), bufp<double>(p, ws, B_PSI_D), bufp<float>(p, ws, B_PSI_D32));
    TPO_LAUNCH_CHECK();
  }
  // X' = X Psi_d with the exact values, padded to dp columns
  xcsr_rowgather(p, in->x_rowptr, in->x_col, val, bufp<double>(p, ws, B_PSI_D), p.d, p.d, xp, p.dp, p.dp, s);
}

void launch_reduce(const Plan& p, void* ws, const tpo_inputs* in, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  float* xp = bufp<float>(p, ws, B_XPRIME);
  const void* x = in->x_u;
  const int64_t ldx = in->ld_x;
  const float* xscale = in->x_scale;
  if (p.xcsr) {
    if (p.reduce) {
      reduce_xcsr(p, ws, in, s);
    } else {
      // rows copied densely into X' (d = d_u <= 128)
      xcsr_dense(p, ws, in->x_rowptr, in->x_col, static_cast<const float*>(in->x_u), xp, s);
    }
    return;
  }
  const int xdt = p.xfp8 ? 2 : p.xbf16 ? 1 : 0;
  if (!p.reduce) {
    const dim3 g(ceil_div(static_cast<int64_t>(p.n) * p.dp, 256));
    if (xdt == 2)
      hipLaunchKernelGGL(k_pad_copy<uint8_t>, g, dim3(256), 0, s, static_cast<const uint8_t*>(x),
                         static_cast<int64_t>(p.n), p.du, ldx, xscale, p.dp, xp, &st->err_bits);
    else if (xdt == 1)
      hipLaunchKernelGGL(k_pad_copy<uint16_t>, g, dim3(256), 0, s, static_cast<const uint16_t*>(x),
                         static_cast<int64_t>(p.n), p.du, ldx, nullptr, p.dp, xp, &st->err_bits);
    else
      hipLaunchKernelGGL(k_pad_copy<float>, g, dim3(256), 0, s, static_cast<const float*>(x),
                         static_cast<int64_t>(p.n), p.du, ldx, nullptr, p.dp, xp, &st->err_bits);
    TPO_LAUNCH_CHECK();
    return;
  }
  double* C = bufp<double>(p, ws, B_C);
  double* colsum = bufp<double>(p, ws, B_COLSUM_X);
  gram(x, xdt, xscale, p.n, p.du, ldx, p.gram_chunks_x, bufp<double>(p, ws, B_GRAM_PART), bufp<double>(p, ws, B_COLSUM_PART), C,
       colsum, s);
  double* ma = bufp<double>(p, ws, B_MR_A);
  double* mb = bufp<double>(p, ws, B_MR_B);
  if (p.lr <= kLdsMaxN) {
    // q + 1 products with C, each followed by Cholesky QR, then P = C M
    double* m = bufp<double>(p, ws, B_SI_M);
    double* pm = bufp<double>(p, ws, B_SI_P);
    subspace_iterate(C, p.du, bufp<double>(p, ws, B_OMR), p.lr, p.par.q + 1, ma, mb, bufp<double>(p, ws, B_SI_GRAM),
                     bufp<double>(p, ws, B_SI_PART), bufp<unsigned>(p, ws, B_SI_BAR), m, pm, &st->err_bits, s);
    rr_reduce_lds(m, pm, p.du, p.lr, p.d, p.dp, colsum, static_cast<int64_t>(p.n), bufp<double>(p, ws, B_EVAL),
                  bufp<double>(p, ws, B_PSI_D), bufp<float>(p, ws, B_PSI_D32), jacobi_log(p, ws), s);
  } else {
    double* gs = bufp<double>(p, ws, B_SMALL_A);
    TPO_HIP_CHECK(hipMemcpyAsync(ma, bufp<double>(p, ws, B_OMR), sizeof(double) * p.du * p.lr,
                                 hipMemcpyDeviceToDevice, s));
    for (int it = 0; it <= p.par.q; ++it) {
      gemm_f64(p.du, p.lr, p.du, C, p.du, ma, p.lr, mb, p.lr, s);
      hipLaunchKernelGGL(k_cholqr, dim3(1), dim3(kSmallThreads), 0, s, mb, p.du, p.lr, p.lr, gs, &st->err_bits);
      TPO_LAUNCH_CHECK();
      std::swap(ma, mb);
    }
    gemm_f64(p.du, p.lr, p.du, C, p.du, ma, p.lr, mb, p.lr, s);  // P = C M
    hipLaunchKernelGGL(k_reduce_rr, dim3(1), dim3(kSmallThreads), 0, s, ma, mb, p.du, p.lr, p.d, p.dp, colsum,
                       static_cast<int64_t>(p.n), bufp<double>(p, ws, B_SMALL_B), bufp<double>(p, ws, B_SMALL_C),
                       bufp<double>(p, ws, B_EVAL), bufp<double>(p, ws, B_PSI_D), bufp<float>(p, ws, B_PSI_D32));
    TPO_LAUNCH_CHECK();
  }
  const float* psi32 = bufp<float>(p, ws, B_PSI_D32);
  if (xdt == 2)
    project_split(p, ws, static_cast<const uint8_t*>(x), ldx, xscale, xp, &st->err_bits, s);
  else if (xdt == 1)
    project_split(p, ws, static_cast<const uint16_t*>(x), ldx, nullptr, xp, &st->err_bits, s);
  else
    project(p, static_cast<const float*>(x), ldx, nullptr, psi32, xp, &st->err_bits, s);
}

// ---------------------------------------------------------------------------
// Random features (Eqs. Z, R-prime, Ri)
// ---------------------------------------------------------------------------
// Random features on FP32 MFMA, two passes over Z (Eqs. Z, R-prime, Ri):
//   pass 1: Zo = sqrt(d) Z_hat Q^T, R' = sqrt(e/d) [sin Zo || cos Zo], and
//           only the FP64 column sums r = sum_i R'_i per workgroup;
//   pass 2: the same R' again (same instructions, so the same values), then
//           R_i = R'_i / sqrt(R'_i . r) written out, with FP64 column sums of
//           R and max |R|.
// A workgroup walks 64-row slabs; wave w takes 16 rows.  The product is
// formed on the raw rows and scaled by 1 / ||Z_i|| afterwards.  MFMA layout:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its v-th result is
// D[4 (l / 16) + v][l % 16].  DT = ceil(d / 16) column tiles.
template <int PASS, int DT>
__global__ void __launch_bounds__(256)
k_feat_mfma(const float* __restrict__ Z, int64_t n, int d, int dp, const float* __restrict__ Qt32,
            int rows_per_block, const double* __restrict__ rsum, float* __restrict__ R, double* __restrict__ part,
            DevStatus* __restrict__ st) {
  constexpr int DPAD = 16 * DT, KS = 4 * DT;
  extern __shared__ float qts[];  // DPAD x DPAD, Q^T[j][l], zero padded
  __shared__ double cs[4][2 * DPAD];
  __shared__ double rsl[2 * DPAD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  for (int e = tid; e < DPAD * DPAD; e += 256) {
    const int j = e / DPAD, l = e - (e / DPAD) * DPAD;
    qts[e] = (j < d && l < d) ? Qt32[j * d + l] : 0.0f;
  }
  if (PASS == 2)
    for (int c = tid; c < DPAD; c += 256) {
      rsl[c] = c < d ? rsum[c] : 0.0;
      rsl[DPAD + c] = c < d ? rsum[d + c] : 0.0;
    }
  __syncthreads();
  const float sqrtd = sqrtf(static_cast<float>(d));
  const float amp = static_cast<float>(sqrt(2.718281828459045235 / static_cast<double>(d)));
  const int twod = 2 * d;
  double csn[DT], ccs[DT];
#pragma unroll
  for (int t = 0; t < DT; ++t) csn[t] = ccs[t] = 0.0;
  float mx = 0.0f;
  bool bad = false;
  const int64_t rb = static_cast<int64_t>(blockIdx.x) * rows_per_block;
  const int64_t re = min(n, rb + rows_per_block);
  for (int64_t r0 = rb; r0 < re; r0 += 64) {
    const int64_t arow = r0 + 16 * w + i16;
    const bool aok = arow < re;
    float a[KS];
    float ss = 0.0f;
#pragma unroll
    for (int st4 = 0; st4 < KS; ++st4) {
      const int k = 4 * st4 + kq;
      a[st4] = (aok && k < d) ? Z[arow * dp + k] : 0.0f;
      ss += a[st4] * a[st4];
    }
    ss += __shfl_xor(ss, 16, 64);
    ss += __shfl_xor(ss, 32, 64);
    const float inv = ss > 0.0f ? 1.0f / sqrtf(ss) : 0.0f;  // for row i16 of the tile
    float invr[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) invr[v] = __shfl(inv, 4 * kq + v, 64);
    float sv[DT][4], cv[DT][4];
#pragma unroll
    for (int t = 0; t < DT; ++t) {
      v4f_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int st4 = 0; st4 < KS; ++st4)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st4], qts[(4 * st4 + kq) * DPAD + 16 * t + i16], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float sn, cn;
        sincosf(sqrtd * (acc[v] * invr[v]), &sn, &cn);
        sv[t][v] = sn * amp;
        cv[t][v] = cn * amp;
      }
    }
    if (PASS == 1) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool live = r0 + 16 * w + 4 * kq + v < re;
#pragma unroll
        for (int t = 0; t < DT; ++t) {
          if (live && 16 * t + i16 < d) {
            csn[t] += static_cast<double>(sv[t][v]);
            ccs[t] += static_cast<double>(cv[t][v]);
          }
        }
      }
    } else {
      double pd[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        pd[v] = 0.0;
#pragma unroll
        for (int t = 0; t < DT; ++t) {
          const int c = 16 * t + i16;
          pd[v] = fma(static_cast<double>(sv[t][v]), rsl[c], pd[v]);
          pd[v] = fma(static_cast<double>(cv[t][v]), rsl[DPAD + c], pd[v]);
        }
      }
#pragma unroll
      for (int o = 1; o < 16; o <<= 1)
#pragma unroll
        for (int v = 0; v < 4; ++v) pd[v] += __shfl_xor(pd[v], o, 64);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 16 * w + 4 * kq + v;
        if (row >= re) continue;
        double dot = pd[v];
        if (!(dot > 0.0) || !isfinite(dot)) {
          bad = true;
          dot = 1.0;
        }
        const float sc = static_cast<float>(1.0 / sqrt(dot));
#pragma unroll
        for (int t = 0; t < DT; ++t) {
          const int c = 16 * t + i16;
          if (c < d) {
            const float o1 = sv[t][v] * sc, o2 = cv[t][v] * sc;
            R[row * twod + c] = o1;
            R[row * twod + d + c] = o2;
            csn[t] += static_cast<double>(o1);
            ccs[t] += static_cast<double>(o2);
            mx = fmaxf(mx, fmaxf(fabsf(o1), fabsf(o2)));
          }
        }
      }
    }
  }
  // per-workgroup column sums: the four lanes of a column, then the waves
#pragma unroll
  for (int t = 0; t < DT; ++t) {
    csn[t] += __shfl_xor(csn[t], 16, 64);
    csn[t] += __shfl_xor(csn[t], 32, 64);
    ccs[t] += __shfl_xor(ccs[t], 16, 64);
    ccs[t] += __shfl_xor(ccs[t], 32, 64);
    if (kq == 0) {
      cs[w][16 * t + i16] = csn[t];
      cs[w][DPAD + 16 * t + i16] = ccs[t];
    }
  }
  if (PASS == 2) {
    if (bad) atomicOr(&st->err_bits, 8);
    mx = wave_max(mx);
    if (lane == 0) atomic_max_nonneg(&st->maxabs_r_bits, mx);
  }
  __syncthreads();
  for (int j = tid; j < twod; j += 256) {
    const int src = j < d ? j : DPAD + (j - d);
    const double v = ((cs[0][src] + cs[1][src]) + cs[2][src]) + cs[3][src];
    part[static_cast<int64_t>(blockIdx.x) * twod + j] = v;
  }
}

template <int DT>
static void features_mfma(const Plan& p, void* ws, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  const int nb = p.rowpass_blocks;
  const int rpb = static_cast<int>((p.n + nb - 1) / nb);
  double* part = bufp<double>(p, ws, B_RPART);
  float* R = bufp<float>(p, ws, B_R);
  const float* Z = bufp<float>(p, ws, B_Z);
  const float* Qt = bufp<float>(p, ws, B_QT32);
  const size_t lds = sizeof(float) * 16 * DT * 16 * DT;
  const int64_t n = p.n;
  hipLaunchKernelGGL((k_feat_mfma<1, DT>), dim3(nb), dim3(256), lds, s, Z, n, p.d, p.dp, Qt, rpb,
                     static_cast<const double*>(nullptr), R, part, st);
  TPO_LAUNCH_CHECK();
  reduce_parts(part, nb, p.twod, bufp<double>(p, ws, B_REDTMP), bufp<double>(p, ws, B_RSUM), s);
  hipLaunchKernelGGL((k_feat_mfma<2, DT>), dim3(nb), dim3(256), lds, s, Z, n, p.d, p.dp, Qt, rpb,
                     bufp<double>(p, ws, B_RSUM), R, part, st);
  TPO_LAUNCH_CHECK();
  reduce_parts(part, nb, p.twod, bufp<double>(p, ws, B_REDTMP), bufp<double>(p, ws, B_RCOLSUM), s);
}

// Deterministic two-level column sums of part (nparts x len): block (x, y)
// sums slice y of the parts for 64 columns (4 interleaved sub-sums added in
// a fixed order), then one thread per column adds the slices in order.
constexpr int kRedSlices = 16;

__global__ void __launch_bounds__(256)
k_reduce_slices(const double* __restrict__ part, int nparts, int len, double* __restrict__ tmp) {
  __shared__ double sh[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  const int per = (nparts + kRedSlices - 1) / kRedSlices;
  const int p0 = blockIdx.y * per, p1 = min(nparts, p0 + per);
  double s = 0.0;
  if (c < len)
    for (int b = p0 + g; b < p1; b += 4) s += part[static_cast<int64_t>(b) * len + c];
  sh[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && c < len) {
    const int t = threadIdx.x & 63;
    tmp[static_cast<int64_t>(blockIdx.y) * len + c] = ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t];
  }
}

__global__ void k_reduce_final(const double* __restrict__ tmp, int len, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= len) return;
  double s = 0.0;
  for (int y = 0; y < kRedSlices; ++y) s += tmp[static_cast<int64_t>(y) * len + c];
  out[c] = s;
}

void reduce_parts(const double* part, int nparts, int len, double* tmp, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_slices, dim3(ceil_div(len, 64), kRedSlices), dim3(256), 0, s, part, nparts, len, tmp);
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce_final, dim3(ceil_div(len, 256)), dim3(256), 0, s, tmp, len, out);
  TPO_LAUNCH_CHECK();
}

__global__ void k_transpose_f32(const double* __restrict__ Q, int d, float* __restrict__ Qt32) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  const int j = idx / d, l = idx % d;
  Qt32[idx] = static_cast<float>(Q[l * d + j]);
}

void launch_features(const Plan& p, void* ws, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  if (p.d <= kLdsMaxN) {
    // Q = G R^-1 by Cholesky QR, done twice (the positive-diagonal QR factor)
    double* Q = bufp<double>(p, ws, B_Q);
    TPO_HIP_CHECK(hipMemcpyAsync(Q, bufp<double>(p, ws, B_G), sizeof(double) * p.d * p.d, hipMemcpyDeviceToDevice, s));
    cholqr_lds(Q, p.d, p.d, p.d, &st->err_bits, s);
    cholqr_lds(Q, p.d, p.d, p.d, &st->err_bits, s);
    hipLaunchKernelGGL(k_transpose_f32, dim3(ceil_div(p.d * p.d, 256)), dim3(256), 0, s, Q, p.d,
                       bufp<float>(p, ws, B_QT32));
    TPO_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL(k_q_from_g, dim3(1), dim3(kSmallThreads), 0, s, bufp<double>(p, ws, B_G), p.d,
                       bufp<double>(p, ws, B_Q), bufp<double>(p, ws, B_SMALL_A), bufp<float>(p, ws, B_QT32),
                       &st->err_bits);
    TPO_LAUNCH_CHECK();
  }
  switch ((p.d + 15) / 16) {
    case 1: features_mfma<1>(p, ws, s); break;
    case 2: features_mfma<2>(p, ws, s); break;
    case 3: features_mfma<3>(p, ws, s); break;
    case 4: features_mfma<4>(p, ws, s); break;
    case 5: features_mfma<5>(p, ws, s); break;
    case 6: features_mfma<6>(p, ws, s); break;
    case 7: features_mfma<7>(p, ws, s); break;
    default: features_mfma<8>(p, ws, s); break;
  }
}

int jacobi_log_n(const Plan& p) {
  int n = 0;
  if (p.reduce && p.lr <= kLdsMaxN) n = p.lr;
  if (p.kp > kLdsMaxN && p.kp <= kWideMaxN) n = std::max(n, p.kp);
  return n;
}

JacobiLog jacobi_log(const Plan& p, void* ws) {
  const int n = jacobi_log_n(p);
  const int np = n + (n & 1);
  char* base = bufp<char>(p, ws, B_JLOG);
  JacobiLog j;
  j.rot = reinterpret_cast<double2*>(base);
  int* ints = reinterpret_cast<int*>(base + sizeof(double2) * jacobi_log_steps(n) * (np / 2 > 0 ? np / 2 : 1));
  j.steps = ints;
  j.count = ints + jacobi_log_steps(n);
  j.perm = j.count + 1;
  return j;
}

void launch_embed(const Plan& p, void* ws, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  double* K = bufp<double>(p, ws, B_K);
  gram(bufp<float>(p, ws, B_R), 0, nullptr, p.n, p.twod, p.twod, p.gram_chunks_r, bufp<double>(p, ws, B_GRAM_PART), nullptr,
       K, nullptr, s);
  if (p.kp <= kWideMaxN) {
    // q products with K, each followed by Cholesky QR, then P = K M
    double* m = bufp<double>(p, ws, B_SI_M);
    double* pm = bufp<double>(p, ws, B_SI_P);
    subspace_iterate(K, p.twod, bufp<double>(p, ws, B_OMEGA), p.kp, p.par.q, bufp<double>(p, ws, B_M_A),
                     bufp<double>(p, ws, B_M_B), bufp<double>(p, ws, B_SI_GRAM), bufp<double>(p, ws, B_SI_PART),
                     bufp<unsigned>(p, ws, B_SI_BAR), m, pm, &st->err_bits, s);
    if (p.kp <= kLdsMaxN)
      embed_final_lds(m, pm, p.twod, p.kp, p.k, bufp<double>(p, ws, B_RCOLSUM), static_cast<int64_t>(p.n),
                      bufp<double>(p, ws, B_EEVAL), bufp<float>(p, ws, B_S32), bufp<double>(p, ws, B_SIGMA),
                      bufp<double>(p, ws, B_PSI), bufp<double>(p, ws, B_H), bufp<float>(p, ws, B_H32), &st->err_bits,
                      s);
    else
      embed_final_wide(m, pm, p.twod, p.kp, p.k, bufp<double>(p, ws, B_RCOLSUM), static_cast<int64_t>(p.n),
                       bufp<double>(p, ws, B_EEVAL), bufp<float>(p, ws, B_S32), bufp<double>(p, ws, B_SIGMA),
                       bufp<double>(p, ws, B_PSI), bufp<double>(p, ws, B_H), bufp<float>(p, ws, B_H32),
                       jacobi_log(p, ws), &st->err_bits, s);
    return;
  }
  hipLaunchKernelGGL(k_embed_small, dim3(1), dim3(kSmallThreads), 0, s, K, bufp<double>(p, ws, B_OMEGA), p.twod,
                     p.kp, p.k, p.par.q, bufp<double>(p, ws, B_RCOLSUM), static_cast<int64_t>(p.n),
                     bufp<double>(p, ws, B_M_A), bufp<double>(p, ws, B_M_B), bufp<double>(p, ws, B_EK_A),
                     bufp<double>(p, ws, B_EK_B), bufp<double>(p, ws, B_EK_C), bufp<double>(p, ws, B_EEVAL),
                     bufp<float>(p, ws, B_S32), bufp<double>(p, ws, B_SIGMA), bufp<double>(p, ws, B_PSI),
                     bufp<double>(p, ws, B_H), bufp<float>(p, ws, B_H32), &st->err_bits);
  TPO_LAUNCH_CHECK();
}

}  // namespace tpo
