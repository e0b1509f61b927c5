// Blocked FP64 Cholesky QR for one workgroup (16 waves), built from 16 x 16
// tiles on FP64 MFMA.  The n x n Gram (n <= 80) is padded to 16 * nb with an
// identity block, so its factor and inverse are blockdiag(L, I) and
// blockdiag(L^{-1}, I).
//
// v_mfma_f64_16x16x4f64 operand layout: lane l supplies A[l % 16][l / 16]
// (16 x 4) and B[l / 16][l % 16] (4 x 16); its v-th result is
// D[4 v + l / 16][l % 16].
#pragma once

#include <hip/hip_runtime.h>

#include "dev_common.hpp"

namespace tpo {

typedef double v4d_t __attribute__((ext_vector_type(4)));

constexpr int kC16Max = 80;          // largest n
constexpr int kC16Ld = kC16Max + 1;  // LDS leading dimension (odd: spreads banks)

// acc += op(A) op(B) for 16 x 16 tiles; ta / tb read the tile transposed.
// `neg` negates op(A).
__device__ __forceinline__ v4d_t mma16(const double* A, int lda, bool ta, const double* B, int ldb, bool tb,
                                       v4d_t acc, bool neg = false) {
  const int l = threadIdx.x & 63;
  const int i = l & 15, k = l >> 4;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int kk = 4 * s + k;
    double a = ta ? A[kk * lda + i] : A[i * lda + kk];
    const double b = tb ? B[i * ldb + kk] : B[kk * ldb + i];
    if (neg) a = -a;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ v4d_t load16(const double* C, int ldc) {
  const int l = threadIdx.x & 63;
  v4d_t r;
#pragma unroll
  for (int v = 0; v < 4; ++v) r[v] = C[(4 * v + (l >> 4)) * ldc + (l & 15)];
  return r;
}

__device__ __forceinline__ void store16(double* C, int ldc, v4d_t acc) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(4 * v + (l >> 4)) * ldc + (l & 15)] = acc[v];
}

// 1/sqrt(d) for a positive normal d: the hardware estimate refined by two
// Newton steps y <- y (1 + (1 - d y^2) / 2) (quadratic convergence, so the
// result is within a few ulp of the exact value).
__device__ __forceinline__ double rsqrt_refined(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double r = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, r, y);
  }
  return y;
}

// One wave: in-place lower Cholesky of a 16 x 16 LDS tile (lower triangle
// read and written); dinv[k] receives 1 / L[k][k].  The tile sits in
// registers for the whole factorisation (lane l holds column l % 16 of rows
// 4 v + l / 16, v = 0..3); the pivot and the factor column of each step
// reach the other lanes by cross-lane reads.  Returns false (wave-uniform)
// on a bad pivot.
__device__ __forceinline__ bool wave_chol16(double* B, int ld, double* dinv) {
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  double x[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) x[v] = B[(4 * v + g) * ld + c];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    double d = __shfl(x[k >> 2], 16 * (k & 3) + k, 64);
    if (!(d > 1e-290) || !isfinite(d)) {  // uniform; the loop runs on (fully unrolled) with a harmless pivot
      ok = false;
      d = 1.0;
    }
    const double inv = rsqrt_refined(d);
    if (c == k) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + g;
        if (r > k) x[v] *= inv;
        if (r == k) x[v] = d * inv;
      }
    }
    if (l == 0) dinv[k] = inv;
    // L[r][k] for this lane's rows r = 4 v + g (lane 16 g + k, register v)
    double lrk[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) lrk[v] = __shfl(x[v], (l & 48) + k, 64);
    // L[c][k] (row c sits in lane 16 (c % 4) + k, register c / 4)
    const int src = 16 * (c & 3) + k;
    const double t0 = __shfl(x[0], src, 64), t1 = __shfl(x[1], src, 64);
    const double t2 = __shfl(x[2], src, 64), t3 = __shfl(x[3], src, 64);
    const int vc = c >> 2;
    const double lck = vc == 0 ? t0 : (vc == 1 ? t1 : (vc == 2 ? t2 : t3));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * v + g;
      if (c > k && c <= r) x[v] -= lrk[v] * lck;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) B[(4 * v + g) * ld + c] = x[v];
  wave_sync();
  return ok;
}

// One wave: X = L^{-1} for a 16 x 16 lower LDS tile with dinv[r] = 1/L[r][r];
// lane c < 16 forms column c by forward substitution in registers.
__device__ __forceinline__ void wave_inv16(const double* L, int ldl, const double* dinv, double* X, int ldx) {
  const int c = threadIdx.x & 63;
  double x[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    double s = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int t = 0; t < r; ++t) s -= L[r * ldl + t] * x[t];
    x[r] = s * dinv[r];
  }
  if (c < 16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) X[r * ldx + c] = x[r];
  }
  wave_sync();
}

// Lane 16 (l / 16) + K's copy of v in every lane l (DPP row broadcast: one
// instruction for the 64-bit value).
template <int K>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x150 + K, 0xF, 0xF, true);  // every lane written: no old value
}

__device__ __forceinline__ double row_bcast_k(double v, int k) {  // k: a constant after unrolling
  switch (k) {
    case 0: return row_bcast<0>(v);
    case 1: return row_bcast<1>(v);
    case 2: return row_bcast<2>(v);
    case 3: return row_bcast<3>(v);
    case 4: return row_bcast<4>(v);
    case 5: return row_bcast<5>(v);
    case 6: return row_bcast<6>(v);
    case 7: return row_bcast<7>(v);
    case 8: return row_bcast<8>(v);
    case 9: return row_bcast<9>(v);
    case 10: return row_bcast<10>(v);
    case 11: return row_bcast<11>(v);
    case 12: return row_bcast<12>(v);
    case 13: return row_bcast<13>(v);
    case 14: return row_bcast<14>(v);
    default: return row_bcast<15>(v);
  }
}

// One wave: L = chol(B) and X = L^{-1} for a 16 x 16 LDS tile whose lower
// triangle holds the symmetric matrix.  On return the lower triangle of B
// holds L, its strictly upper triangle holds X transposed (B[c][r] = X[r][c],
// r > c), X (ldx) holds X with zeros above the diagonal, and dinv[k] =
// 1 / L[k][k].  Lane l keeps column c = l % 16 of the symmetric trailing
// matrix in registers (the four groups of 16 lanes hold the same, so a row
// broadcast from lane k of each group reaches every lane).  Step k
// broadcasts the pivot and column k of S, so every lane has column k of L;
// lane c stores its own entry L[c][k] = S[k][c] / sqrt(S[k][k]) (by the
// symmetry of the trailing matrix S) and then applies the rank-one update
// to its whole column: the columns already finished are never read again,
// so no lane needs a mask for it.  Column c of X solves L y = e_c and is
// advanced in the same loop.  Returns false (wave-uniform) on a bad pivot.
__device__ __forceinline__ bool wave_chol_inv16(double* B, int ld, double* dinv, double* X, int ldx) {
  const int l = threadIdx.x & 63, c = l & 15;
  double x[16], y[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    x[r] = r >= c ? B[r * ld + c] : B[c * ld + r];
    y[r] = r == c ? 1.0 : 0.0;
  }
  wave_sync();  // every lane has read B before L is written into it
  bool ok = true;
  double d = row_bcast<0>(x[0]);
  if (!(d > 1e-290) || !isfinite(d)) {  // uniform; the loop runs on (fully unrolled) with a harmless pivot
    ok = false;
    d = 1.0;
  }
  double inv = rsqrt_refined(d);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    // with s_r = S[r][k] (lane k's column) and L[r][k] = s_r inv:
    //   x[r] -= L[r][k] L[c][k] = s_r (inv L[c][k]),  y[r] -= L[r][k] y_k = s_r (inv y_k)
    const double lck = x[k] * inv;  // L[c][k] for c >= k
    if (l < 16 && c >= k) B[c * ld + k] = lck;
    if (l == 0) dinv[k] = inv;
    const double a = lck * inv;
    const double yk = y[k] * inv;
    const double b = yk * inv;
    y[k] = yk;
    double inv_next = 1.0;
    if (k + 1 < 16) {
      // the next pivot first, so that its square root overlaps the updates
      const double s1 = row_bcast_k(x[k + 1], k);
      x[k + 1] = fma(-s1, a, x[k + 1]);
      y[k + 1] = fma(-s1, b, y[k + 1]);
      double dn = row_bcast_k(x[k + 1], k + 1);
      if (!(dn > 1e-290) || !isfinite(dn)) {
        ok = false;
        dn = 1.0;
      }
      inv_next = rsqrt_refined(dn);
    }
#pragma unroll
    for (int r = k + 2; r < 16; ++r) {
      const double sr = row_bcast_k(x[r], k);
      x[r] = fma(-sr, a, x[r]);
      y[r] = fma(-sr, b, y[r]);
    }
    inv = inv_next;
    // keep each step's arithmetic in its step: left alone, the compiler
    // defers it and holds every step's column of L live at once
#pragma unroll
    for (int r = 0; r < 16; ++r) __asm__ volatile("" : "+v"(x[r]), "+v"(y[r]));
  }
  if (ok && l < 16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r > c) B[c * ld + r] = y[r];
      X[r * ldx + c] = y[r];
    }
  }
  wave_sync();
  return ok;
}

// Blocked Cholesky of the padded nb x nb tile matrix G (LDS, ld) with the
// inverses of its diagonal tiles left in Li; then Li = L^{-1} (lower).
// scratch: 16 waves x 16 x 16 doubles (or at least (nb - 1) tiles).
// Returns false uniformly when a pivot fails.
__device__ bool blk_chol_inv16(double* G, double* Li, int ld, int nb, double* scratch, int* flag) {
  __shared__ double dinv[kC16Max];
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  if (threadIdx.x == 0) *flag = 0;
  __syncthreads();
  for (int J = 0; J < nb; ++J) {
    double* GJJ = G + 16 * J * ld + 16 * J;
    double* LJJ = Li + 16 * J * ld + 16 * J;
    if (w == 0) {
      if (!wave_chol16(GJJ, ld, dinv + 16 * J)) {
        if ((threadIdx.x & 63) == 0) *flag = 1;
      } else {
        wave_inv16(GJJ, ld, dinv + 16 * J, LJJ, ld);
      }
    }
    __syncthreads();
    if (*flag) return false;
    // panel: L_IJ = G_IJ L_JJ^{-T}
    for (int I = J + 1 + w; I < nb; I += nw) {
      double* GIJ = G + 16 * I * ld + 16 * J;
      v4d_t acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(GIJ, ld, false, LJJ, ld, true, acc);
      store16(GIJ, ld, acc);
    }
    __syncthreads();
    // trailing: G_IK -= L_IJ L_KJ^T for J < K <= I
    const int m = nb - 1 - J;
    for (int p = w; p < m * (m + 1) / 2; p += nw) {
      int I = 0, rem = p;
      while (rem > I) {
        rem -= I + 1;
        ++I;
      }
      const int K = rem;  // 0 <= K <= I
      double* GIK = G + 16 * (J + 1 + I) * ld + 16 * (J + 1 + K);
      const double* LIJ = G + 16 * (J + 1 + I) * ld + 16 * J;
      const double* LKJ = G + 16 * (J + 1 + K) * ld + 16 * J;
      v4d_t acc = load16(GIK, ld);
      acc = mma16(LIJ, ld, false, LKJ, ld, true, acc, true);
      store16(GIK, ld, acc);
    }
    __syncthreads();
  }
  // zero the strictly upper tiles of Li, then Li_IJ = -Li_II sum_K L_IK Li_KJ
  for (int e = threadIdx.x; e < 16 * nb * 16 * nb; e += blockDim.x) {
    const int i = e / (16 * nb), j = e % (16 * nb);
    if (j / 16 > i / 16) Li[i * ld + j] = 0.0;
  }
  __syncthreads();
  for (int I = 1; I < nb; ++I) {
    for (int J = w; J < I; J += nw) {
      v4d_t acc = {0.0, 0.0, 0.0, 0.0};
      for (int K = J; K < I; ++K)
        acc = mma16(G + 16 * I * ld + 16 * K, ld, false, Li + 16 * K * ld + 16 * J, ld, false, acc);
      double* T = scratch + 256 * w;
      store16(T, 16, acc);
      wave_sync();
      v4d_t out = {0.0, 0.0, 0.0, 0.0};
      out = mma16(Li + 16 * I * ld + 16 * I, ld, false, T, 16, false, out, true);
      store16(Li + 16 * I * ld + 16 * J, ld, out);
    }
    __syncthreads();
  }
  return true;
}

// In-place variant: the lower tiles of G (LDS, ld) end as L^{-1}, so that
// one n x n array serves for n up to 128.  Factorisation as above, with the
// inverse of each diagonal tile kept in scratch tile 0 for the panel and
// transposed above the diagonal for later; then, for the block
// columns J from the last to the first, with the trailing block already
// inverted in place,
//   Li_IJ = -(sum_{J < K <= I} Li_IK L_KJ) Li_JJ   (I > J),
// the sums formed before any tile of column J is overwritten.
// scratch: nb tiles of 16 x 16 doubles; dinv: 16 nb doubles.
// Returns false uniformly when a pivot fails (G is then left part-factored).
__device__ __forceinline__ bool blk_chol_inv16_inplace(double* G, int ld, int nb, double* scratch, double* dinv, int* flag) {
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  double* S0 = scratch;
  if (threadIdx.x == 0) *flag = 0;
  __syncthreads();
  for (int J = 0; J < nb; ++J) {
    double* GJJ = G + 16 * J * ld + 16 * J;
    if (w == 0 && !wave_chol_inv16(GJJ, ld, dinv + 16 * J, S0, 16) && (threadIdx.x & 63) == 0) *flag = 1;
    __syncthreads();
    if (*flag) return false;
    for (int I = J + 1 + w; I < nb; I += nw) {
      double* GIJ = G + 16 * I * ld + 16 * J;
      v4d_t acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(GIJ, ld, false, S0, 16, true, acc);
      store16(GIJ, ld, acc);
    }
    __syncthreads();
    const int m = nb - 1 - J;
    for (int p = w; p < m * (m + 1) / 2; p += nw) {
      int I = 0, rem = p;
      while (rem > I) {
        rem -= I + 1;
        ++I;
      }
      const int K = rem;
      double* GIK = G + 16 * (J + 1 + I) * ld + 16 * (J + 1 + K);
      const double* LIJ = G + 16 * (J + 1 + I) * ld + 16 * J;
      const double* LKJ = G + 16 * (J + 1 + K) * ld + 16 * J;
      v4d_t acc = load16(GIK, ld);
      acc = mma16(LIJ, ld, false, LKJ, ld, true, acc, true);
      store16(GIK, ld, acc);
    }
    __syncthreads();
  }
  for (int J = nb - 1; J >= 0; --J) {
    double* GJJ = G + 16 * J * ld + 16 * J;
    if (w == 0) {  // Li_JJ from its transposed copy above the diagonal
      const int l = threadIdx.x & 63;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + (l >> 4), c = l & 15;
        S0[r * 16 + c] = r > c ? GJJ[c * ld + r] : (r == c ? dinv[16 * J + r] : 0.0);
      }
    }
    const int I = J + 1 + w;  // nb - 1 - J <= 7 < nw tiles below the diagonal
    v4d_t acc = {0.0, 0.0, 0.0, 0.0};
    if (I < nb) {
      for (int K = J + 1; K <= I; ++K)
        acc = mma16(G + 16 * I * ld + 16 * K, ld, false, G + 16 * K * ld + 16 * J, ld, false, acc);
    }
    __syncthreads();
    if (I < nb) {
      double* T = scratch + 256 * (1 + w);
      store16(T, 16, acc);
      wave_sync();
      v4d_t out = {0.0, 0.0, 0.0, 0.0};
      out = mma16(T, 16, false, S0, 16, false, out, true);
      store16(G + 16 * I * ld + 16 * J, ld, out);
    }
    if (w == nw - 1) {
      const int l = threadIdx.x & 63;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + (l >> 4), c = l & 15;
        GJJ[r * ld + c] = S0[r * 16 + c];
      }
    }
    __syncthreads();
  }
  return true;
}

// A (m x n, global, row-major lda) <- A Li^T with Li lower (LDS, padded to
// 16 nb).  Wave w owns row tiles w, w + 16, ...: it loads the tile's A
// operands for every k step first, then writes all its column tiles.
__device__ void apply_linv_t(double* A, int lda, int m, int n, const double* Li, int ld, int nb) {
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int l = threadIdx.x & 63, i = l & 15, k = l >> 4;
  const int nrt = (m + 15) / 16;
  for (int rt = w; rt < nrt; rt += nw) {
    const int row = 16 * rt + i;
    double a[4 * (kC16Max / 16)];
#pragma unroll
    for (int kt = 0; kt < kC16Max / 16; ++kt)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int col = 16 * kt + 4 * s + k;
        a[4 * kt + s] = (kt < nb && row < m && col < n) ? A[row * lda + col] : 0.0;
      }
#pragma unroll
    for (int ct = 0; ct < kC16Max / 16; ++ct) {
      if (ct >= nb) break;
      v4d_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kt = 0; kt <= ct; ++kt)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int kk = 16 * kt + 4 * s + k;  // k index of this lane
          const double b = Li[(16 * ct + i) * ld + kk];  // Li^T[kk][16 ct + i]
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[4 * kt + s], b, acc, 0, 0, 0);
        }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * rt + 4 * v + k, c = 16 * ct + i;
        if (r < m && c < n) A[r * lda + c] = acc[v];
      }
    }
  }
  __syncthreads();
}

// G (padded, LDS) = A^T A over the m rows of A (global).  Waves take output
// tiles; each loads 16 k steps (64 rows) of operands before the MFMAs.
__device__ void gram16(const double* A, int lda, int m, int n, double* G, int ld, int nb) {
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int l = threadIdx.x & 63, i = l & 15, k = l >> 4;
  const int ntiles = nb * (nb + 1) / 2;
  for (int t = w; t < ntiles; t += nw) {
    int ta = 0, rem = t;
    while (rem >= nb - ta) {
      rem -= nb - ta;
      ++ta;
    }
    const int tb = ta + rem;
    const int ca = 16 * ta + i, cb = 16 * tb + i;
    v4d_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int r0 = 0; r0 < m; r0 += 64) {
      double av[16], bv[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int r = r0 + 4 * s + k;
        av[s] = (r < m && ca < n) ? A[r * lda + ca] : 0.0;
        bv[s] = (r < m && cb < n) ? A[r * lda + cb] : 0.0;
      }
#pragma unroll
      for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * ta + 4 * v + k, c = 16 * tb + i;
      double val = acc[v];
      if (r >= n || c >= n) val = (r == c) ? 1.0 : 0.0;  // identity padding
      G[r * ld + c] = val;
      if (ta != tb) G[c * ld + r] = val;
    }
  }
  __syncthreads();
}

}  // namespace tpo
