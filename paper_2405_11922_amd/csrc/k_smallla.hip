// Single-workgroup FP64 kernels for the small dense steps of the randomized
// SVDs, with every small (n x n, n <= 80) matrix resident in LDS and the
// tall factors (m x n, m up to a few hundred) streamed through LDS in row
// chunks:
//   k_cholqr_lds   Cholesky QR of a tall m x n block (in place)
//   k_rr_reduce    Rayleigh-Ritz of the attribute reduction
//   k_embed_final  B = Q^T R, its SVD, Gamma's right factor S, Psi, Sigma
#include "blk_chol16.hpp"
#include "blk_linalg.hpp"
#include "dev_common.hpp"
#include "tpo_internal.hpp"

namespace tpo {

constexpr int kLdsN = 80;     // largest n kept in LDS
constexpr int kStage = 16;    // rows per staging chunk
constexpr int kLT = 1024;     // threads

typedef double v4d __attribute__((ext_vector_type(4)));

// G (n x n, ldg, LDS) = A^T B over m rows of A and B (global, row-major,
// n <= kLdsN columns) with FP64 MFMA 16x16x4: wave w takes output tiles
// w, w + 16, ...; a tile accumulates 4 rows per instruction.  Operand layout
// of v_mfma_f64_16x16x4f64: lane l supplies A[row = l % 16][k = l / 16] and
// B[k = l / 16][col = l % 16]; its v-th result is D[4 v + l / 16][l % 16]
// (rows interleaved across the four 16-lane groups, unlike the FP32 form).
// With sym the upper tiles are formed and mirrored.
__device__ void mfma_gram_f64(const double* A, int lda, const double* B, int ldb, int m, int n, double* G, int ldg,
                              bool sym) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nt = (n + 15) / 16;
  const int ntiles = sym ? nt * (nt + 1) / 2 : nt * nt;
  const int i16 = lane & 15, kq = lane >> 4;
  for (int t = w; t < ntiles; t += nw) {
    int ta, tb;
    if (sym) {
      int rem = t;
      ta = 0;
      while (rem >= nt - ta) {
        rem -= nt - ta;
        ++ta;
      }
      tb = ta + rem;
    } else {
      ta = t / nt;
      tb = t - ta * nt;
    }
    const int ca = ta * 16 + i16, cb = tb * 16 + i16;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    int r0 = 0;
    for (; r0 + 16 <= m; r0 += 16) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + 4 * u + kq;
        a[u] = ca < n ? A[r * lda + ca] : 0.0;
        b[u] = cb < n ? B[r * ldb + cb] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
    for (; r0 < m; r0 += 4) {
      const int r = r0 + kq;
      const double a = (r < m && ca < n) ? A[r * lda + ca] : 0.0;
      const double b = (r < m && cb < n) ? B[r * ldb + cb] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ta * 16 + 4 * v + kq, j = tb * 16 + i16;
      if (i < n && j < n && (!sym || i <= j)) G[i * ldg + j] = acc[v];
    }
  }
  __syncthreads();
  if (sym) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e - (e / n) * n;
      if (i > j) G[i * ldg + j] = G[j * ldg + i];
    }
    __syncthreads();
  }
}

// In-place lower Cholesky of an LDS matrix with one barrier per column: step
// j reads the pivot d = G[j][j] (final after the previous barrier), updates
// the trailing lower triangle with the unscaled column j and 1/d, and scales
// column j - 1 (no longer read).  Returns false uniformly on a non-positive
// or non-finite pivot.
__device__ bool lds_chol(double* G, int n, int ld) {
  const int tid = threadIdx.x;
  const int tr = tid >> 4, tc = tid & 15;  // 64 row lanes x 16 column lanes
  double prev_d = 0.0;
  for (int j = 0; j < n; ++j) {
    const double d = G[j * ld + j];
    if (!(d > 0.0) || !isfinite(d)) return false;
    const double inv = 1.0 / d;
    if (j > 0) {
      // column j - 1 is no longer read: finish it with its pivot sqrt(prev_d)
      const double sp = sqrt(prev_d);
      for (int i = j + tid; i < n; i += blockDim.x) G[i * ld + (j - 1)] /= sp;
      if (tid == 0) G[(j - 1) * ld + (j - 1)] = sp;
    }
    for (int i = j + 1 + tr; i < n; i += 64) {
      const double gij = G[i * ld + j] * inv;
      for (int l = j + 1 + tc; l <= i; l += 16) G[i * ld + l] -= gij * G[l * ld + j];
    }
    __syncthreads();
    prev_d = d;
  }
  if (tid == 0 && n > 0) G[(n - 1) * ld + (n - 1)] = sqrt(prev_d);
  __syncthreads();
  return true;
}

// A (m x n rows in global memory) <- A L^{-T}: per row, forward substitution
// L x^T = a^T.  Q threads share a row (Q divides 64); thread q keeps the
// entries t = q + Q u (u < NU) in registers, partial dot products are summed
// across the Q threads with xor shuffles.  No block barriers.
template <int Q, int NU>
__device__ void reg_trsm_lt(double* A, int lda, int m, int n, const double* L, int ldl) {
  const int q = threadIdx.x % Q;
  const int rows_per_pass = blockDim.x / Q;
  for (int r = threadIdx.x / Q; r - static_cast<int>(threadIdx.x / Q) < m; r += rows_per_pass) {
    const bool live = r < m;
    double xr[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int t = q + Q * u;
      xr[u] = (live && t < n) ? A[r * lda + t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      for (int jq = 0; jq < Q; ++jq) {
        const int j = u * Q + jq;
        if (j >= n) break;
        double part = 0.0;
#pragma unroll
        for (int u2 = 0; u2 <= u; ++u2) {
          const int t = q + Q * u2;
          if (t < j) part = fma(L[j * ldl + t], xr[u2], part);
        }
#pragma unroll
        for (int o = 1; o < Q; o <<= 1) part += __shfl_xor(part, o, 64);
        if (q == jq) xr[u] = (xr[u] - part) / L[j * ldl + j];
      }
    }
    if (live) {
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int t = q + Q * u;
        if (t < n) A[r * lda + t] = xr[u];
      }
    }
  }
  __syncthreads();
}

__device__ void trsm_rows(double* A, int lda, int m, int n, const double* L, int ldl) {
  if (m >= 256)
    reg_trsm_lt<4, (kLdsN + 3) / 4>(A, lda, m, n, L, ldl);
  else if (m >= 128)
    reg_trsm_lt<8, (kLdsN + 7) / 8>(A, lda, m, n, L, ldl);
  else
    reg_trsm_lt<16, (kLdsN + 15) / 16>(A, lda, m, n, L, ldl);
}




__global__ void __launch_bounds__(kLT)
k_cholqr_lds(double* __restrict__ A, int m, int n, int lda, int32_t* __restrict__ err_bits) {
  __shared__ double G[kC16Max * kC16Ld];
  __shared__ double Li[kC16Max * kC16Ld];
  __shared__ double scratch[4 * 256];
  __shared__ int flag;
  const int nb = (n + 15) / 16;
  gram16(A, lda, m, n, G, kC16Ld, nb);
  if (!blk_chol_inv16(G, Li, kC16Ld, nb, scratch, &flag)) {
    if (threadIdx.x == 0) atomicOr(err_bits, 16);
    return;
  }
  apply_linv_t(A, lda, m, n, Li, kC16Ld, nb);
}

// Jacobi of an n x n symmetric LDS matrix with V in LDS, then eigenpairs in
// decreasing order (perm, ev).
__device__ void lds_eig(double* A, double* V, int n, double* sh, double* red, int* perm, double* ev) {
  blk_jacobi(A, n, V, n, n, sh, red, 40);
  blk_sort_desc(A, n, n, ev, perm);
}

// Rows [0, rows) of X (leading dimension ldx, n <= 128 columns, global) times
// the rotations blk_jacobi logged, in the logged order: x <- x J_1 J_2 ...
// One wave per row, the row staged in LDS; lane i applies pair i of each
// step (the pairs of a step are disjoint; the wave's LDS accesses are in
// program order).
__global__ void __launch_bounds__(256)
k_jacobi_replay(const double2* __restrict__ rlog, const int* __restrict__ rsteps, const int* __restrict__ rcount,
                int n, double* __restrict__ X, int rows, int ldx) {
  __shared__ double xs[4][kJacobiMaxN];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = blockIdx.x * 4 + w;
  if (r >= rows) return;  // wave-uniform; no workgroup barrier below
  double* x = xs[w];
  for (int c = lane; c < n; c += 64) x[c] = X[static_cast<int64_t>(r) * ldx + c];
  wave_sync();
  const int np = n + (n & 1), npairs = np / 2;
  const int cnt = *rcount;
  // eight steps' rotations are loaded before they are applied
  constexpr int kB = 8;
  for (int e0 = 0; e0 < cnt; e0 += kB) {
    double2 cs[kB];
    int st[kB];
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const bool ok = e0 + b < cnt && lane < npairs;
      st[b] = e0 + b < cnt ? rsteps[e0 + b] : 0;
      cs[b] = ok ? rlog[static_cast<int64_t>(e0 + b) * npairs + lane] : make_double2(1.0, 0.0);
    }
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      if (lane < npairs && cs[b].y != 0.0) {
        int p, q;
        jacobi_pair(st[b], lane, np, p, q);
        if (q < n) {
          const double vp = x[p], vq = x[q];
          x[p] = cs[b].x * vp - cs[b].y * vq;
          x[q] = cs[b].y * vp + cs[b].x * vq;
        }
      }
      wave_sync();
    }
  }
  for (int c = lane; c < n; c += 64) X[static_cast<int64_t>(r) * ldx + c] = x[c];
}

// Rayleigh-Ritz of the reduction: T = M^T P (P = C M), eigenpairs, top d:
// Psi_d = M V_d, sigma_d = sqrt(lambda); sign convention on X' = X Psi_d.
// Three launches: the Jacobi on T in LDS without eigenvectors, logging its
// rotations (jlog; the raw eigenvalues in decreasing order go to evals);
// k_jacobi_replay applies them to the rows of M (M V, as V itself would be
// formed); the top d columns of M V in eigenvalue order, the sign convention
// and the FP32 copy.
__global__ void __launch_bounds__(kLT)
k_rr_eig(const double* __restrict__ M, const double* __restrict__ P, int du, int l, double* __restrict__ evals,
         JacobiLog jlog) {
  __shared__ double T[kLdsN * (kLdsN + 1)];
  __shared__ __align__(16) double sh[3 * 40 + 8];
  __shared__ int perm[kLdsN];
  __shared__ double ev[kLdsN];
  const int lt = l | 1;  // odd leading dimension of T: column walks spread over the LDS banks
  mfma_gram_f64(M, l, P, l, du, l, T, lt, false);
  for (int e = threadIdx.x; e < l * l; e += kLT) {
    const int i = e / l, j = e % l;
    if (i < j) {
      const double a = 0.5 * (T[i * lt + j] + T[j * lt + i]);
      T[i * lt + j] = a;
      T[j * lt + i] = a;
    }
  }
  __syncthreads();
  blk_jacobi(T, lt, nullptr, 0, l, sh, nullptr, kJacobiLogSweeps, jlog.rot, jlog.steps, jlog.count);
  blk_sort_desc(T, lt, l, ev, perm);
  for (int c = threadIdx.x; c < l; c += kLT) {
    evals[c] = ev[c];
    jlog.perm[c] = perm[c];
  }
}

// psi = (M V)[:, perm[:d]] from the replayed rows of M; evals[c] <- sigma_c.
__global__ void __launch_bounds__(kLT)
k_rr_finish(const double* __restrict__ MV, int du, int l, int d, int dp, const double* __restrict__ colsum_x,
            int64_t n, const int* __restrict__ perm, double* __restrict__ evals, double* __restrict__ psi,
            float* __restrict__ psi32) {
  __shared__ double ev[kLdsN];
  __shared__ double sgn[kLdsN];
  for (int c = threadIdx.x; c < d; c += kLT) ev[c] = evals[c];
  for (int e = threadIdx.x; e < du * d; e += kLT) {
    const int i = e / d, c = e - (e / d) * d;
    psi[e] = MV[static_cast<int64_t>(i) * l + min(max(perm[c], 0), l - 1)];
  }
  __syncthreads();
  // sign: colsum(X') = colsum(X) Psi_d; degenerate -> largest |Psi_d| entry
  // (the first one on a tie).  One wave per column.
  {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int c = w; c < d; c += kLT / 64) {
      const double lam = ev[c] > 0.0 ? ev[c] : 0.0;
      double s = 0.0;
      for (int i = lane; i < du; i += 64) s = fma(colsum_x[i], psi[i * d + c], s);
      s = wave_sum(s);
      if (fabs(s) <= 1e-9 * sqrt(static_cast<double>(n)) * sqrt(lam)) {
        double best = -1.0, bv = 0.0;
        int bi = du;
        for (int i = lane; i < du; i += 64) {
          const double v = psi[i * d + c];
          if (fabs(v) > best) {
            best = fabs(v);
            bv = v;
            bi = i;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, 64), ov = __shfl_xor(bv, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bv = ov;
            bi = oi;
          }
        }
        s = bv;
      }
      if (lane == 0) {
        evals[c] = sqrt(lam);
        sgn[c] = s < 0.0 ? -1.0 : 1.0;
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < du * dp; e += kLT) {
    const int i = e / dp, c = e % dp;
    if (c < d) {
      const double v = psi[i * d + c] * sgn[c];
      psi[i * d + c] = v;
      psi32[e] = static_cast<float>(v);
    } else {
      psi32[e] = 0.0f;
    }
  }
}

void rr_reduce_lds(double* M, const double* P, int du, int l, int d, int dp, const double* colsum_x, int64_t n,
                   double* evals, double* psi, float* psi32, JacobiLog jlog, hipStream_t s) {
  hipLaunchKernelGGL(k_rr_eig, dim3(1), dim3(kLT), 0, s, M, P, du, l, evals, jlog);
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_jacobi_replay, dim3(ceil_div(du, 4)), dim3(256), 0, s, jlog.rot, jlog.steps, jlog.count, l, M,
                     du, l);
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_rr_finish, dim3(1), dim3(kLT), 0, s, M, du, l, d, dp, colsum_x, n, jlog.perm, evals, psi,
                     psi32);
  TPO_LAUNCH_CHECK();
}

// Final step of RandomizedSVD(R, k) on K = R^T R with P = K M given:
//   L = chol(M^T P); B^T = P L^{-T}; M <- M L^{-T};  B B^T = U diag(lambda) U^T
//   S = M U_k (Gamma = R S), sigma = sqrt(lambda_k), Psi = B^T U_k / sigma,
// the column sign convention, and H = Psi Sigma (Eq. init-HY).
__global__ void __launch_bounds__(kLT)
k_embed_final(double* __restrict__ M, double* __restrict__ P, int twod, int kp, int k,
              const double* __restrict__ colsum_r, int64_t n, double* __restrict__ S, float* __restrict__ S32,
              double* __restrict__ sigma, double* __restrict__ psi, double* __restrict__ H,
              float* __restrict__ H32, int32_t* __restrict__ err_bits) {
  __shared__ double Gs[kC16Max * kC16Ld];
  __shared__ double Ls[kC16Max * kC16Ld];
  __shared__ double scratch[4 * 256];
  __shared__ int flag;
  __shared__ double red[kLT];
  __shared__ __align__(16) double sh[3 * 40 + 8];
  __shared__ int perm[kLdsN];
  __shared__ double ev[kLdsN];
  __shared__ double sgn[kLdsN];
  const int nb = (kp + 15) / 16;
  // M^T K M straight into the padded layout (identity on the padding)
  mfma_gram_f64(M, kp, P, kp, twod, kp, Gs, kC16Ld, false);
  for (int e = threadIdx.x; e < 16 * nb * 16 * nb; e += kLT) {
    const int i = e / (16 * nb), j = e % (16 * nb);
    if (i >= kp || j >= kp) {
      Gs[i * kC16Ld + j] = (i == j) ? 1.0 : 0.0;
    } else if (i < j) {
      const double a = 0.5 * (Gs[i * kC16Ld + j] + Gs[j * kC16Ld + i]);
      Gs[i * kC16Ld + j] = a;
      Gs[j * kC16Ld + i] = a;
    }
  }
  __syncthreads();
  // L = chol(M^T K M), Ls = L^{-1}; P <- B^T = K M L^{-T}; M <- M L^{-T}
  if (!blk_chol_inv16(Gs, Ls, kC16Ld, nb, scratch, &flag)) {
    if (threadIdx.x == 0) atomicOr(err_bits, 16);
    return;
  }
  apply_linv_t(P, kp, twod, kp, Ls, kC16Ld, nb);
  apply_linv_t(M, kp, twod, kp, Ls, kC16Ld, nb);
  mfma_gram_f64(P, kp, P, kp, twod, kp, Gs, kp, true);  // B B^T
  __syncthreads();
  lds_eig(Gs, Ls, kp, sh, red, perm, ev);
  for (int c = threadIdx.x; c < k; c += kLT) sigma[c] = sqrt(ev[c] > 0.0 ? ev[c] : 0.0);
  __syncthreads();
  for (int e = threadIdx.x; e < twod * k; e += kLT) {
    const int i = e / k, c = e % k;
    const int pc = perm[c];
    double a = 0.0, b = 0.0;
    for (int t = 0; t < kp; ++t) {
      a = fma(M[i * kp + t], Ls[t * kp + pc], a);
      b = fma(P[i * kp + t], Ls[t * kp + pc], b);
    }
    S[e] = a;
    psi[e] = sigma[c] > 0.0 ? b / sigma[c] : 0.0;
  }
  __syncthreads();
  // sign: colsum(Gamma) = colsum(R) S, ||Gamma[:, c]|| = 1
  for (int c = threadIdx.x; c < k; c += kLT) {
    double s = 0.0;
    for (int i = 0; i < twod; ++i) s = fma(colsum_r[i], S[i * k + c], s);
    if (fabs(s) <= 1e-9 * sqrt(static_cast<double>(n))) {
      double best = -1.0;
      s = 0.0;
      for (int i = 0; i < twod; ++i) {
        const double v = psi[i * k + c];
        if (fabs(v) > best) {
          best = fabs(v);
          s = v;
        }
      }
    }
    sgn[c] = s < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < twod * k; e += kLT) {
    const int c = e % k;
    const double sv = S[e] * sgn[c];
    const double pv = psi[e] * sgn[c];
    S[e] = sv;
    psi[e] = pv;
    S32[e] = static_cast<float>(sv);
    H[e] = pv * sigma[c];
    H32[e] = static_cast<float>(pv * sigma[c]);
  }
}

void cholqr_lds(double* A, int m, int n, int lda, int32_t* err_bits, hipStream_t s) {
  hipLaunchKernelGGL(k_cholqr_lds, dim3(1), dim3(kLT), 0, s, A, m, n, lda, err_bits);
  TPO_LAUNCH_CHECK();
}


// A (m x n, row-major, global) <- A Li^T with Li lower in LDS (ld), in
// stages of 16 rows copied to st (16 n doubles of LDS) first.
__device__ void apply_linv_t_staged(double* A, int m, int n, const double* Li, int ld, double* st) {
  for (int r0 = 0; r0 < m; r0 += 16) {
    const int nr = min(16, m - r0);
    for (int e = threadIdx.x; e < nr * n; e += blockDim.x) st[e] = A[static_cast<int64_t>(r0) * n + e];
    __syncthreads();
    for (int e = threadIdx.x; e < nr * n; e += blockDim.x) {
      const int r = e / n, c = e - (e / n) * n;
      double s = 0.0;
      for (int t = 0; t <= c; ++t) s = fma(st[r * n + t], Li[c * ld + t], s);
      A[static_cast<int64_t>(r0) * n + e] = s;
    }
    __syncthreads();
  }
}

// The same final step as k_embed_final for k' in 81..128, where the k' x k'
// eigenproblem and its eigenvectors do not both fit in LDS.  Three launches:
// (1) the Cholesky factor is inverted in place, M <- M L^-T and P <- K M L^-T
// in global memory, and the Jacobi runs on B B^T in LDS without
// eigenvectors, logging its rotations (jlog); (2) k_jacobi_replay applies the
// logged rotations to the rows of M and P (M V and P V, as V itself would be
// formed: V = J_1 J_2 ...); (3) the top k columns in eigenvalue order, the
// sign convention and the FP32 copies.
// jlog: the rotation log (JacobiLog), then the eigenvalue order.
__global__ void __launch_bounds__(kLT)
k_embed_wide_eig(double* __restrict__ M, double* __restrict__ P, int twod, int kp, int k,
                 double* __restrict__ sigma, JacobiLog jlog, int32_t* __restrict__ err_bits) {
  constexpr int kW = 128;
  __shared__ double G[kW * (kW + 1)];
  __shared__ __align__(16) double scr[8 * 256];  // factorisation scratch tiles; staged rows
  __shared__ double dinv[kW];
  __shared__ int flag;
  __shared__ __align__(16) double sh[3 * (kW / 2)];
  __shared__ int perm[kW];
  __shared__ double ev[kW];
  const int nb = (kp + 15) / 16;
  const int ld = 16 * nb + 1;
  // M^T K M in the padded layout (identity on the padding)
  mfma_gram_f64(M, kp, P, kp, twod, kp, G, ld, false);
  for (int e = threadIdx.x; e < 16 * nb * 16 * nb; e += kLT) {
    const int i = e / (16 * nb), j = e % (16 * nb);
    if (i >= kp || j >= kp) {
      G[i * ld + j] = (i == j) ? 1.0 : 0.0;
    } else if (i < j) {
      const double a = 0.5 * (G[i * ld + j] + G[j * ld + i]);
      G[i * ld + j] = a;
      G[j * ld + i] = a;
    }
  }
  __syncthreads();
  // L = chol(M^T K M) with L^{-1} in place; P <- B^T = K M L^{-T}; M <- M L^{-T}
  if (!blk_chol_inv16_inplace(G, ld, nb, scr, dinv, &flag)) {
    // breakdown (flagged): no rotations, the identity order, sigma zero
    if (threadIdx.x == 0) {
      atomicOr(err_bits, 16);
      *jlog.count = 0;
    }
    for (int c = threadIdx.x; c < k; c += kLT) {
      sigma[c] = 0.0;
      jlog.perm[c] = c;
    }
    return;
  }
  apply_linv_t_staged(P, twod, kp, G, ld, scr);
  apply_linv_t_staged(M, twod, kp, G, ld, scr);
  const int lj = kp | 1;
  mfma_gram_f64(P, kp, P, kp, twod, kp, G, lj, true);  // B B^T
  __syncthreads();
  blk_jacobi<2>(G, lj, nullptr, 0, kp, sh, nullptr, kJacobiLogSweeps, jlog.rot, jlog.steps, jlog.count);
  blk_sort_desc(G, lj, kp, ev, perm);
  for (int c = threadIdx.x; c < k; c += kLT) {
    sigma[c] = sqrt(ev[c] > 0.0 ? ev[c] : 0.0);
    jlog.perm[c] = perm[c];
  }
}



// S = (M V)[:, perm[:k]], psi = (P V)[:, perm[:k]] / sigma, then the sign
// convention (colsum(Gamma) = colsum(R) S; degenerate -> largest |psi| entry)
// and the FP32 copies.
__global__ void __launch_bounds__(kLT)
k_embed_wide_finish(const double* __restrict__ MV, const double* __restrict__ PV, int twod, int kp, int k,
                    const double* __restrict__ colsum_r, int64_t n, const int* __restrict__ perm,
                    double* __restrict__ S, float* __restrict__ S32, const double* __restrict__ sigma,
                    double* __restrict__ psi, double* __restrict__ H, float* __restrict__ H32) {
  __shared__ double sgn[128];
  for (int e = threadIdx.x; e < twod * k; e += kLT) {
    const int i = e / k, c = e % k;
    const int pc = min(max(perm[c], 0), kp - 1);
    S[e] = MV[i * kp + pc];
    psi[e] = sigma[c] > 0.0 ? PV[i * kp + pc] / sigma[c] : 0.0;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += kLT) {
    double s = 0.0;
    for (int i = 0; i < twod; ++i) s = fma(colsum_r[i], S[i * k + c], s);
    if (fabs(s) <= 1e-9 * sqrt(static_cast<double>(n))) {
      double best = -1.0;
      s = 0.0;
      for (int i = 0; i < twod; ++i) {
        const double v = psi[i * k + c];
        if (fabs(v) > best) {
          best = fabs(v);
          s = v;
        }
      }
    }
    sgn[c] = s < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < twod * k; e += kLT) {
    const int c = e % k;
    const double sv = S[e] * sgn[c];
    const double pv = psi[e] * sgn[c];
    S[e] = sv;
    psi[e] = pv;
    S32[e] = static_cast<float>(sv);
    H[e] = pv * sigma[c];
    H32[e] = static_cast<float>(pv * sigma[c]);
  }
}

void embed_final_wide(double* M, double* P, int twod, int kp, int k, const double* colsum_r, int64_t n, double* S,
                      float* S32, double* sigma, double* psi, double* H, float* H32, JacobiLog jlog,
                      int32_t* err_bits, hipStream_t s) {
  hipLaunchKernelGGL(k_embed_wide_eig, dim3(1), dim3(kLT), 0, s, M, P, twod, kp, k, sigma, jlog, err_bits);
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_jacobi_replay, dim3(ceil_div(twod, 4)), dim3(256), 0, s, jlog.rot, jlog.steps, jlog.count, kp,
                     M, twod, kp);
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_jacobi_replay, dim3(ceil_div(twod, 4)), dim3(256), 0, s, jlog.rot, jlog.steps, jlog.count, kp,
                     P, twod, kp);
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_embed_wide_finish, dim3(1), dim3(kLT), 0, s, M, P, twod, kp, k, colsum_r, n, jlog.perm, S, S32,
                     sigma, psi, H, H32);
  TPO_LAUNCH_CHECK();
}

void embed_final_lds(double* M, double* P, int twod, int kp, int k, const double* colsum_r, int64_t n, double* S,
                     float* S32, double* sigma, double* psi, double* H, float* H32, int32_t* err_bits,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_embed_final, dim3(1), dim3(kLT), 0, s, M, P, twod, kp, k, colsum_r, n, S, S32, sigma, psi,
                     H, H32, err_bits);
  TPO_LAUNCH_CHECK();
}

}  // namespace tpo
