// Workgroup-level FP64 dense linear algebra on small matrices (sizes up to a
// few hundred), used by single-workgroup kernels.  Every routine is called by
// all threads of the block and ends with a barrier.  Matrices are row-major;
// pointers may address LDS or global memory.
#pragma once

#include <hip/hip_runtime.h>

namespace tpo {

// C = alpha * op(A) * op(B) + beta * C; op(A) is m x k, op(B) is k x n.
__device__ inline void blk_gemm(int m, int n, int k, const double* A, int lda, bool ta, const double* B, int ldb,
                                bool tb, double* C, int ldc, double alpha, double beta) {
  const int nt = blockDim.x;
  for (int idx = threadIdx.x; idx < m * n; idx += nt) {
    const int r = idx / n, c = idx - (idx / n) * n;
    double acc = 0.0;
    for (int t = 0; t < k; ++t) {
      const double a = ta ? A[t * lda + r] : A[r * lda + t];
      const double b = tb ? B[c * ldb + t] : B[t * ldb + c];
      acc = fma(a, b, acc);
    }
    C[r * ldc + c] = (beta == 0.0) ? alpha * acc : alpha * acc + beta * C[r * ldc + c];
  }
  __syncthreads();
}

__device__ inline void blk_copy(int m, int n, const double* A, int lda, double* B, int ldb) {
  for (int idx = threadIdx.x; idx < m * n; idx += blockDim.x) {
    const int r = idx / n, c = idx - (idx / n) * n;
    B[r * ldb + c] = A[r * lda + c];
  }
  __syncthreads();
}

// In-place Cholesky G = L L^T (lower triangle, upper part left untouched).
// Returns false (uniformly) if a pivot is not positive and finite.
__device__ inline bool blk_chol(double* G, int n, int ld, int* sh_flag) {
  if (threadIdx.x == 0) *sh_flag = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      const double d = G[j * ld + j];
      if (!(d > 0.0) || !isfinite(d)) *sh_flag = 1;
      G[j * ld + j] = sqrt(d > 0.0 ? d : 1.0);
    }
    __syncthreads();
    if (*sh_flag) return false;
    const double piv = G[j * ld + j];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) G[i * ld + j] /= piv;
    __syncthreads();
    const int rem = n - j - 1;
    for (int idx = threadIdx.x; idx < rem * rem; idx += blockDim.x) {
      const int i = j + 1 + idx / rem, l = j + 1 + idx % rem;
      if (l <= i) G[i * ld + l] -= G[i * ld + j] * G[l * ld + j];
    }
    __syncthreads();
  }
  return true;
}

// A (m x n) <- A L^{-T} with L lower triangular (n x n): row-wise forward
// substitution, one thread per row.
__device__ inline void blk_trsm_right_lt(double* A, int m, int n, int lda, const double* L, int ldl) {
  for (int r = threadIdx.x; r < m; r += blockDim.x) {
    double* a = A + r * lda;
    for (int j = 0; j < n; ++j) {
      double x = a[j];
      for (int t = 0; t < j; ++t) x -= L[j * ldl + t] * a[t];
      a[j] = x / L[j * ldl + j];
    }
  }
  __syncthreads();
}

// A (m x n) <- A L^{-T} via explicit inverse is not used; this computes
// X = L^{-1} B for B (n x c), one thread per column.
__device__ inline void blk_trsm_left_l(double* B, int n, int c, int ldb, const double* L, int ldl) {
  for (int col = threadIdx.x; col < c; col += blockDim.x) {
    for (int j = 0; j < n; ++j) {
      double x = B[j * ldb + col];
      for (int t = 0; t < j; ++t) x -= L[j * ldl + t] * B[t * ldb + col];
      B[j * ldb + col] = x / L[j * ldl + j];
    }
  }
  __syncthreads();
}

// Orthonormalise the columns of A (m x n) in place by Cholesky QR:
// G = A^T A = L L^T, A <- A L^{-T}.  G is n x n scratch (LDS preferred).
__device__ inline bool blk_cholqr(double* A, int m, int n, int lda, double* G, int ldg, int* sh_flag) {
  blk_gemm(n, n, m, A, lda, true, A, lda, false, G, ldg, 1.0, 0.0);
  if (!blk_chol(G, n, ldg, sh_flag)) return false;
  blk_trsm_right_lt(A, m, n, lda, G, ldg);
  return true;
}

// Deterministic block sum (fixed tree order); sh holds blockDim.x doubles and
// blockDim.x must be a power of two.
__device__ inline double blk_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Cyclic Jacobi eigensolver for a symmetric n x n matrix A (in place; on exit
// the diagonal holds the eigenvalues) with eigenvectors in the columns of V.
// Parallel (round-robin) ordering: n/2 disjoint rotations per step.
// sh: scratch of 3 * ((n + 1) / 2) + 1 doubles; red: blockDim.x doubles.
__device__ inline void blk_jacobi(double* A, int lda, double* V, int ldv, int n, double* sh, double* red,
                                  int max_sweeps) {
  const int np = n + (n & 1);
  const int npairs = np / 2;
  double* cs = sh;               // c
  double* sn = sh + npairs;      // s
  int* pp = reinterpret_cast<int*>(sh + 2 * npairs);
  int* qq = pp + npairs;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int r = idx / n, c = idx % n;
    V[r * ldv + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence: off-diagonal mass relative to the diagonal
    double off = 0.0, dia = 0.0;
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
      const int i = idx / n, j = idx % n;
      const double v = A[i * lda + j];
      if (i == j) dia += v * v; else off += v * v;
    }
    off = blk_sum(off, red);
    dia = blk_sum(dia, red);
    if (off <= 1e-30 * dia || off == 0.0) break;
    for (int step = 0; step < np - 1; ++step) {
      for (int i = threadIdx.x; i < npairs; i += blockDim.x) {
        int p, q;
        if (i == 0) {
          p = step;
          q = np - 1;
        } else {
          p = (step + i) % (np - 1);
          q = (step - i + (np - 1)) % (np - 1);
        }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * lda + q];
          if (apq != 0.0) {
            const double app = A[p * lda + p], aqq = A[q * lda + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        cs[i] = c;
        sn[i] = s;
        pp[i] = p;
        qq[i] = q < n ? q : -1;
      }
      __syncthreads();
      // rows: A <- J^T A  (threads: 32 pair lanes x 32 column lanes)
      {
        const int tr = threadIdx.x >> 5, tcc = threadIdx.x & 31;
        for (int i = tr; i < npairs; i += (blockDim.x >> 5)) {
          const int q = qq[i];
          if (q < 0 || sn[i] == 0.0) continue;
          const int p = pp[i];
          const double c = cs[i], s = sn[i];
          for (int j = tcc; j < n; j += 32) {
            const double apj = A[p * lda + j], aqj = A[q * lda + j];
            A[p * lda + j] = c * apj - s * aqj;
            A[q * lda + j] = s * apj + c * aqj;
          }
        }
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      {
        const int tr = threadIdx.x >> 5, tcc = threadIdx.x & 31;
        for (int i = tr; i < npairs; i += (blockDim.x >> 5)) {
          const int q = qq[i];
          if (q < 0 || sn[i] == 0.0) continue;
          const int p = pp[i];
          const double c = cs[i], s = sn[i];
          for (int r = tcc; r < n; r += 32) {
            const double arp = A[r * lda + p], arq = A[r * lda + q];
            A[r * lda + p] = c * arp - s * arq;
            A[r * lda + q] = s * arp + c * arq;
            const double vrp = V[r * ldv + p], vrq = V[r * ldv + q];
            V[r * ldv + p] = c * vrp - s * vrq;
            V[r * ldv + q] = s * vrp + c * vrq;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Order eigenpairs by decreasing eigenvalue (ties keep the lower index):
// evals[i] <- sorted diagonal of A, perm[i] <- source column.
__device__ inline void blk_sort_desc(const double* A, int lda, int n, double* evals, int* perm) {
  if (threadIdx.x == 0) {
    for (int i = 0; i < n; ++i) {
      evals[i] = A[i * lda + i];
      perm[i] = i;
    }
    for (int i = 1; i < n; ++i) {  // stable insertion sort, descending
      const double v = evals[i];
      const int pi = perm[i];
      int j = i - 1;
      while (j >= 0 && evals[j] < v) {
        evals[j + 1] = evals[j];
        perm[j + 1] = perm[j];
        --j;
      }
      evals[j + 1] = v;
      perm[j + 1] = pi;
    }
  }
  __syncthreads();
}

}  // namespace tpo
