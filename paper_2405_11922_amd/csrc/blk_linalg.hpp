// Workgroup-level FP64 dense linear algebra on small matrices (sizes up to a
// few hundred), used by single-workgroup kernels.  Every routine is called by
// all threads of the block and ends with a barrier.  Matrices are row-major;
// pointers may address LDS or global memory.
#pragma once

#include <hip/hip_runtime.h>

#include "dev_common.hpp"

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

// Off-diagonal entries below this multiple of sqrt(|a_pp a_qq|) are treated
// as converged (relative accuracy at the level of FP64 rounding).
constexpr double kJacobiTol = 1e-16;

// 1/x and 1/sqrt(x) for positive normal x: the hardware estimates refined by
// two Newton steps each (quadratic convergence: a few ulp from exact).
__device__ __forceinline__ double rcp_refined(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

__device__ __forceinline__ double rsq_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// Cyclic Jacobi eigensolver for a symmetric n x n matrix A (in place; on exit
// the diagonal holds the eigenvalues) with eigenvectors in the columns of V.
// Parallel (round-robin) ordering: n/2 disjoint rotations per step.  A step
// is two phases: thread i < n/2 forms the rotation of pair i; then wave w
// applies A <- J^T A J to the 2 x 2 blocks (pair i rows, pair j columns) of
// its pairs i = w, w + waves, ... with lane j taking block (i, j), and
// V <- V J to the rows (one per lane) of the same pairs.  The coupling of a
// rotated pair is set to zero.  Stops after a sweep that rotates nothing (or
// after max_sweeps).  Returns the number of sweeps taken.
// sh: scratch of 3 * ((n + 1) / 2) + 1 doubles; red: unused.

__device__ inline int blk_jacobi(double* A, int lda, double* V, int ldv, int n, double* sh, double* red,
                                 int max_sweeps) {
  (void)red;
  const int np = n + (n & 1);
  const int npairs = np / 2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double* cs = sh;               // c
  double* sn = sh + npairs;      // s
  int* pp = reinterpret_cast<int*>(sh + 2 * npairs);
  int* qq = pp + npairs;
  int* rotated = qq + npairs;    // set when a sweep applied any rotation
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int r = idx / n, c = idx % n;
    V[r * ldv + c] = (r == c) ? 1.0 : 0.0;
  }
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) *rotated = 0;
    __syncthreads();
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
          const double app = A[p * lda + p], aqq = A[q * lda + q];
          // rotate only while the pair is coupled above rounding level
          if (fabs(apq) > kJacobiTol * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-140) {
            // t = tan of the angle that annihilates a_pq: with a = a_qq - a_pp
            // and b = 2 a_pq, t = sign(a) b / (|a| + sqrt(a^2 + b^2))
            const double da = aqq - app, db = 2.0 * apq;
            const double h = fma(da, da, db * db);
            const double root = h * rsq_refined(h);
            const double t = (da >= 0.0 ? db : -db) * rcp_refined(fabs(da) + root);
            c = rsq_refined(fma(t, t, 1.0));
            s = t * c;
            if (s != 0.0) *rotated = 1;
          }
        }
        cs[i] = c;
        sn[i] = s;
        pp[i] = p;
        qq[i] = q < n ? q : -1;
      }
      __syncthreads();
      for (int i = w; i < npairs; i += nw) {
        const double si = sn[i];
        const double ci = cs[i];
        const int pi = pp[i], qi = qq[i];
        // A <- J^T A J on blocks (i, j): rows of pair i by J_i^T, columns of pair j by J_j
        for (int j = lane; j < npairs; j += 64) {
          const double sj = sn[j], cj = cs[j];
          const int pj = pp[j], qj = qq[j];
          if (si == 0.0 && sj == 0.0) continue;
          const double a = A[pi * lda + pj];
          const double b = qj >= 0 ? A[pi * lda + qj] : 0.0;
          const double c = qi >= 0 ? A[qi * lda + pj] : 0.0;
          const double d = (qi >= 0 && qj >= 0) ? A[qi * lda + qj] : 0.0;
          const double a1 = ci * a - si * c, b1 = ci * b - si * d;
          const double c1 = si * a + ci * c, d1 = si * b + ci * d;
          const double a2 = cj * a1 - sj * b1;
          double b2 = sj * a1 + cj * b1;
          double c2 = cj * c1 - sj * d1;
          const double d2 = sj * c1 + cj * d1;
          if (i == j && si != 0.0) {  // the rotated pair's own coupling is annihilated
            b2 = 0.0;
            c2 = 0.0;
          }
          A[pi * lda + pj] = a2;
          if (qj >= 0) A[pi * lda + qj] = b2;
          if (qi >= 0) A[qi * lda + pj] = c2;
          if (qi >= 0 && qj >= 0) A[qi * lda + qj] = d2;
        }
        // V <- V J_i on this lane's rows
        if (si != 0.0) {
          for (int r = lane; r < n; r += 64) {
            const double vp = V[r * ldv + pi], vq = V[r * ldv + qi];
            V[r * ldv + pi] = ci * vp - si * vq;
            V[r * ldv + qi] = si * vp + ci * vq;
          }
        }
      }
      __syncthreads();
    }
    const int any = *rotated;
    __syncthreads();
    if (!any) break;
  }
  __syncthreads();
  return sweep;
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
