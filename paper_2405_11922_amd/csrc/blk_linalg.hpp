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
constexpr int kJacobiMaxN = 160;  // largest n (steps per sweep: n - 1 or n)

// Coupled above rounding level: |a_pq| > tol sqrt(|a_pp a_qq|), tested on
// squares (no square root), and |a_pq| > 1e-140.
__device__ __forceinline__ bool jacobi_coupled(double apq, double app, double aqq) {
  return apq * apq > (kJacobiTol * kJacobiTol) * fabs(app * aqq) && fabs(apq) > 1e-140;
}

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

// Pair i of step `step` of the round-robin order over np (even) indices:
// (step, np - 1) for i = 0, else ((step + i) mod m, (step - i) mod m) with
// m = np - 1; returned with p < q.
__device__ __forceinline__ void jacobi_pair(int step, int i, int np, int& p, int& q) {
  const int m = np - 1;
  if (i == 0) {
    p = step;
    q = m;
  } else {
    p = step + i;
    if (p >= m) p -= m;
    q = step - i;
    if (q < 0) q += m;
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// Cyclic Jacobi eigensolver for a symmetric n x n matrix A (in place; on exit
// the diagonal holds the eigenvalues) with eigenvectors in the columns of V.
// Parallel (round-robin) ordering: n/2 disjoint rotations per step.  A step
// is two phases: thread i < n/2 forms the rotation of pair i; then the
// threads share out the 2 x 2 blocks (pair i rows, pair j columns) of
// A <- J^T A J and the (pair, row) items of V <- V J evenly.  The coupling of a
// rotated pair is set to zero.  Each sweep starts by marking the steps that
// hold a pair coupled above the threshold (pair (p, q) belongs to step p when
// q is the fixed index np - 1, else to the step s with 2 s = p + q modulo
// np - 1) and runs only those: a pair that becomes coupled again later in
// the sweep waits for the next one.  Stops when no step is marked (or after
// max_sweeps).  Returns the number of sweeps taken.
// V may be null: then no eigenvectors are formed, and when rlog is given the
// rotations of every step run are logged instead (rlog[e * (np / 2) + i] =
// (c, s) of pair i of the e-th step run, rsteps[e] = that step's index in its
// sweep, *rcount = steps run), for k_jacobi_replay to apply to other rows:
// V <- V J is then the same as x <- x J on every row x.
// sh: scratch of 3 * ((n + 1) / 2) doubles (16-byte aligned); red: unused.
// Each thread takes kBatches batches of 2 blocks and 4 rows of V:
// (n / 2)^2 <= 2 kBatches blockDim.x and n^2 / 2 <= 4 kBatches blockDim.x
// (kBatches = 1: n <= 80 with 1024 threads; 2: n <= 128; 4: n <= 160).

template <int kBatches = 1>
__device__ inline int blk_jacobi(double* A, int lda, double* V, int ldv, int n, double* sh, double* red,
                                 int max_sweeps, double2* rlog = nullptr, int* rsteps = nullptr,
                                 int* rcount = nullptr) {
  (void)red;
  constexpr int kA = 2, kV = 4;  // blocks and rows of V per thread and batch
  constexpr int kAT = kA * kBatches, kVT = kV * kBatches;
  const int np = n + (n & 1);
  const int npairs = np / 2;
  const int m = np - 1;          // steps per sweep (odd)
  const int half = (m + 1) / 2;  // 2 half = 1 modulo m
  double2* rot = reinterpret_cast<double2*>(sh);        // (c, s) of pair i
  int2* pq = reinterpret_cast<int2*>(sh + 2 * npairs);  // (p, q) of pair i; q = -1 off the matrix
  __shared__ int active[kJacobiMaxN];
  __shared__ int any;
  if (V) {
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
      const int r = idx / n, c = idx % n;
      V[r * ldv + c] = (r == c) ? 1.0 : 0.0;
    }
  }
  int nrun = 0;  // steps run (the rotation log's length)
  // this thread's items, fixed for the whole run: blocks (i, j) of J^T A J
  // and (pair i, row r) items of V J
  int bi[kAT], bj[kAT], vi[kVT], vr[kVT];
#pragma unroll
  for (int k = 0; k < kAT; ++k) {
    const int e = threadIdx.x + k * blockDim.x;
    bi[k] = e < npairs * npairs ? e / npairs : -1;
    bj[k] = e < npairs * npairs ? e - (e / npairs) * npairs : 0;
  }
#pragma unroll
  for (int k = 0; k < kVT; ++k) {
    const int e = threadIdx.x + k * blockDim.x;
    vi[k] = (V && e < npairs * n) ? e / n : -1;
    vr[k] = e < npairs * n ? e - (e / n) * n : 0;
  }
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) any = 0;
    for (int st = threadIdx.x; st < m; st += blockDim.x) active[st] = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int p = e / n, q = e - (e / n) * n;
      if (p < q && jacobi_coupled(A[p * lda + q], A[p * lda + p], A[q * lda + q])) {
        active[q == m ? p : ((p + q) * half) % m] = 1;
        any = 1;
      }
    }
    __syncthreads();
    if (!any) break;
    for (int step = 0; step < m; ++step) {
      if (!active[step]) continue;  // uniform
      for (int i = threadIdx.x; i < npairs; i += blockDim.x) {
        int p, q;
        jacobi_pair(step, i, np, p, q);
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * lda + q];
          const double app = A[p * lda + p], aqq = A[q * lda + q];
          // rotate only while the pair is coupled above rounding level
          if (jacobi_coupled(apq, app, aqq)) {
            // t = tan of the angle that annihilates a_pq: with a = a_qq - a_pp
            // and b = 2 a_pq, t = sign(a) b / (|a| + sqrt(a^2 + b^2))
            const double da = aqq - app, db = 2.0 * apq;
            const double h = fma(da, da, db * db);
            const double root = h * rsq_refined(h);
            const double t = (da >= 0.0 ? db : -db) * rcp_refined(fabs(da) + root);
            c = rsq_refined(fma(t, t, 1.0));
            s = t * c;
          }
        }
        rot[i] = make_double2(c, s);
        pq[i] = make_int2(p, q < n ? q : -1);
        if (rlog) rlog[static_cast<int64_t>(nrun) * npairs + i] = make_double2(c, s);
      }
      if (rlog && threadIdx.x == 0) rsteps[nrun] = step;
      ++nrun;
      __syncthreads();
      // the items of a step touch disjoint entries, so within a batch every
      // load is issued before any store (the compiler cannot prove that on its own)
#pragma unroll
      for (int bt = 0; bt < kBatches; ++bt) {
        double2 ra[kA], rb[kA], rv[kV];
        int2 xa[kA], xb[kA], xv[kV];
        double va[kA][4], vv[kV][2];
#pragma unroll
        for (int k = 0; k < kA; ++k) {
          ra[k] = rb[k] = make_double2(1.0, 0.0);
          xa[k] = xb[k] = make_int2(-1, -1);
          if (bi[bt * kA + k] >= 0) {
            ra[k] = rot[bi[bt * kA + k]];
            xa[k] = pq[bi[bt * kA + k]];
            rb[k] = rot[bj[bt * kA + k]];
            xb[k] = pq[bj[bt * kA + k]];
          }
        }
#pragma unroll
        for (int k = 0; k < kV; ++k) {
          rv[k] = make_double2(1.0, 0.0);
          xv[k] = make_int2(-1, -1);
          if (vi[bt * kV + k] >= 0) {
            rv[k] = rot[vi[bt * kV + k]];
            xv[k] = pq[vi[bt * kV + k]];
          }
        }
#pragma unroll
        for (int k = 0; k < kA; ++k) {
          va[k][0] = va[k][1] = va[k][2] = va[k][3] = 0.0;
          const int p_i = xa[k].x, q_i = xa[k].y, p_j = xb[k].x, q_j = xb[k].y;
          if (p_i >= 0 && (ra[k].y != 0.0 || rb[k].y != 0.0)) {
            va[k][0] = A[p_i * lda + p_j];
            if (q_j >= 0) va[k][1] = A[p_i * lda + q_j];
            if (q_i >= 0) va[k][2] = A[q_i * lda + p_j];
            if (q_i >= 0 && q_j >= 0) va[k][3] = A[q_i * lda + q_j];
          }
        }
#pragma unroll
        for (int k = 0; k < kV; ++k) {
          vv[k][0] = vv[k][1] = 0.0;
          if (xv[k].x >= 0 && rv[k].y != 0.0) {
            vv[k][0] = V[vr[bt * kV + k] * ldv + xv[k].x];
            vv[k][1] = V[vr[bt * kV + k] * ldv + xv[k].y];
          }
        }
#pragma unroll
        for (int k = 0; k < kA; ++k) {
          const int p_i = xa[k].x, q_i = xa[k].y, p_j = xb[k].x, q_j = xb[k].y;
          const double ci = ra[k].x, si = ra[k].y, cj = rb[k].x, sj = rb[k].y;
          if (p_i >= 0 && (si != 0.0 || sj != 0.0)) {
            const double a = va[k][0], b = va[k][1], c = va[k][2], d = va[k][3];
            const double a1 = ci * a - si * c, b1 = ci * b - si * d;
            const double c1 = si * a + ci * c, d1 = si * b + ci * d;
            const double a2 = cj * a1 - sj * b1;
            double b2 = sj * a1 + cj * b1;
            double c2 = cj * c1 - sj * d1;
            const double d2 = sj * c1 + cj * d1;
            if (bi[bt * kA + k] == bj[bt * kA + k] && si != 0.0) {  // the rotated pair's own coupling is annihilated
              b2 = 0.0;
              c2 = 0.0;
            }
            A[p_i * lda + p_j] = a2;
            if (q_j >= 0) A[p_i * lda + q_j] = b2;
            if (q_i >= 0) A[q_i * lda + p_j] = c2;
            if (q_i >= 0 && q_j >= 0) A[q_i * lda + q_j] = d2;
          }
        }
#pragma unroll
        for (int k = 0; k < kV; ++k) {
          if (xv[k].x >= 0 && rv[k].y != 0.0) {
            const double c = rv[k].x, s = rv[k].y, vp = vv[k][0], vq = vv[k][1];
            V[vr[bt * kV + k] * ldv + xv[k].x] = c * vp - s * vq;
            V[vr[bt * kV + k] * ldv + xv[k].y] = s * vp + c * vq;
          }
        }
      }
      __syncthreads();
    }
  }
  if (rlog && threadIdx.x == 0) *rcount = nrun;
  __syncthreads();
  return sweep;
}




// Order eigenpairs by decreasing eigenvalue (ties keep the lower index):
// evals[i] <- sorted diagonal of A, perm[i] <- source column.
__device__ inline void blk_sort_desc(const double* A, int lda, int n, double* evals, int* perm) {
  // rank sort: element i goes after every larger value and after equal
  // values of lower index (a NaN counts as -inf, so the ranks stay a permutation)
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = A[i * lda + i];
    const double key = isnan(v) ? -INFINITY : v;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      double u = A[j * lda + j];
      u = isnan(u) ? -INFINITY : u;
      rank += (u > key || (u == key && j < i)) ? 1 : 0;
    }
    evals[rank] = v;
    perm[rank] = i;
  }
  __syncthreads();
}

}  // namespace tpo
