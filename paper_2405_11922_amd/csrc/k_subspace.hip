// Randomized subspace iteration on a small symmetric FP64 matrix A (N x N:
// the attribute Gram C = X^T X of the reduction, or K = R^T R of
// RandomizedSVD), with the basis re-orthonormalised by Cholesky QR after
// every product (Halko et al., Algorithms 4.4 and 5.1, as used by
// Algorithm 2 and by the attribute reduction of Section 3.2.1).
//
// With P_i = A Q_{i-1} and L_i = chol(P_i^T P_i), Q_i = P_i L_i^{-T}.  The
// product of the next step is re-associated so that Q_i is never formed:
//   P_{i+1} = A Q_i = (A P_i) L_i^{-T}.
// One step is one distributed kernel (a workgroup per 16 rows of P, one wave
// per 16-column tile, FP64 MFMA) that forms its rows of P_{i+1} and their
// contribution to the Gram P_{i+1}^T P_{i+1}; one single-workgroup kernel
// adds the contributions in a fixed order and factors the Gram (blocked
// Cholesky with the inverse L^{-1} kept).  The last step also writes Q.
#include "blk_chol16.hpp"
#include "dev_common.hpp"
#include "tpo_internal.hpp"

namespace tpo {

constexpr int kSiBatch = 16;  // partials loaded per batch before they are summed

// Y = A[rows] Pp;  Pn[rows] = Y Li^T (or Y when Li is null);  the lower
// 16 x 16 tiles of Pn[rows]^T Pn[rows] to part[blockIdx];  when Qout is
// given, Qout[rows] = Pp[rows] Li^T (or Pp[rows]).
// Li is l x l lower (row-major, ld l).  part holds (16 NB)^2 doubles per
// block.  NB = number of 16-column tiles (l <= 16 NB <= 80).
template <int NB>
__global__ void __launch_bounds__(64 * NB)
k_si_step(const double* __restrict__ A, int N, const double* __restrict__ Pp, int l, const double* __restrict__ Li,
          double* __restrict__ Pn, double* __restrict__ part, double* __restrict__ Qout) {
  constexpr int NP = 16 * NB;
  constexpr int LD = NP + 1;
  __shared__ double Ys[16 * LD];
  __shared__ double Ps[16 * LD];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int rt = blockIdx.x;
  const int arow = 16 * rt + i16;
  const bool arow_ok = arow < N;
  const int col = 16 * w + i16;
  const bool col_ok = col < l;
  // Y tile (rows 16 rt.., columns 16 w..) = sum_k A[arow][k] Pp[k][col], in
  // four interleaved partial sums (independent MFMA chains) added at the end
  v4d_t acc4[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc4[c] = v4d_t{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < N; k0 += 128) {
    double av[32], bv[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int k = k0 + 4 * u + kq;
      av[u] = (arow_ok && k < N) ? A[static_cast<int64_t>(arow) * N + k] : 0.0;
      bv[u] = (col_ok && k < N) ? Pp[static_cast<int64_t>(k) * l + col] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 32; ++u)
      acc4[u & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc4[u & 3], 0, 0, 0);
  }
  const v4d_t acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
#pragma unroll
  for (int v = 0; v < 4; ++v) Ys[(4 * v + kq) * LD + col] = acc[v];
  __syncthreads();
  // P tile = Y Li^T over the k tiles kt <= w (Li lower)
  v4d_t pn = acc;
  if (Li) {
    pn = v4d_t{0.0, 0.0, 0.0, 0.0};
    for (int kt = 0; kt <= w; ++kt) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = 16 * kt + 4 * u + kq;
        const double a = Ys[i16 * LD + kk];
        const double b = (col_ok && kk < l) ? Li[col * l + kk] : 0.0;  // Li^T[kk][col]
        pn = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, pn, 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 16 * rt + 4 * v + kq;
    const bool ok = r < N && col_ok;
    if (ok) Pn[static_cast<int64_t>(r) * l + col] = pn[v];
    Ps[(4 * v + kq) * LD + col] = ok ? pn[v] : 0.0;
  }
  if (Qout) {
    v4d_t qa = {0.0, 0.0, 0.0, 0.0};
    if (Li) {
      for (int kt = 0; kt <= w; ++kt) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = 16 * kt + 4 * u + kq;
          const double a = (arow_ok && kk < l) ? Pp[static_cast<int64_t>(arow) * l + kk] : 0.0;
          const double b = (col_ok && kk < l) ? Li[col * l + kk] : 0.0;
          qa = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, qa, 0, 0, 0);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * rt + 4 * v + kq;
        if (r < N && col_ok) Qout[static_cast<int64_t>(r) * l + col] = qa[v];
      }
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * rt + 4 * v + kq;
        if (r < N && col_ok) Qout[static_cast<int64_t>(r) * l + col] = Pp[static_cast<int64_t>(r) * l + col];
      }
    }
  }
  if (!part) return;
  __syncthreads();
  // lower tiles (ta >= tb) of Ps^T Ps, summed over the 16 rows
  double* out = part + static_cast<int64_t>(blockIdx.x) * NP * NP;
  for (int t = w; t < NB * (NB + 1) / 2; t += NB) {
    int ta = 0, rem = t;
    while (rem > ta) {
      rem -= ta + 1;
      ++ta;
    }
    const int tb = rem;  // 0 <= tb <= ta
    v4d_t g = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = 4 * u + kq;
      g = __builtin_amdgcn_mfma_f64_16x16x4f64(Ps[r * LD + 16 * ta + i16], Ps[r * LD + 16 * tb + i16], g, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(16 * ta + 4 * v + kq) * NP + 16 * tb + i16] = g[v];
  }
}

// G = sum of the nparts lower-tile partials (fixed order), identity on the
// padding beyond l; L = chol(G); Li = L^{-1} (l x l, zero above the diagonal).
__global__ void __launch_bounds__(1024)
k_si_chol(const double* __restrict__ part, int nparts, int l, double* __restrict__ Li,
          int32_t* __restrict__ err_bits) {
  __shared__ double G[kC16Max * kC16Ld];
  __shared__ double L[kC16Max * kC16Ld];
  __shared__ double scratch[4 * 256];
  __shared__ int flag;
  const int nb = (l + 15) / 16;
  const int np = 16 * nb;
  // every load is issued before the (fixed-order) sums: the partials come
  // from other XCDs' writes, so each load pays the full memory latency
  for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
    const int i = e / np, j = e - (e / np) * np;
    const bool in = i / 16 >= j / 16 && i < l && j < l;
    double s = 0.0;
    for (int b0 = 0; b0 < nparts; b0 += kSiBatch) {
      double v[kSiBatch];
#pragma unroll
      for (int b = 0; b < kSiBatch; ++b)
        v[b] = (in && b0 + b < nparts) ? part[static_cast<int64_t>(b0 + b) * np * np + e] : 0.0;
#pragma unroll
      for (int b = 0; b < kSiBatch; ++b) s += v[b];
    }
    if (!in) s = (i / 16 >= j / 16 && i == j) ? 1.0 : 0.0;
    G[i * kC16Ld + j] = s;
  }
  __syncthreads();
  const bool ok = blk_chol_inv16(G, L, kC16Ld, nb, scratch, &flag);
  if (!ok && threadIdx.x == 0) atomicOr(err_bits, 16);
  for (int e = threadIdx.x; e < l * l; e += blockDim.x) {
    const int i = e / l, j = e - (e / l) * l;
    double v = (i == j) ? 1.0 : 0.0;  // identity after a breakdown keeps later values finite
    if (ok) v = j <= i ? L[i * kC16Ld + j] : 0.0;
    Li[e] = v;
  }
}

template <int NB>
static void si_run(const double* A, int N, const double* omega, int l, int n_orth, double* pa, double* pb,
                   double* li, double* part, double* m_out, double* p_out, int32_t* err_bits, hipStream_t s) {
  const int nrt = (N + 15) / 16;
  // the first product uses omega directly
  const double* prev = omega;
  const double* prev_li = nullptr;
  double* cur = pa;
  for (int i = 0; i < n_orth; ++i) {
    hipLaunchKernelGGL((k_si_step<NB>), dim3(nrt), dim3(64 * NB), 0, s, A, N, prev, l, prev_li, cur, part,
                       static_cast<double*>(nullptr));
    TPO_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_si_chol, dim3(1), dim3(1024), 0, s, part, nrt, l, li, err_bits);
    TPO_LAUNCH_CHECK();
    prev = cur;
    prev_li = li;
    cur = (cur == pa) ? pb : pa;
  }
  // P = A M and M itself for the last basis M (omega when n_orth = 0)
  hipLaunchKernelGGL((k_si_step<NB>), dim3(nrt), dim3(64 * NB), 0, s, A, N, prev, l, prev_li, p_out,
                     static_cast<double*>(nullptr), m_out);
  TPO_LAUNCH_CHECK();
}

void subspace_iterate(const double* A, int N, const double* omega, int l, int n_orth, double* pa, double* pb,
                      double* li, double* part, double* m_out, double* p_out, int32_t* err_bits, hipStream_t s) {
  switch ((l + 15) / 16) {
    case 1: si_run<1>(A, N, omega, l, n_orth, pa, pb, li, part, m_out, p_out, err_bits, s); break;
    case 2: si_run<2>(A, N, omega, l, n_orth, pa, pb, li, part, m_out, p_out, err_bits, s); break;
    case 3: si_run<3>(A, N, omega, l, n_orth, pa, pb, li, part, m_out, p_out, err_bits, s); break;
    case 4: si_run<4>(A, N, omega, l, n_orth, pa, pb, li, part, m_out, p_out, err_bits, s); break;
    case 5: si_run<5>(A, N, omega, l, n_orth, pa, pb, li, part, m_out, p_out, err_bits, s); break;
    default: throw std::runtime_error("subspace_iterate: width beyond the LDS path");
  }
}

size_t subspace_part_doubles(int N, int l) {
  const size_t np = 16 * static_cast<size_t>((l + 15) / 16);
  return static_cast<size_t>((N + 15) / 16) * np * np;
}

}  // namespace tpo
