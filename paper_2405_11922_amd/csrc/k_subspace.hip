// Randomized subspace iteration on a small symmetric FP64 matrix A (N x N:
// the attribute Gram C = X^T X of the reduction, or K = R^T R of
// RandomizedSVD), with the basis re-orthonormalised by Cholesky QR after
// every product (Halko et al., Algorithms 4.4 and 5.1, as used by
// Algorithm 2 and by the attribute reduction of Section 3.2.1).
//
// With P_i = A Q_{i-1} and L_i = chol(P_i^T P_i), Q_i = P_i L_i^{-T}.  The
// product of the next step is re-associated so that Q_i is never formed:
//   P_{i+1} = A Q_i = (A P_i) L_i^{-T}.
// The whole iteration is one kernel with grid barriers.  Each workgroup owns blocks
// of 16 rows of P (one wave per 16-column tile, FP64 MFMA) and adds their
// contribution to the Gram P^T P into its own partial; after a grid barrier
// the workgroups add the partials entry by entry in a fixed order; after a
// second barrier every workgroup reads the Gram and factors it in its own
// LDS (blocked Cholesky with L^{-1} formed in place), so that the next
// product has L^{-1} at hand without another launch.  All workgroups factor
// the same sums in the same order and so hold the same L^{-1}.
#include <mutex>

#include "blk_chol16.hpp"
#include "dev_common.hpp"
#include "tpo_internal.hpp"

namespace tpo {

constexpr int kSiThreads = 512;  // 8 waves: one per 16-column tile, and one per tile below the diagonal (nb <= 8)
constexpr int kSiBatch = 16;      // loads in flight per lane before they are used (A from global memory)
constexpr int kSiWideBatch = 32;  // the same with A's row tile in LDS
constexpr int kSiMaxGrid = 256;  // and at most the device's CU count
constexpr size_t kLdsBytes = 160 * 1024;

// Grid-wide barrier.  The grid has at most one workgroup per CU (and at most
// kSiMaxGrid), so every workgroup is resident once the CUs it waits for are
// free; the launch does not depend on any later work.  bar[0] counts
// arrivals, bar[1] is the generation: the last workgroup to arrive resets
// the count and advances the generation, the others wait for it to change.
// Each workgroup's writes are released before it arrives and the others'
// acquired after it leaves.  A wait longer than kSiBarrierTicks sets bit 64
// of err_bits and goes on, so that the kernel always ends.
constexpr uint64_t kSiBarrierTicks = 200000000;  // 2 s of the 100 MHz constant clock

__device__ __forceinline__ void grid_barrier(unsigned* bar, int32_t* err_bits) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == gridDim.x - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > kSiBarrierTicks) {
          atomicOr(err_bits, 64);
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
}

__global__ void k_si_bar_reset(unsigned* bar) {
  if (threadIdx.x < 2) bar[threadIdx.x] = 0u;
}

// One product's K loop for this lane's 16 x 16 tile of Y = A[rows] P with
// P^T (l x N) in global memory: lane (i16, kq) takes the contiguous k range
// k0 + kq KB .. k0 + kq KB + KB - 1 of each block of 4 KB values of k, so its
// loads of P^T (and of A) are runs of consecutive addresses from one base.
// Lanes outside the matrix read row or column 0 instead; their results are
// never stored.
template <int KB, bool TAIL>
__device__ __forceinline__ void si_kbatch(const double* __restrict__ A, const double* As, int N,
                                          const double* __restrict__ Pt, int colc, int arowc, int i16, int kq, int k0,
                                          v4d_t* acc4) {
  const int kbase = k0 + kq * KB;
  const double* pt = Pt + static_cast<int64_t>(colc) * N + kbase;
  double bv[KB];
#pragma unroll
  for (int u = 0; u < KB; ++u) bv[u] = (!TAIL || kbase + u < N) ? pt[u] : 0.0;
  if (As) {
    const double* ar = As + i16 * (N + 1) + kbase;
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const double a = (!TAIL || kbase + u < N) ? ar[u] : 0.0;
      acc4[u & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[u], acc4[u & 3], 0, 0, 0);
    }
  } else {
    const double* ag = A + static_cast<int64_t>(arowc) * N + kbase;
    double av[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) av[u] = (!TAIL || kbase + u < N) ? ag[u] : 0.0;
#pragma unroll
    for (int u = 0; u < KB; ++u) acc4[u & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc4[u & 3], 0, 0, 0);
  }
}

template <int KB>
__device__ __forceinline__ void si_kloop(const double* __restrict__ A, const double* As, int N,
                                         const double* __restrict__ Pt, int colc, int arowc, int i16, int kq,
                                         v4d_t* acc4) {
  int k0 = 0;
  for (; k0 + 4 * KB <= N; k0 += 4 * KB) si_kbatch<KB, false>(A, As, N, Pt, colc, arowc, i16, kq, k0, acc4);
  if (k0 < N) si_kbatch<KB, true>(A, As, N, Pt, colc, arowc, i16, kq, k0, acc4);
}

// This workgroup's rows 16 rt .. 16 rt + 15, with P given as Pt = P^T (l x N):
//   Y = A[rows] P,  Pn[rows] = Y Li^T (Y when Li is null),
//   Qout[rows] = P[rows] Li^T (P[rows] when Li is null) when Qout is given,
//   gpart (NP x NP, lower tiles) = Pn[rows]^T Pn[rows] (gfirst) or += it, when
//   gpart is given (wave w: tiles w, w + 8, ...; the same lanes write and
//   re-read each entry).
// Pn is written as Pn^T (l x N) unless pn_rowmajor (N x l); Qout is N x l.
// As: the row tile of A in LDS (row stride N + 1), or null to read A.
// Li: LDS, lower, leading dimension ldl.  Ys: 16 x (16 NB + 1) doubles of LDS.
template <int NB>
__device__ __forceinline__ void si_rows(const double* __restrict__ A, const double* As, int N,
                                        const double* __restrict__ Pt, int l, const double* Li, int ldl,
                                        double* __restrict__ Pn, bool pn_rowmajor, double* __restrict__ Qout,
                                        double* Ys, int rt, double* __restrict__ gpart, bool gfirst) {
  constexpr int NP = 16 * NB;
  constexpr int LD = NP + 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int arow = 16 * rt + i16;
  const bool arow_ok = arow < N;
  const int col = 16 * w + i16;
  const bool col_ok = w < NB && col < l;
  v4d_t acc = {0.0, 0.0, 0.0, 0.0};
  if (w < NB) {
    // four interleaved partial sums (independent MFMA chains)
    v4d_t acc4[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc4[c] = v4d_t{0.0, 0.0, 0.0, 0.0};
    const int colc = col_ok ? col : 0, arowc = arow_ok ? arow : 0;
    if (!As)
      si_kloop<kSiBatch>(A, nullptr, N, Pt, colc, arowc, i16, kq, acc4);
    else if (N >= 4 * kSiWideBatch)
      si_kloop<kSiWideBatch>(A, As, N, Pt, colc, arowc, i16, kq, acc4);
    else if (N >= 2 * kSiWideBatch)
      si_kloop<kSiWideBatch / 2>(A, As, N, Pt, colc, arowc, i16, kq, acc4);
    else
      si_kloop<kSiWideBatch / 4>(A, As, N, Pt, colc, arowc, i16, kq, acc4);
    acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
#pragma unroll
    for (int v = 0; v < 4; ++v) Ys[(4 * v + kq) * LD + col] = acc[v];
  }
  __syncthreads();
  v4d_t pn = acc;
  if (w < NB) {
    if (Li) {
      pn = v4d_t{0.0, 0.0, 0.0, 0.0};
      for (int kt = 0; kt <= w; ++kt) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = 16 * kt + 4 * u + kq;
          const double a = Ys[i16 * LD + kk];
          const double b = (col_ok && kk < l) ? Li[col * ldl + kk] : 0.0;  // Li^T[kk][col]
          pn = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, pn, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * rt + 4 * v + kq;
      if (r < N && col_ok) {
        if (pn_rowmajor)
          Pn[static_cast<int64_t>(r) * l + col] = pn[v];
        else
          Pn[static_cast<int64_t>(col) * N + r] = pn[v];
      }
    }
    if (Qout) {
      v4d_t qa = {0.0, 0.0, 0.0, 0.0};
      if (Li) {
        for (int kt = 0; kt <= w; ++kt) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kk = 16 * kt + 4 * u + kq;
            const double a = (arow_ok && kk < l) ? Pt[static_cast<int64_t>(kk) * N + arow] : 0.0;
            const double b = (col_ok && kk < l) ? Li[col * ldl + kk] : 0.0;
            qa = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, qa, 0, 0, 0);
          }
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * rt + 4 * v + kq;
          qa[v] = (r < N && col_ok) ? Pt[static_cast<int64_t>(col) * N + r] : 0.0;
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * rt + 4 * v + kq;
        if (r < N && col_ok) Qout[static_cast<int64_t>(r) * l + col] = qa[v];
      }
    }
  }
  if (!gpart) return;
  __syncthreads();  // every wave is done with Y
  if (w < NB) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * rt + 4 * v + kq;
      Ys[(4 * v + kq) * LD + col] = (r < N && col_ok) ? pn[v] : 0.0;
    }
  }
  __syncthreads();
  constexpr int NT = NB * (NB + 1) / 2;
#pragma unroll
  for (int idx = 0; idx < (NT + kSiThreads / 64 - 1) / (kSiThreads / 64); ++idx) {
    const int t = w + idx * (kSiThreads / 64);
    if (t >= NT) break;
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
      g = __builtin_amdgcn_mfma_f64_16x16x4f64(Ys[r * LD + 16 * ta + i16], Ys[r * LD + 16 * tb + i16], g, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double* o = gpart + (16 * ta + 4 * v + kq) * NP + 16 * tb + i16;
      *o = gfirst ? g[v] : *o + g[v];
    }
  }
  __syncthreads();  // Ys is free again
}

// n_orth orthonormalisations from omega, then P = A M with M the last basis
// (omega when n_orth = 0): m_out = M, p_out = P.  part: gridDim.x partial
// Grams (NP x NP, lower tiles); gsum: NP x NP.
template <int NB>
__global__ void __launch_bounds__(kSiThreads)
k_si_fused(const double* __restrict__ A, int N, const double* __restrict__ omega, int l, int n_orth,
           double* __restrict__ pa, double* __restrict__ pb, double* __restrict__ part, double* __restrict__ gsum,
           unsigned* __restrict__ bar, double* __restrict__ m_out, double* __restrict__ p_out,
           int32_t* __restrict__ err_bits, int a_lds) {
  constexpr int NP = 16 * NB;
  constexpr int LD = NP + 1;
  __shared__ double G[NP * LD];  // Gram, factor and inverse (lower tiles)
  __shared__ double Ys[16 * LD];  // one row block of Y / P; the factorisation's scratch tiles
  __shared__ double dinv[NP];
  __shared__ int flag;
  extern __shared__ double As_dyn[];  // a_lds: rows 16 b .. 16 b + 15 of A (stride N + 1), b = blockIdx.x
  const int nrt = (N + 15) / 16;
  const double* prev = omega;
  double* cur = pa;
  bool have_li = false;
  const double* As = nullptr;
  if (a_lds) {  // one row tile per workgroup: its rows of A stay in LDS for every product
    for (int e = threadIdx.x; e < 16 * N; e += kSiThreads) {
      const int r = e / N, c = e - (e / N) * N;
      const int row = 16 * blockIdx.x + r;
      As_dyn[r * (N + 1) + c] = row < N ? A[static_cast<int64_t>(row) * N + c] : 0.0;
    }
    __syncthreads();
    As = As_dyn;
  }
  // omega^T into pb: the products read P^T
  for (int e = blockIdx.x * kSiThreads + threadIdx.x; e < N * l; e += gridDim.x * kSiThreads) {
    const int r = e / l, c = e - (e / l) * l;
    pb[static_cast<int64_t>(c) * N + r] = omega[e];
  }
  grid_barrier(bar, err_bits);
  prev = pb;
  for (int it = 0; it <= n_orth; ++it) {
    const bool last = it == n_orth;
    double* mypart = part + static_cast<int64_t>(blockIdx.x) * NP * NP;
    for (int rt = blockIdx.x; rt < nrt; rt += gridDim.x)
      si_rows<NB>(A, As, N, prev, l, have_li ? G : nullptr, LD, last ? p_out : cur, last, last ? m_out : nullptr,
                  Ys, rt, last ? nullptr : mypart, rt == static_cast<int>(blockIdx.x));
    if (last) break;
    grid_barrier(bar, err_bits);
    // Gram = sum of the partials, entry by entry in block order
    const int nparts = gridDim.x;
    for (int e = blockIdx.x * kSiThreads + threadIdx.x; e < NP * NP; e += gridDim.x * kSiThreads) {
      const int i = e / NP, j = e - (e / NP) * NP;
      if (i / 16 < j / 16) continue;
      double s = 0.0;
      for (int b0 = 0; b0 < nparts; b0 += kSiBatch) {
        double v[kSiBatch];
#pragma unroll
        for (int b = 0; b < kSiBatch; ++b)
          v[b] = b0 + b < nparts ? part[static_cast<int64_t>(b0 + b) * NP * NP + e] : 0.0;
#pragma unroll
        for (int b = 0; b < kSiBatch; ++b) s += v[b];
      }
      gsum[e] = s;
    }
    grid_barrier(bar, err_bits);
    // every workgroup: L = chol(Gram), L^{-1} in place; identity on the
    // padding beyond l, and after a breakdown (keeps later values finite)
#pragma unroll 4
    for (int e = threadIdx.x; e < NP * NP; e += kSiThreads) {
      const int i = e / NP, j = e - (e / NP) * NP;
      double v = 0.0;
      if (i / 16 >= j / 16) v = (i < l && j < l) ? gsum[e] : (i == j ? 1.0 : 0.0);
      G[i * LD + j] = v;
    }
    __syncthreads();
    if (!blk_chol_inv16_inplace(G, LD, NB, Ys, dinv, &flag)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err_bits, 16);
      for (int e = threadIdx.x; e < NP * NP; e += kSiThreads) {
        const int i = e / NP, j = e - (e / NP) * NP;
        G[i * LD + j] = i == j ? 1.0 : 0.0;
      }
      __syncthreads();
    }
    have_li = true;
    prev = cur;
    cur = (cur == pa) ? pb : pa;
  }
}

template <int NB>
static void si_run(const double* A, int N, const double* omega, int l, int n_orth, double* pa, double* pb,
                   double* gsum, double* part, unsigned* bar, double* m_out, double* p_out, int32_t* err_bits,
                   hipStream_t s) {
  const int nrt = (N + 15) / 16;
  // one workgroup per CU at most, so that the whole grid is resident
  static const int cus = [] {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
      c = 64;
    return c;
  }();
  const int grid = std::min({nrt, kSiMaxGrid, cus});
  constexpr size_t kStatic = (16 * NB * (16 * NB + 1) + 16 * (16 * NB + 1) + 16 * NB) * sizeof(double) + 64;
  const size_t a_bytes = static_cast<size_t>(16) * (N + 1) * sizeof(double);
  const int a_lds = nrt <= grid && kStatic + a_bytes <= kLdsBytes ? 1 : 0;
  const size_t dyn = a_lds ? a_bytes : 0;
  // the kernel's dynamic-LDS limit is a process-wide attribute: set once, to
  // the most any launch can ask for, so that concurrent callers (serving
  // threads) never see a smaller value set by another thread between their
  // own set and launch
  static std::once_flag once;
  std::call_once(once, [] {
    TPO_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_si_fused<NB>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      static_cast<int>(kLdsBytes - kStatic)));
  });
  hipLaunchKernelGGL(k_si_bar_reset, dim3(1), dim3(64), 0, s, bar);
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_si_fused<NB>), dim3(grid), dim3(kSiThreads), dyn, s, A, N, omega, l, n_orth, pa, pb, part,
                     gsum, bar, m_out, p_out, err_bits, a_lds);
  TPO_LAUNCH_CHECK();
}

void subspace_iterate(const double* A, int N, const double* omega, int l, int n_orth, double* pa, double* pb,
                      double* gsum, double* part, unsigned* bar, double* m_out, double* p_out, int32_t* err_bits,
                      hipStream_t s) {
  switch ((l + 15) / 16) {
    case 1: si_run<1>(A, N, omega, l, n_orth, pa, pb, gsum, part, bar, m_out, p_out, err_bits, s); break;
    case 2: si_run<2>(A, N, omega, l, n_orth, pa, pb, gsum, part, bar, m_out, p_out, err_bits, s); break;
    case 3: si_run<3>(A, N, omega, l, n_orth, pa, pb, gsum, part, bar, m_out, p_out, err_bits, s); break;
    case 4: si_run<4>(A, N, omega, l, n_orth, pa, pb, gsum, part, bar, m_out, p_out, err_bits, s); break;
    case 5: si_run<5>(A, N, omega, l, n_orth, pa, pb, gsum, part, bar, m_out, p_out, err_bits, s); break;
    case 6: si_run<6>(A, N, omega, l, n_orth, pa, pb, gsum, part, bar, m_out, p_out, err_bits, s); break;
    case 7: si_run<7>(A, N, omega, l, n_orth, pa, pb, gsum, part, bar, m_out, p_out, err_bits, s); break;
    case 8: si_run<8>(A, N, omega, l, n_orth, pa, pb, gsum, part, bar, m_out, p_out, err_bits, s); break;
    default: throw std::runtime_error("subspace_iterate: width beyond 128");
  }
}

size_t subspace_part_doubles(int N, int l) {
  const size_t np = 16 * static_cast<size_t>((l + 15) / 16);
  return static_cast<size_t>(std::min((N + 15) / 16, kSiMaxGrid)) * np * np;
}

size_t subspace_gsum_doubles(int l) {
  const size_t np = 16 * static_cast<size_t>((l + 15) / 16);
  return np * np;
}

}  // namespace tpo
