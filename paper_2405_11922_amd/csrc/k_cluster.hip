// Greedy orthogonal NMF (Algorithm 2), NCI generation (Algorithm 3)
// and the k-ABGC objective (Eq. obj1).
//
// Row passes stream R (n x 2d) once per ONMF round: each row's new Upsilon
// entries depend only on that row, R H and two k x k matrices, and the same
// pass accumulates R^T Upsilon and Upsilon^T Upsilon for the next round's H
// update (Eq. update-Q).  Sums grouped by cluster label (NCI's Phi = Ups^T Y
// and the cluster sums of R in the objective) use 64-bit fixed point so that
// their result does not depend on the order of the atomic additions.
#include <algorithm>
#include <type_traits>
#include <mutex>

#include "blk_linalg.hpp"
#include "dev_common.hpp"
#include "tpo_internal.hpp"

namespace tpo {

enum RowPassMode { kProject = 0, kOnmf = 1 };

typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef double v4d_t __attribute__((ext_vector_type(4)));

// Row passes on FP32 MFMA (v_mfma_f32_16x16x4f32: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16], its v-th result is
// D[4 (l / 16) + v][l % 16]).
//
// A workgroup of eight (or four) waves walks slabs of 64 (or 32) rows of R (rows padded
// to TD = 16 JT columns, zeros beyond 2d), with the next slab's loads in
// flight while the current one is processed.  The waves split the 16-row
// tiles and the 16-column output tiles of the slab:
//   kProject: O = R S            (Gamma; also written as Upsilon)
//   kOnmf:    P = R H, Q = U A,  O = U * sqrt(P / Q)   (Eq. update-Y; a zero
//             denominator keeps U, a negative ratio gives 0)
// Which contraction index an MFMA's four depth slots stand for is free as
// long as both operands agree: the j-th of four consecutive MFMAs gives slot
// q the index 16 m + 4 q + j, so a lane's four A values are adjacent in a row
// of the slab and its four B values adjacent in a row of S^T (or A^T), and
// each comes in with one 16-byte LDS read.  A wave reads its slab rows once
// for all its output tiles.  Every wave first forms all its P and Q tiles in
// registers; after a barrier O replaces U in the same LDS slab, so one slab
// buffer serves both.  Then the waves accumulate R^T O (2d x k) and the upper
// triangle of the symmetric O^T O (k x k), tiles dealt round-robin from one
// list, in FP32 registers over the workgroup's rows; the totals are written as
// FP64 partials (both halves of O^T O).  S^T (or H^T) and A^T stay in LDS for
// the whole pass when they fit.
constexpr int kRpRows = 64;
// Waves per workgroup: eight for k in 65..128 with 2d <= 128, where a
// workgroup of four could run only one wave per SIMD (S and A fill the LDS);
// four otherwise (two or more such workgroups share a CU, and for 2d = 256
// with k > 64 the registers would not fit two waves a SIMD).
__host__ __device__ constexpr int rp_waves(int jt, int kt) { return (kt >= 5 && jt * kt <= 64) ? 8 : 4; }
// Waves per SIMD the registers must allow: two, except where a workgroup of
// four carries 2d >= 128 with k in 33..64 (its 64-row slabs need more than
// half a SIMD's registers) or 2d = 256 with k > 64.
__host__ __device__ constexpr int rp_occupancy(int jt, int kt) {
  return (jt * kt > 64 || (kt == 4 && jt >= 8)) ? 1 : 2;
}

template <int MODE, int JT, int KT>
__global__ void __launch_bounds__(64 * rp_waves(JT, KT)) __attribute__((amdgpu_waves_per_eu(rp_occupancy(JT, KT))))
k_rowpass_mfma(const float* __restrict__ R, int64_t n, int twod, int k, const float* __restrict__ Sm,
               const float* __restrict__ A32, float* __restrict__ U, float* __restrict__ out,
               float* __restrict__ out2, int rows_per_block, double* __restrict__ part,
               DevStatus* __restrict__ st) {
  constexpr int kRpWaves = rp_waves(JT, KT), kRpThreads = 64 * kRpWaves;
  constexpr int TD = 16 * JT, KP = 16 * KT;
  // row strides of the slabs and of S^T, A^T: 4 floats past a multiple of 16,
  // so the 16-byte reads of 8 consecutive lanes fall in distinct banks
  constexpr int RS = TD + 4, OS = KP + 4, SS = TD + 4, AS = KP + 4;
  // tiles of R^T O and of the upper triangle of O^T O, each list dealt
  // round-robin over the waves
  constexpr int NT1 = JT * KT, NT2 = KT * (KT + 1) / 2;
  constexpr int NQ1 = (NT1 + kRpWaves - 1) / kRpWaves, NQ2 = (NT2 + kRpWaves - 1) / kRpWaves, NQ = NQ1 + NQ2;
  constexpr int LDS_CAP = 156 * 1024;
  // LDS: the R slab (ROWS x RS), the U/O slab (ROWS x OS), S^T (KP x SS) and,
  // for kOnmf, A^T (KP x AS) when they fit; slabs of 64 rows, or 32 when 64
  // would not fit.  Operands that do not fit are read from global memory.
  constexpr bool SLDS = KP * SS * 4 <= 72 * 1024;
  constexpr int SFIX = SLDS ? KP * SS : 0;
  constexpr bool ALDS = MODE == kOnmf && 4 * ((kRpRows / 2) * (RS + OS) + SFIX + KP * AS) <= LDS_CAP;
  constexpr int FIXED = SFIX + (ALDS ? KP * AS : 0);
  // (64-row slabs also only where their prefetch keeps to 32 values of R a
  // thread, and in eight-wave kernels, capped at 256 registers, to 24 of R
  // and U together)
  constexpr bool R64 = 4 * (kRpRows * (RS + OS) + FIXED) <= LDS_CAP && kRpRows * TD / kRpThreads <= 32 &&
                       (kRpWaves < 8 || kRpRows * (TD + KP) / kRpThreads <= 24);
  constexpr int ROWS = R64 ? kRpRows : kRpRows / 2;
  constexpr int RTILES = ROWS / 16, WPR = kRpWaves / RTILES;  // waves per row tile
  constexpr int KTW = (KT + WPR - 1) / WPR;                    // column tiles per wave
  // Splitting one tile pair between two SIMDs: when exactly one wave per row
  // tile has no last tile (KT = 7 over four waves), that wave (the helper)
  // forms the P of the last tile of the wave before it (the owner), which
  // forms only that tile's Q and takes its P from LDS: the SIMDs then carry
  // 208 / 212 MFMAs per slab instead of 240 / 240 with a repeated tile pair.
  constexpr int RLAST = KT - (KTW - 1) * WPR;  // waves per row tile with a last tile
  constexpr bool SPLIT = MODE == kOnmf && KTW >= 2 && RLAST == WPR - 1;
  // slab prefetch: thread tid loads column tid % TD (of U: tid % KP) of
  // slab rows tid / TD + RSTEP u (tid / KP + USTEP u), RPT (UPT) values
  constexpr int RSTEP = kRpThreads / TD, USTEP = kRpThreads / KP;
  constexpr int RPT = ROWS / RSTEP, UPT = (ROWS + USTEP - 1) / USTEP;
  __shared__ __align__(16) float Rt[ROWS * RS];
  __shared__ __align__(16) float Ut[ROWS * OS];
  __shared__ __align__(16) float Ss[SLDS ? KP * SS : 4];  // S^T (or H^T): Ss[c * SS + r] = S[r][c], zero padded
  __shared__ __align__(16) float As[ALDS ? KP * AS : 4];  // A^T (kOnmf): As[c * AS + t] = A[t][c], zero padded
  __shared__ float Pex[SPLIT ? RTILES * 256 : 1];          // the helpers' P tiles, one per row tile
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i16 = lane & 15, kq = lane >> 4;
  if (SLDS)
    for (int e = tid; e < TD * KP; e += kRpThreads) {
      const int r = e / KP, c = e - (e / KP) * KP;
      Ss[c * SS + r] = (r < twod && c < k) ? Sm[r * k + c] : 0.0f;
    }
  if (ALDS)
    for (int e = tid; e < KP * KP; e += kRpThreads) {
      const int r = e / KP, c = e - (e / KP) * KP;
      As[c * AS + r] = (r < k && c < k) ? A32[r * k + c] : 0.0f;
    }
  // B operands of the P and Q tiles: contraction indices 16 m + 4 kq + (0..3)
  // of output column 16 kt + i16
  auto s_frag = [&](int m, int kt) -> v4f_t {
    if (SLDS) return *reinterpret_cast<const v4f_t*>(&Ss[(16 * kt + i16) * SS + 16 * m + 4 * kq]);
    v4f_t b;
    const int c = 16 * kt + i16;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 16 * m + 4 * kq + j;
      b[j] = (r < twod && c < k) ? Sm[r * k + c] : 0.0f;
    }
    return b;
  };
  auto a_frag = [&](int m, int kt) -> v4f_t {
    if (ALDS) return *reinterpret_cast<const v4f_t*>(&As[(16 * kt + i16) * AS + 16 * m + 4 * kq]);
    v4f_t b;
    const int c = 16 * kt + i16;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 16 * m + 4 * kq + j;
      b[j] = (r < k && c < k) ? A32[r * k + c] : 0.0f;
    }
    return b;
  };
  // the q-th tile of the upper triangle of O^T O: its two column tiles
  auto tri_tile = [&](int q, int& ta, int& tb) {
    int t = 0, rem = q;
    while (rem >= KT - t) {
      rem -= KT - t;
      ++t;
    }
    ta = t;
    tb = t + rem;
  };
  v4f_t acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = v4f_t{0.f, 0.f, 0.f, 0.f};
  float mx = 0.0f;
  int hits = 0;
  bool bad = false;
  const int64_t rb = static_cast<int64_t>(blockIdx.x) * rows_per_block;
  const int64_t re = min(n, rb + rows_per_block);
  float rr_[RPT], uu_[UPT];
  const int rrow = tid / TD, rcol = tid - (tid / TD) * TD;
  const int urow = tid / KP, ucol = tid - (tid / KP) * KP;
  const bool uact = urow < USTEP;  // threads beyond USTEP whole rows of KP idle
  auto fetch = [&](int64_t r0) {
    const int left = static_cast<int>(min<int64_t>(re - r0, ROWS));  // rows of this slab that exist
    const float* rs = R + r0 * twod;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int rr = rrow + RSTEP * u;
      rr_[u] = (rr < left && rcol < twod) ? rs[rr * twod + rcol] : 0.0f;
    }
    if (MODE == kOnmf) {
      const float* us = U + r0 * k;
#pragma unroll
      for (int u = 0; u < UPT; ++u) {
        const int rr = urow + USTEP * u;
        uu_[u] = (uact && rr < left && ucol < k) ? us[rr * k + ucol] : 0.0f;
      }
    }
  };
  if (rb < re) fetch(rb);
  const int rw = 16 * (w % RTILES);  // this wave's rows in the slab
  const int kt0 = w / RTILES;         // its column tiles: kt0, kt0 + WPR, ...
  for (int64_t r0 = rb; r0 < re; r0 += ROWS) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) Rt[(rrow + RSTEP * u) * RS + rcol] = rr_[u];
    if (MODE == kOnmf) {
#pragma unroll
      for (int u = 0; u < UPT; ++u) {
        const int rr = urow + USTEP * u;
        if (uact && rr < ROWS) Ut[rr * OS + ucol] = uu_[u];
      }
    }
    __syncthreads();
    if (r0 + ROWS < re) fetch(r0 + ROWS);
    // P (and Q) of every owned tile, in registers
    v4f_t pv[KTW], qv[KTW];
#pragma unroll
    for (int i = 0; i < KTW; ++i) {
      pv[i] = v4f_t{0.f, 0.f, 0.f, 0.f};
      qv[i] = v4f_t{0.f, 0.f, 0.f, 0.f};
    }
    // a wave with fewer than KTW tiles repeats its last one (the copy is
    // discarded), so that no MFMA sits behind a branch
    constexpr bool LIGHT = RPT + UPT <= 24;  // the slab prefetch holds few registers
    constexpr int UNS = SLDS && LIGHT ? 2 : 1, UNA = ALDS && LIGHT ? 2 : 1;
    // P over the first NS of the wave's tiles
    auto p_loop = [&](auto ns_c) {
      constexpr int NS = decltype(ns_c)::value;
#pragma unroll UNS
      for (int m = 0; m < JT; ++m) {
        const v4f_t a = *reinterpret_cast<const v4f_t*>(&Rt[(rw + i16) * RS + 16 * m + 4 * kq]);
        v4f_t b[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) b[i] = s_frag(m, min(kt0 + i * WPR, KT - 1));
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < NS; ++i) pv[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[i][j], pv[i], 0, 0, 0);
      }
    };
    // Q over the first NS of the wave's tiles
    auto q_loop = [&](auto ns_c) {
      constexpr int NS = decltype(ns_c)::value;
#pragma unroll UNA
      for (int m = 0; m < KT; ++m) {
        const v4f_t a = *reinterpret_cast<const v4f_t*>(&Ut[(rw + i16) * OS + 16 * m + 4 * kq]);
        v4f_t b[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) b[i] = a_frag(m, min(kt0 + i * WPR, KT - 1));
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < NS; ++i) qv[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[i][j], qv[i], 0, 0, 0);
      }
    };
    const bool owner = SPLIT && kt0 == RLAST - 1, helper = SPLIT && kt0 == RLAST;  // wave-uniform
    constexpr int KTS = SPLIT ? KTW - 1 : KTW;  // tiles of the owner's P and the helper's Q
    if (owner)
      p_loop(std::integral_constant<int, KTS>{});
    else
      p_loop(std::integral_constant<int, KTW>{});
    if (MODE == kOnmf) {
      if (helper) {
        // the owner's last tile is this wave's repeated slot: hand its P over
#pragma unroll
        for (int v = 0; v < 4; ++v) Pex[(rw / 16) * 256 + (4 * kq + v) * 16 + i16] = pv[KTW - 1][v];
        q_loop(std::integral_constant<int, KTS>{});
      } else {
        q_loop(std::integral_constant<int, KTW>{});
      }
      // every wave has read the U slab (and the helpers' P tiles are in LDS);
      // O replaces U
      __syncthreads();
      if (owner)
#pragma unroll
        for (int v = 0; v < 4; ++v) pv[KTW - 1][v] = Pex[(rw / 16) * 256 + (4 * kq + v) * 16 + i16];
    }
    // O, without branches: the ratio as P times the hardware reciprocal and
    // its hardware square root (each within about one unit in the last place)
    {
      const int rl0 = rw + 4 * kq;
      const int left = static_cast<int>(min<int64_t>(re - (r0 + rl0), 4));  // rows of the lane's four that exist
      float* ob = (MODE == kProject ? out : U) + (r0 + rl0) * k;
      float* ob2 = out2 ? out2 + (r0 + rl0) * k : nullptr;  // a second copy (kProject: Upsilon; kOnmf: the output)
#pragma unroll
      for (int i = 0; i < KTW; ++i) {
        const int kt = kt0 + i * WPR;
        if (kt >= KT) continue;
        const int c = 16 * kt + i16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool live = v < left && c < k;
          float o;
          if (MODE == kProject) {
            o = pv[i][v];
          } else {
            const float u = Ut[(rl0 + v) * OS + c];
            const float q = qv[i][v];
            const float ratio = pv[i][v] * __builtin_amdgcn_rcpf(q);
            const bool keep = q == 0.0f, neg = !keep && ratio < 0.0f;
            o = keep ? u : (neg ? 0.0f : u * __builtin_amdgcn_sqrtf(ratio));
            hits += (live && (keep || neg)) ? 1 : 0;
          }
          o = live ? o : 0.0f;
          Ut[(rl0 + v) * OS + c] = o;
          if (live) {
            bad = bad || !isfinite(o);
            mx = fmaxf(mx, fabsf(o));
            ob[v * k + c] = o;
            if (ob2) ob2[v * k + c] = o;
          }
        }
      }
    }
    __syncthreads();
    // R^T O, then O^T O, in chunks of CH MFMAs; a chunk's operands are read
    // while the previous chunk's MFMAs run (eight reads in flight, within what
    // the LDS counter tracks)
    constexpr int S4 = ROWS / 4, CH = 4, NCH = S4 / CH;
    float fa[2][CH], fb[2][CH];  // (the second buffer only with DB)
    auto load1 = [&](int q, int h, float* xa, float* xb) {
      const int jt = q / KT, kt = q - (q / KT) * KT;
      const float* pa = Rt + (4 * h * CH + kq) * RS + 16 * jt + i16;
      const float* pb = Ut + (4 * h * CH + kq) * OS + 16 * kt + i16;
#pragma unroll
      for (int s4 = 0; s4 < CH; ++s4) {
        xa[s4] = pa[4 * s4 * RS];
        xb[s4] = pb[4 * s4 * OS];
      }
    };
    auto load2 = [&](int q, int h, float* xa, float* xb) {
      int ta, tb;
      tri_tile(q, ta, tb);
      const float* pa = Ut + (4 * h * CH + kq) * OS + 16 * ta + i16;
      const float* pb = Ut + (4 * h * CH + kq) * OS + 16 * tb + i16;
#pragma unroll
      for (int s4 = 0; s4 < CH; ++s4) {
        xa[s4] = pa[4 * s4 * OS];
        xb[s4] = pb[4 * s4 * OS];
      }
    };
    // step t < NQ1 * NCH: chunk t % NCH of R^T O tile w + waves (t / NCH);
    // then the O^T O tiles likewise
    // A wave with fewer tiles than NQ1 (NQ2) repeats the list's last tile
    // (the copy is not written out), so that no MFMA sits behind a branch.
    auto load_step = [&](int t, float* xa, float* xb) {
      if (t < NQ1 * NCH)
        load1(min(w + kRpWaves * (t / NCH), NT1 - 1), t % NCH, xa, xb);
      else
        load2(min(w + kRpWaves * ((t - NQ1 * NCH) / NCH), NT2 - 1), t % NCH, xa, xb);
    };
    // (kernels whose slab prefetch holds many registers read each chunk just
    // before its MFMAs)
    constexpr bool DB = LIGHT;
    if (DB) load_step(0, fa[0], fb[0]);
#pragma unroll
    for (int t = 0; t < NQ * NCH; ++t) {
      if (DB && t + 1 < NQ * NCH) load_step(t + 1, fa[(t + 1) & 1], fb[(t + 1) & 1]);
      if (!DB) load_step(t, fa[0], fb[0]);
      const int qi = t / NCH;
#pragma unroll
      for (int s4 = 0; s4 < CH; ++s4)
        acc[qi] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[DB ? t & 1 : 0][s4], fb[DB ? t & 1 : 0][s4], acc[qi], 0, 0,
                                                       0);
    }
    __syncthreads();
  }
  const int len = twod * k + k * k;
  double* pb = part + static_cast<int64_t>(blockIdx.x) * len;
#pragma unroll
  for (int qi = 0; qi < NQ1; ++qi) {
    const int q = w + kRpWaves * qi;
    if (q >= NT1) continue;
    const int jt = q / KT, kt = q - (q / KT) * KT;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = 16 * jt + 4 * kq + v, c = 16 * kt + i16;
      if (j < twod && c < k) pb[j * k + c] = static_cast<double>(acc[qi][v]);
    }
  }
#pragma unroll
  for (int qi = 0; qi < NQ2; ++qi) {
    const int q = w + kRpWaves * qi;
    if (q >= NT2) continue;
    int ta, tb;
    tri_tile(q, ta, tb);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * ta + 4 * kq + v, c = 16 * tb + i16;
      const double x = static_cast<double>(acc[NQ1 + qi][v]);
      if (a < k && c < k) {
        pb[twod * k + a * k + c] = x;
        if (ta != tb) pb[twod * k + c * k + a] = x;
      }
    }
  }
  if (hits) atomicAdd(&st->guard_hits, hits);
  if (bad) atomicOr(&st->err_bits, 32);
  mx = wave_max(mx);
  if (lane == 0) atomic_max_nonneg(&st->maxabs_ups_bits, mx);
}

// H update (Eq. update-Q), one thread per entry of the new H; every entry
// reads the old row of H, so the new values go to hn.
__global__ void __launch_bounds__(256)
k_onmf_h(const double* __restrict__ rtu_utu, int twod, int k, const double* __restrict__ H,
         double* __restrict__ hn, DevStatus* __restrict__ st) {
  const double* RtU = rtu_utu;
  const double* UtU = rtu_utu + twod * k;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= twod * k) return;
  const int j = idx / k, c = idx - (idx / k) * k;
  double den = 0.0;
#pragma unroll 8
  for (int t = 0; t < k; ++t) den = fma(H[j * k + t], UtU[t * k + c], den);
  const double h = H[idx];
  if (den == 0.0) {
    hn[idx] = h;
    atomicAdd(&st->guard_hits, 1);
  } else {
    hn[idx] = h * (RtU[idx] / den);
  }
}

// A = (R^T U)^T H_new for the U update, and H <- H_new (FP64 and FP32).
__global__ void __launch_bounds__(256)
k_onmf_a(const double* __restrict__ rtu_utu, int twod, int k, const double* __restrict__ hn, double* __restrict__ H,
         float* __restrict__ H32, float* __restrict__ A32) {
  const double* RtU = rtu_utu;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx < k * k) {
    const int a = idx / k, b = idx - (idx / k) * k;
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < twod; ++j) s = fma(RtU[j * k + a], hn[j * k + b], s);
    A32[idx] = static_cast<float>(s);
  }
  if (idx < twod * k) {
    H[idx] = hn[idx];
    H32[idx] = static_cast<float>(hn[idx]);
  }
}

template <int JT, int KT>
static void rowpass_jk(const Plan& p, void* ws, int mode, const float* Sm, const float* A32, float* copy,
                       hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  const int nb = p.rowpass_blocks;
  const int rpb = static_cast<int>((p.n + nb - 1) / nb);
  if (mode == kProject)
    hipLaunchKernelGGL((k_rowpass_mfma<kProject, JT, KT>), dim3(nb), dim3(64 * rp_waves(JT, KT)), 0, s, bufp<float>(p, ws, B_R),
                       static_cast<int64_t>(p.n), p.twod, p.k, Sm, A32, bufp<float>(p, ws, B_UPS),
                       bufp<float>(p, ws, B_GAMMA), bufp<float>(p, ws, B_UPS), rpb,
                       bufp<double>(p, ws, B_ONMF_PART), st);
  else
    hipLaunchKernelGGL((k_rowpass_mfma<kOnmf, JT, KT>), dim3(nb), dim3(64 * rp_waves(JT, KT)), 0, s, bufp<float>(p, ws, B_R),
                       static_cast<int64_t>(p.n), p.twod, p.k, Sm, A32, bufp<float>(p, ws, B_UPS), nullptr,
                       copy, rpb, bufp<double>(p, ws, B_ONMF_PART), st);
  TPO_LAUNCH_CHECK();
}

template <int JT>
static void rowpass_j(const Plan& p, void* ws, int mode, const float* Sm, const float* A32, float* copy,
                      hipStream_t s) {
  if (p.k <= 16)
    rowpass_jk<JT, 1>(p, ws, mode, Sm, A32, copy, s);
  else if (p.k <= 32)
    rowpass_jk<JT, 2>(p, ws, mode, Sm, A32, copy, s);
  else if (p.k <= 64)
    rowpass_jk<JT, 4>(p, ws, mode, Sm, A32, copy, s);
  else if (p.k <= 80)
    rowpass_jk<JT, 5>(p, ws, mode, Sm, A32, copy, s);
  else if (p.k <= 96)
    rowpass_jk<JT, 6>(p, ws, mode, Sm, A32, copy, s);
  else if (p.k <= 112)
    rowpass_jk<JT, 7>(p, ws, mode, Sm, A32, copy, s);
  else
    rowpass_jk<JT, 8>(p, ws, mode, Sm, A32, copy, s);
}

static void rowpass_any(const Plan& p, void* ws, int mode, const float* Sm, const float* A32, float* copy,
                        hipStream_t s) {
  if (p.twod <= 16)
    rowpass_j<1>(p, ws, mode, Sm, A32, copy, s);
  else if (p.twod <= 32)
    rowpass_j<2>(p, ws, mode, Sm, A32, copy, s);
  else if (p.twod <= 64)
    rowpass_j<4>(p, ws, mode, Sm, A32, copy, s);
  else if (p.twod <= 128)
    rowpass_j<8>(p, ws, mode, Sm, A32, copy, s);
  else
    rowpass_j<16>(p, ws, mode, Sm, A32, copy, s);
}

void launch_onmf(const Plan& p, void* ws, hipStream_t s, float* emb_out) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  const int len = p.twod * p.k + p.k * p.k;
  double* rtu = bufp<double>(p, ws, B_RTU);
  // Gamma = R S, Upsilon = Gamma, and R^T Ups, Ups^T Ups for the first round
  rowpass_any(p, ws, kProject, bufp<float>(p, ws, B_S32), nullptr, nullptr, s);
  for (int t = 0; t < p.par.t_f; ++t) {
    reduce_parts(bufp<double>(p, ws, B_ONMF_PART), p.rowpass_blocks, len, bufp<double>(p, ws, B_REDTMP), rtu, s);
    const int nh = p.twod * p.k, na = std::max(nh, p.k * p.k);
    hipLaunchKernelGGL(k_onmf_h, dim3((nh + 255) / 256), dim3(256), 0, s, rtu, p.twod, p.k, bufp<double>(p, ws, B_H),
                       bufp<double>(p, ws, B_H_NEW), st);
    TPO_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_onmf_a, dim3((na + 255) / 256), dim3(256), 0, s, rtu, p.twod, p.k,
                       bufp<double>(p, ws, B_H_NEW), bufp<double>(p, ws, B_H), bufp<float>(p, ws, B_H32),
                       bufp<float>(p, ws, B_A32));
    TPO_LAUNCH_CHECK();
    // the last round also writes Upsilon to the caller's embedding
    rowpass_any(p, ws, kOnmf, bufp<float>(p, ws, B_H32), bufp<float>(p, ws, B_A32),
                t + 1 == p.par.t_f ? emb_out : nullptr, s);
  }
}

// ---------------------------------------------------------------------------
// NCI (Algorithm 3)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fixed_point_shift(float maxabs, int64_t n) {
  // |sum| <= n * maxabs * 2^S < 2^61
  int ln = 0;
  while ((1ll << ln) < n) ++ln;
  int lm = 0;
  if (maxabs > 0.0f && isfinite(maxabs)) {
    int e;
    frexpf(maxabs, &e);  // maxabs < 2^e
    lm = e;
  }
  int sft = 60 - ln - lm;
  if (sft > 62) sft = 62;
  if (sft < 0) sft = 0;
  return sft;
}

// round(v 2^sft) to nearest, ties to even (the value llrint(ldexp(v, sft))
// has), from the float's bits with integer operations only: v = m 2^e with a
// 24-bit m, so v 2^sft is m shifted left, or m shifted right with the
// dropped bits rounded.  Callers keep |v| 2^sft below 2^61.
__device__ __forceinline__ long long to_fixed(float v, int sft) {
  const uint32_t b = __float_as_uint(v);
  const uint32_t ex = (b >> 23) & 0xffu;
  uint32_t m = b & 0x7fffffu;
  int e = -149;
  if (ex != 0) {
    m |= 0x800000u;
    e = static_cast<int>(ex) - 150;
  }
  const int sh = e + sft;
  unsigned long long r = 0;
  if (sh >= 0) {
    r = static_cast<unsigned long long>(m) << sh;
  } else if (sh >= -24) {
    const int s = -sh;
    const uint32_t q = m >> s, rem = m & ((1u << s) - 1u), half = 1u << (s - 1);
    r = q + ((rem > half || (rem == half && (q & 1u))) ? 1u : 0u);
  }
  return (b >> 31) ? -static_cast<long long>(r) : static_cast<long long>(r);
}

// Sum of per-block integer partials.  part holds len x nb values (entry o of
// block b at part[o * nb + b]); one wave per entry.  Integer addition makes
// the result independent of the order.  NCI rounds: nothing when *skip is 0
// (see nci_skip), and *changed set when a sum differs from the one it
// replaces.
__global__ void __launch_bounds__(256)
k_sum_parts_i64(const long long* __restrict__ part, int nb, int len, long long* __restrict__ sum,
                const int32_t* __restrict__ skip, int32_t* __restrict__ changed) {
  if (skip && *skip == 0) return;
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (o >= len) return;
  long long acc = 0;
  const long long* src = part + static_cast<int64_t>(o) * nb;
  for (int b = lane; b < nb; b += 64) acc += src[b];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) {
    if (changed && sum[o] != acc) atomicOr(changed, 1);
    sum[o] = acc;
  }
}

static void sum_parts_i64(const long long* part, int nb, int len, long long* sum, hipStream_t s,
                          const int32_t* skip = nullptr, int32_t* changed = nullptr) {
  hipLaunchKernelGGL(k_sum_parts_i64, dim3(ceil_div(len, 4)), dim3(256), 0, s, part, nb, len, sum, skip, changed);
  TPO_LAUNCH_CHECK();
}

// A fixed point of the NCI rounds: round t scores against Phi of the label
// sums of round t - 1.  When the sums of round t - 1 equal those of round
// t - 2 (integer sums, compared exactly), Phi and therefore every later
// round's labels and sums repeat round t - 1's, so rounds t.. are skipped and
// the result is the one all T_g rounds give.  changed[t - 1] (zeroed before
// the rounds) is set by round t - 1's sums when they differ from round t -
// 2's; round t's kernels do nothing when it is 0.  A skipped round leaves
// its own flag 0, so the rounds after it are skipped too.  Rounds 1 and 2
// always run (round 1 scores against the identity, not against sums).
static const int32_t* nci_skip(const int32_t* changed, int t) {
  return t >= 3 ? changed + (t - 2) : nullptr;
}

// One round: scores = U Phi (FP64), l* = first argmax, labels written.  Phi
// is phi_g (k x k, Phi[t][l] at t * k + l) when given, else the identity when
// `sums` is null, else Phi[t][l] = c_l[t] / sqrt(|C_l|)
// with c_l the fixed-point sum of the U rows labelled l and |C_l| their count
// (sums: k x k values c_l[t] at l * k + t, then k counts).  When `part` is
// given, the block's own fixed-point sums and counts for the labels of this
// round are written there (transposed, entry o at part[o * gridDim.x + block]).
// KT: compile-time bound on k; one row per lane, its k entries and k scores in
// registers, Phi (zero padded to KT x KT) in LDS.
template <int KT>
__global__ void __launch_bounds__(256)
k_nci_round(const float* __restrict__ U, int64_t n, int k, const long long* __restrict__ sums,
            const double* __restrict__ phi_g, long long* __restrict__ part, int32_t* __restrict__ labels,
            int rows_per_block, DevStatus* __restrict__ st, const int32_t* __restrict__ skip, int round) {
  if (skip && *skip == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(&st->nci_rounds, round);
  constexpr int LD = KT + 1;  // staging stride (odd for even KT)
  __shared__ double phi[KT * KT];
  __shared__ double fac[KT];
  __shared__ long long accl[KT * KT + KT];  // k x k sums (stride k), then k counts
  __shared__ float ut[4 * 64 * LD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int sft = fixed_point_shift(__uint_as_float(st->maxabs_ups_bits), n);
  const double inv_scale = ldexp(1.0, -sft);
  if (sums && tid < k) {
    const long long c = sums[k * k + tid];
    fac[tid] = c > 0 ? inv_scale / sqrt(static_cast<double>(c)) : 0.0;
  }
  for (int e = tid; e < k * k + k; e += 256) accl[e] = 0;
  __syncthreads();
  for (int e = tid; e < KT * KT; e += 256) {
    const int t = e / KT, l = e - (e / KT) * KT;
    double v = 0.0;
    if (t < k && l < k)
      v = phi_g ? phi_g[t * k + l] : sums ? static_cast<double>(sums[l * k + t]) * fac[l] : (t == l ? 1.0 : 0.0);
    phi[e] = v;
  }
  __syncthreads();
  float* myut = ut + w * 64 * LD;
  const int64_t rb = static_cast<int64_t>(blockIdx.x) * rows_per_block;
  const int64_t re = min(n, rb + rows_per_block);
  const int rpi = 64 / k;  // rows per accumulation step (k <= 64)
  for (int64_t b0 = rb + static_cast<int64_t>(w) * 64; b0 < re; b0 += 256) {
    const int64_t row = b0 + lane;
    const bool live = row < re;
    float u[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) u[t] = (live && t < k) ? U[row * k + t] : 0.0f;
    double sc[KT];
#pragma unroll
    for (int l = 0; l < KT; ++l) sc[l] = 0.0;
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      if (t < k) {
        const double x = static_cast<double>(u[t]);
#pragma unroll
        for (int l = 0; l < KT; ++l) sc[l] = fma(x, phi[t * KT + l], sc[l]);
      }
    }
    int best = 0;
    double bestv = sc[0];
#pragma unroll
    for (int l = 1; l < KT; ++l)
      if (l < k && sc[l] > bestv) {
        bestv = sc[l];
        best = l;
      }
    if (live) labels[row] = best;
    if (part) {
      const int nr = static_cast<int>(min(static_cast<int64_t>(64), re - b0));
#pragma unroll
      for (int t = 0; t < KT; ++t)
        if (t < k) myut[lane * LD + t] = u[t];
      wave_sync();
      const int g = lane / k, t = lane - (lane / k) * k;
      for (int r0 = 0; r0 < nr; r0 += rpi) {
        const int rr = r0 + g;
        const int lab = __shfl(best, rr < 64 ? rr : 63, 64);
        if (g < rpi && rr < nr) {
          atomicAdd(reinterpret_cast<unsigned long long*>(&accl[lab * k + t]),
                    static_cast<unsigned long long>(to_fixed(myut[rr * LD + t], sft)));
          if (t == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&accl[k * k + lab]), 1ull);
        }
      }
      wave_sync();
    }
  }
  __syncthreads();
  if (part) {
    for (int e = tid; e < k * k + k; e += 256) part[static_cast<int64_t>(e) * gridDim.x + blockIdx.x] = accl[e];
  }
}

// k > 32: scoring and the label sums in two kernels (Phi for 128 labels
// fills much of the LDS on its own; for k in 33..64 the one-kernel round
// above needs a whole SIMD's registers per wave for its k scores).
//
// Scores on FP32 MFMA (v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16], its v-th result is D[4 (l / 16) + v][l % 16]).  A wave
// forms S^T = Phi^T U^T for 16 rows at a time: A = Phi^T (a 16-label tile),
// B = U^T (the 16 rows), so lane l ends with the scores of row l % 16 for the
// labels 16 c + 4 (l / 16) + v; the first maximum and the runner-up are found
// in registers and then over the four lanes that share the row.  Phi^T (16 LT
// x k, FP64 values rounded to FP32, zero padded) sits in LDS, shared by the
// workgroup's eight waves.  The j-th of four consecutive MFMAs gives depth slot l / 16 the
// contraction index 16 m + 4 (l / 16) + j, so a lane's four values of a U row
// come in with one 16-byte load (k a multiple of 4) and its four of Phi^T
// with one 16-byte LDS read.
//
// The decision must be the one FP64 scores give.  Each FP32 score is within
// (k + 2) 2^-24 ||u_i||_2 max_l ||phi_l||_2 of the exact one (k rounded
// products and sums, and the rounding of Phi to FP32); a row whose two best
// scores are closer than twice that (with a factor two to spare) goes to a
// list, and k_nci_recheck recomputes its scores in FP64.
constexpr int kNciWide = 128;
constexpr int kNciMaxRounds = 1024;  // round counters of the recheck list

constexpr int kNciScoreWaves = 8;
constexpr int kNciFusedWaves = 16;

// ACC: the same kernel also forms this round's label sums (the next round's
// Phi) for the rows whose decision it makes, in int64 fixed point in LDS
// (dynamic, k x k + k), written as partial column blockIdx.x of part (entry
// o at part[o * pstride + column]); the last column, pstride - 1, is zeroed
// here by workgroup 0 and takes the rows k_nci_recheck decides.
template <int LT, bool ACC>
__global__ void __launch_bounds__(64 * (ACC ? kNciFusedWaves : kNciScoreWaves))
k_nci_score_mfma(const float* __restrict__ U, int64_t n, int k, const long long* __restrict__ sums,
                 const double* __restrict__ phi_g, int32_t* __restrict__ labels, int32_t* __restrict__ check_count,
                 int32_t* __restrict__ check_rows, const DevStatus* __restrict__ st,
                 const int32_t* __restrict__ skip, long long* __restrict__ part, int pstride) {
  if (skip && *skip == 0) return;
  constexpr int WV = ACC ? kNciFusedWaves : kNciScoreWaves;
  extern __shared__ long long accl[];  // ACC: k x k sums, then k counts
  constexpr int NL = 16 * LT;
  constexpr int NLP = NL + 4;  // row stride of Phi^T: 16-byte reads of 8 consecutive lanes in distinct banks
  __shared__ __align__(16) float phit[NL * NLP];  // phit[l * NLP + t] = Phi[t][l]
  __shared__ double fac[NL];
  __shared__ unsigned int colmax_bits;  // max_l ||phi_l||_2 as float bits
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int sft = fixed_point_shift(__uint_as_float(st->maxabs_ups_bits), n);
  const double inv_scale = ldexp(1.0, -sft);
  if (tid == 0) colmax_bits = 0u;
  if (sums && tid < k) {
    const long long c = sums[k * k + tid];
    fac[tid] = c > 0 ? inv_scale / sqrt(static_cast<double>(c)) : 0.0;
  }
  __syncthreads();
  auto phi64 = [&](int t, int l) -> double {
    if (t >= k || l >= k) return 0.0;
    return phi_g ? phi_g[t * k + l] : sums ? static_cast<double>(sums[l * k + t]) * fac[l] : (t == l ? 1.0 : 0.0);
  };
  // k < 16 LT: the last step (m = LT - 1) gives slot l / 16 of its j-th MFMA
  // the index 16 m + 4 j + l / 16 instead, so that the MFMAs whose four
  // slots all lie at or beyond k are left out (uniform); that block of Phi^T
  // is stored permuted to match (index 16 m + 4 j + q at 16 m + 4 q + j), so
  // its 16-byte reads are the same as the other steps'
  const bool tail = k < 16 * LT;
  for (int e = tid; e < NL * NL; e += 64 * WV) {
    const int t = e / NL, l = e - (e / NL) * NL;
    int pos = t;
    if (tail && t >= 16 * (LT - 1)) {
      const int r = t - 16 * (LT - 1);
      pos = 16 * (LT - 1) + 4 * (r & 3) + (r >> 2);
    }
    phit[l * NLP + pos] = static_cast<float>(phi64(t, l));
  }
  if (ACC) {
    for (int e = tid; e < k * k + k; e += 64 * WV) accl[e] = 0;
    if (blockIdx.x == 0)
      for (int e = tid; e < k * k + k; e += 64 * WV) part[static_cast<int64_t>(e) * pstride + (pstride - 1)] = 0;
  }
  if (tid < k) {
    double ss = 0.0;
    for (int t = 0; t < k; ++t) {
      const double v = phi64(t, tid);
      ss = fma(v, v, ss);
    }
    // rounded up: an upper bound on the column norm
    atomicMax(&colmax_bits, __float_as_uint(__double2float_ru(sqrt(ss))));
  }
  __syncthreads();
  const double tol_scale = static_cast<double>(k + 2) * ldexp(1.0, -24) * 2.0 * 2.0 *
                           static_cast<double>(__uint_as_float(colmax_bits));
  const bool vec = (k & 3) == 0;  // rows of U start on 16-byte boundaries
  const int64_t ntiles = (n + 15) / 16;
  for (int64_t tile = static_cast<int64_t>(blockIdx.x) * WV + w; tile < ntiles;
       tile += static_cast<int64_t>(gridDim.x) * WV) {
    const int64_t row = tile * 16 + i16;
    const bool live = row < n;
    const float* urow = U + row * k;
    v4f_t ub[LT];
    double u2 = 0.0;
#pragma unroll
    for (int m = 0; m < LT; ++m) {
      const int t0 = 16 * m + 4 * g;
      if (m == LT - 1 && tail) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int t = 16 * m + 4 * j + g;
          ub[m][j] = (live && t < k) ? urow[t] : 0.0f;
        }
      } else if (vec) {
        ub[m] = (live && t0 < k) ? *reinterpret_cast<const v4f_t*>(urow + t0) : v4f_t{0.f, 0.f, 0.f, 0.f};
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) ub[m][j] = (live && t0 + j < k) ? urow[t0 + j] : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) u2 = fma(static_cast<double>(ub[m][j]), static_cast<double>(ub[m][j]), u2);
    }
    v4f_t acc[LT];
#pragma unroll
    for (int c = 0; c < LT; ++c) acc[c] = v4f_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < LT; ++m) {
      if (16 * m >= k) break;  // uniform: the padded steps add zeros
#pragma unroll
      for (int c = 0; c < LT; ++c) {
        const v4f_t a = *reinterpret_cast<const v4f_t*>(&phit[(16 * c + i16) * NLP + 16 * m + 4 * g]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (m == LT - 1 && tail && 16 * m + 4 * j >= k) break;  // uniform
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], ub[m][j], acc[c], 0, 0, 0);
        }
      }
    }
    // first maximum and runner-up: labels in increasing order within the
    // lane, then the lower label wins a tie between lanes
    int best = 4 * g;
    float bestv = -INFINITY, second = -INFINITY;
#pragma unroll
    for (int c = 0; c < LT; ++c) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int L = 16 * c + 4 * g + v;
        if (L < k) {
          const float x = acc[c][v];
          if (x > bestv) {
            second = bestv;
            bestv = x;
            best = L;
          } else if (x > second) {
            second = x;
          }
        }
      }
    }
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      const float ov = __shfl_xor(bestv, off, 64);
      const float os = __shfl_xor(second, off, 64);
      const int ob = __shfl_xor(best, off, 64);
      u2 += __shfl_xor(u2, off, 64);
      if (ov > bestv || (ov == bestv && ob < best)) {
        second = fmaxf(bestv, os);
        bestv = ov;
        best = ob;
      } else {
        second = fmaxf(second, ov);
      }
    }
    // (the four lanes of a row hold the same best, runner-up and norm)
    const bool close = static_cast<double>(bestv) - static_cast<double>(second) <= tol_scale * sqrt(u2);
    if (live && g == 0) {
      labels[row] = best;
      if (close) {
        const int slot = atomicAdd(check_count, 1);
        check_rows[slot] = static_cast<int32_t>(row);
      }
    }
    if (ACC && live && !close) {
#pragma unroll
      for (int m = 0; m < LT; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int t = (m == LT - 1 && tail) ? 16 * m + 4 * j + g : 16 * m + 4 * g + j;
          if (t < k)
            atomicAdd(reinterpret_cast<unsigned long long*>(&accl[best * k + t]),
                      static_cast<unsigned long long>(to_fixed(ub[m][j], sft)));
        }
      if (g == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&accl[k * k + best]), 1ull);
    }
  }
  if (ACC) {
    __syncthreads();
    for (int e = tid; e < k * k + k; e += 64 * WV) part[static_cast<int64_t>(e) * pstride + blockIdx.x] = accl[e];
  }
}

// The rows whose FP32 decision was too close: FP64 scores (Phi from the same
// sums, or phi_g, or the identity), first maximum, one wave per row.  A
// workgroup with rows to decide forms Phi (k x k, FP64) in LDS once, and each
// wave stages its row of U there, so the scores read both from LDS.
constexpr int kNciRecheckMaxLds = 128 * 128 * 8;
__global__ void __launch_bounds__(256)
k_nci_recheck(const float* __restrict__ U, int k, const long long* __restrict__ sums,
              const double* __restrict__ phi_g, const int32_t* __restrict__ check_count,
              const int32_t* __restrict__ check_rows, int32_t* __restrict__ labels, int64_t n,
              DevStatus* __restrict__ st, const int32_t* __restrict__ skip, int round, long long* __restrict__ part,
              int pstride) {
  if (skip && *skip == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(&st->nci_rounds, round);
  const int lane = threadIdx.x & 63;
  const int cnt = *check_count;
  if (blockIdx.x == 0 && threadIdx.x == 0 && cnt > 0) atomicAdd(&st->nci_rechecked, cnt);
  const int sft = fixed_point_shift(__uint_as_float(st->maxabs_ups_bits), n);
  const double inv_scale = ldexp(1.0, -sft);
  const int waves = static_cast<int>(gridDim.x) * 4;
  if (static_cast<int>(blockIdx.x) * 4 >= cnt) return;  // uniform: no row for this workgroup
  extern __shared__ double phs[];  // phs[t k + l] = Phi[t][l]
  __shared__ float us[4][128];      // each wave's row of U
  for (int e = threadIdx.x; e < k * k; e += 256) {
    const int t = e / k, l = e - (e / k) * k;
    double ph;
    if (phi_g) {
      ph = phi_g[e];
    } else if (sums) {
      const long long c = sums[k * k + l];
      const double f = c > 0 ? inv_scale / sqrt(static_cast<double>(c)) : 0.0;
      ph = static_cast<double>(sums[l * k + t]) * f;
    } else {
      ph = t == l ? 1.0 : 0.0;
    }
    phs[e] = ph;
  }
  __syncthreads();
  float* ur = us[threadIdx.x >> 6];
  for (int i = static_cast<int>(blockIdx.x) * 4 + static_cast<int>(threadIdx.x >> 6); i < cnt; i += waves) {
    const int64_t row = check_rows[i];
    const float* urow = U + row * k;
    for (int t = lane; t < k; t += 64) ur[t] = urow[t];
    wave_sync();
    int best = -1;
    double bestv = 0.0;
    for (int l = lane; l < k; l += 64) {
      double sc = 0.0;
      for (int t = 0; t < k; ++t) sc = fma(static_cast<double>(ur[t]), phs[t * k + l], sc);
      if (best < 0 || sc > bestv) {
        bestv = sc;
        best = l;
      }
    }
    wave_sync();  // every lane has read the row before the next one replaces it
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double ov = __shfl_xor(bestv, off, 64);
      const int ob = __shfl_xor(best, off, 64);
      if (ob >= 0 && (best < 0 || ov > bestv || (ov == bestv && ob < best))) {
        bestv = ov;
        best = ob;
      }
    }
    if (lane == 0) labels[row] = best;
    if (part) {  // the fused scoring left this row's sums to its final decision
      long long* col = part + (pstride - 1);
      for (int l = lane; l < k; l += 64)
        atomicAdd(reinterpret_cast<unsigned long long*>(&col[static_cast<int64_t>(best * k + l) * pstride]),
                  static_cast<unsigned long long>(to_fixed(urow[l], sft)));
      if (lane == 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(&col[static_cast<int64_t>(k * k + best) * pstride]), 1ull);
    }
  }
}

__global__ void k_zero_i32(int32_t* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// Fixed-point sums of the U rows per label and the label counts for this
// workgroup's rows [rb, rb + rows_per_block), written transposed (entry o at
// part[o * gridDim.x + block]).  A wave takes 64 rows at a time and reads
// them as one contiguous run of 64 k values, eight loads in flight per lane;
// element e of the run is (row e / k, column e % k), tracked incrementally
// (k > 32: a step of 64 elements crosses at most two row ends).
constexpr int kNciAccBatch = 8;

__global__ void __launch_bounds__(1024)
k_nci_accum_wide(const float* __restrict__ U, int64_t n, int k, const int32_t* __restrict__ labels,
                 long long* __restrict__ part, int64_t rows_per_block, const DevStatus* __restrict__ st,
                 const int32_t* __restrict__ skip) {
  if (skip && *skip == 0) return;
  extern __shared__ long long accl[];  // k x k sums, then k counts (dynamic: sized to k)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int sft = fixed_point_shift(__uint_as_float(st->maxabs_ups_bits), n);
  for (int e = tid; e < k * k + k; e += 1024) accl[e] = 0;
  __syncthreads();
  const int64_t rb = static_cast<int64_t>(blockIdx.x) * rows_per_block;
  const int64_t re = min(n, rb + rows_per_block);
  for (int64_t r0 = rb + 64 * static_cast<int64_t>(w); r0 < re; r0 += 64 * 16) {
    const int nr = static_cast<int>(min(static_cast<int64_t>(64), re - r0));
    const int lab = lane < nr ? labels[r0 + lane] : 0;
    if (lane < nr) atomicAdd(reinterpret_cast<unsigned long long*>(&accl[k * k + lab]), 1ull);
    const float* src = U + r0 * k;
    const int total = nr * k;
    int row = lane / k, col = lane - (lane / k) * k;  // of element lane
    for (int e0 = 0; e0 < total; e0 += 64 * kNciAccBatch) {
      float v[kNciAccBatch];
#pragma unroll
      for (int b = 0; b < kNciAccBatch; ++b) {
        const int e = e0 + 64 * b + lane;
        v[b] = e < total ? src[e] : 0.0f;
      }
#pragma unroll
      for (int b = 0; b < kNciAccBatch; ++b) {
        const int e = e0 + 64 * b + lane;
        const int lr = __shfl(lab, row < 64 ? row : 63, 64);
        if (e < total)
          atomicAdd(reinterpret_cast<unsigned long long*>(&accl[lr * k + col]),
                    static_cast<unsigned long long>(to_fixed(v[b], sft)));
        col += 64;
        if (col >= k) {
          col -= k;
          ++row;
        }
        if (col >= k) {
          col -= k;
          ++row;
        }
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < k * k + k; e += 1024) part[static_cast<int64_t>(e) * gridDim.x + blockIdx.x] = accl[e];
}

// dynamic LDS of k_nci_recheck (Phi, k x k FP64); its limit is set once
static size_t nci_recheck_lds(int k) {
  static std::once_flag once;
  std::call_once(once, [] {
    TPO_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nci_recheck),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kNciRecheckMaxLds));
  });
  return static_cast<size_t>(k) * k * sizeof(double);
}

// One round's scores and decisions.  With `acc` and k <= 112 (Phi^T and the
// k x k + k sums both fit the LDS) the scoring kernel also forms the round's
// label sums, as partial columns of part: the return value is their number
// (at most max_cols), 0 when the sums are left to k_nci_accum_wide.
template <int LT>
static int nci_score_mfma(const float* U, int64_t n, int k, const long long* sums, const double* phi_g,
                          int32_t* labels, int32_t* check_count, int32_t* check_rows, DevStatus* st,
                          const int32_t* skip, int round, long long* part, int max_cols, bool acc, hipStream_t s) {
  const int64_t ntiles = (n + 15) / 16;
  if constexpr (LT <= 7) {
    if (acc && max_cols >= 2) {
      constexpr int NL = 16 * LT;
      static std::once_flag once;
      std::call_once(once, [] {
        TPO_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nci_score_mfma<LT, true>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          static_cast<int>((NL * NL + NL) * sizeof(long long))));
      });
      const size_t dyn = static_cast<size_t>(k * k + k) * sizeof(long long);
      int b = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(&k_nci_score_mfma<LT, true>),
                                                       64 * kNciFusedWaves, dyn) != hipSuccess ||
          b < 1)
        b = 1;
      const int nb = static_cast<int>(std::max<int64_t>(
          1, std::min<int64_t>({(ntiles + kNciFusedWaves - 1) / kNciFusedWaves, 256 * static_cast<int64_t>(b),
                                static_cast<int64_t>(max_cols - 1)})));
      hipLaunchKernelGGL((k_nci_score_mfma<LT, true>), dim3(nb), dim3(64 * kNciFusedWaves), dyn, s, U, n, k, sums,
                         phi_g, labels, check_count, check_rows, st, skip, part, nb + 1);
      TPO_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_nci_recheck, dim3(64), dim3(256), nci_recheck_lds(k), s, U, k, sums, phi_g, check_count,
                         check_rows, labels,
                         n, st, skip, round, part, nb + 1);
      TPO_LAUNCH_CHECK();
      return nb + 1;
    }
  }
  // workgroups resident per CU (LDS and registers), asked once: the grid is
  // the number that fits, so the last of its tiles does not run alone
  static const int per_cu = [] {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(&k_nci_score_mfma<LT, false>),
                                                     64 * kNciScoreWaves, 0) != hipSuccess ||
        b < 1)
      b = 1;
    return b;
  }();
  const int nb = static_cast<int>(
      std::max<int64_t>(1, std::min<int64_t>((ntiles + kNciScoreWaves - 1) / kNciScoreWaves, 256 * per_cu)));
  hipLaunchKernelGGL((k_nci_score_mfma<LT, false>), dim3(nb), dim3(64 * kNciScoreWaves), 0, s, U, n, k, sums, phi_g,
                     labels, check_count, check_rows, st, skip, nullptr, 0);
  TPO_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_nci_recheck, dim3(64), dim3(256), nci_recheck_lds(k), s, U, k, sums, phi_g, check_count,
                     check_rows, labels, n,
                     st, skip, round, nullptr, 0);
  TPO_LAUNCH_CHECK();
  return 0;
}

// Procrustes form of the Phi update: Phi = the orthogonal factor of the polar
// decomposition of M = Ups^T Y, which is the orthogonal matrix minimising
// ||Ups Phi - Y||_F (Section 3.4 states this minimisation; the printed update
// Ups^T Y is not orthogonal).  An empty cluster leaves a zero column in M;
// Phi is then the polar factor of M's other columns with that column zero
// (the partial isometry), M being of full rank on the nonzero columns.
//
// k <= 64: Newton-Schulz, X <- X (3 I - X^T X) / 2 from X = M / ||M||_F, which
// takes every nonzero singular value to 1 (quadratically once near it) and
// keeps a zero column zero; it stops when an iteration moves X by at most
// 1e-14 sqrt(k) in Frobenius norm (at most kNsMaxIter iterations).  X, X^T X
// and the next X in LDS, one workgroup.
constexpr int kNsMaxIter = 200;

template <int KW, int NT>
__global__ void __launch_bounds__(NT)
k_nci_polar_ns(const long long* __restrict__ sums, int k, int64_t n, const DevStatus* __restrict__ st,
               double* __restrict__ phi, const int32_t* __restrict__ skip) {
  if (skip && *skip == 0) return;
  __shared__ double Xa[KW * (KW + 1)];
  __shared__ double Xb[KW * (KW + 1)];
  __shared__ double G[KW * (KW + 1)];
  __shared__ double red[NT];
  __shared__ double fac[KW];
  const int tid = threadIdx.x;
  const int la = k | 1;
  const int sft = fixed_point_shift(__uint_as_float(st->maxabs_ups_bits), n);
  const double inv_scale = ldexp(1.0, -sft);
  for (int c = tid; c < k; c += NT) {
    const long long cnt = sums[k * k + c];
    fac[c] = cnt > 0 ? inv_scale / sqrt(static_cast<double>(cnt)) : 0.0;
  }
  __syncthreads();
  double ss = 0.0;
  for (int e = tid; e < k * k; e += NT) {
    const int t = e / k, l = e - (e / k) * k;
    const double v = static_cast<double>(sums[l * k + t]) * fac[l];
    Xa[t * la + l] = v;
    ss = fma(v, v, ss);
  }
  const double nrm2 = blk_sum(ss, red);
  if (nrm2 == 0.0) {  // uniform: no rows at all
    for (int e = tid; e < k * k; e += NT) phi[e] = 0.0;
    return;
  }
  const double inv = 1.0 / sqrt(nrm2);
  for (int e = tid; e < k * k; e += NT) {
    const int t = e / k, l = e - (e / k) * k;
    Xa[t * la + l] *= inv;
  }
  __syncthreads();
  double* X = Xa;
  double* Xn = Xb;
  const double tol2 = 1e-28 * k;
  for (int it = 0; it < kNsMaxIter; ++it) {
    for (int e = tid; e < k * k; e += NT) {
      const int i = e / k, j = e - (e / k) * k;
      double a = 0.0;
      for (int t = 0; t < k; ++t) a = fma(X[t * la + i], X[t * la + j], a);
      G[i * la + j] = a;
    }
    __syncthreads();
    double dd = 0.0;
    for (int e = tid; e < k * k; e += NT) {
      const int t = e / k, j = e - (e / k) * k;
      double a = 0.0;
      for (int i = 0; i < k; ++i) a = fma(X[t * la + i], G[i * la + j], a);
      const double x = X[t * la + j];
      const double y = fma(-0.5, a, 1.5 * x);
      Xn[t * la + j] = y;
      dd = fma(y - x, y - x, dd);
    }
    const double d2 = blk_sum(dd, red);  // ends with a barrier
    double* tmp = X;
    X = Xn;
    Xn = tmp;
    if (d2 <= tol2) break;  // uniform
  }
  for (int e = tid; e < k * k; e += NT) {
    const int t = e / k, l = e - (e / k) * k;
    phi[e] = X[t * la + l];
  }
}

// k > 64: M^T M = V diag(lambda) V^T by Jacobi and Phi = M V diag(d) V^T with
// d_i = 1 / sqrt(lambda_i) for lambda_i > 0 (an empty cluster's zero column
// gives an exactly zero row and column of M^T M, which no rotation touches,
// so its lambda is exactly 0; 1e-24 of the largest guards the division).  One
// workgroup of NT threads for k <= KW; M and V in global scratch (k x k,
// row-major), M^T M and then V diag(d) V^T in LDS.
template <int KW, int NT, int KB>
__global__ void __launch_bounds__(NT)
k_nci_polar(const long long* __restrict__ sums, int k, int64_t n, const DevStatus* __restrict__ st,
            double* __restrict__ Mg, double* __restrict__ Vg, double* __restrict__ phi,
            const int32_t* __restrict__ skip) {
  if (skip && *skip == 0) return;
  __shared__ double A[KW * (KW + 1)];
  __shared__ __align__(16) double sh[3 * (KW / 2)];
  __shared__ double fac[KW];
  __shared__ double dl[KW];
  __shared__ double lmax;
  double* M = Mg;
  double* V = Vg;
  const int tid = threadIdx.x;
  const int sft = fixed_point_shift(__uint_as_float(st->maxabs_ups_bits), n);
  const double inv_scale = ldexp(1.0, -sft);
  for (int c = tid; c < k; c += NT) {
    const long long cnt = sums[k * k + c];
    fac[c] = cnt > 0 ? inv_scale / sqrt(static_cast<double>(cnt)) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += NT) {
    const int t = e / k, l = e - (e / k) * k;
    M[e] = static_cast<double>(sums[l * k + t]) * fac[l];
  }
  __syncthreads();
  const int la = k | 1;
  // M^T M, both triangles by the same product order (exactly symmetric)
  for (int e = tid; e < k * k; e += NT) {
    const int i = e / k, j = e - (e / k) * k;
    double a = 0.0;
    for (int t = 0; t < k; ++t) a = fma(M[t * k + i], M[t * k + j], a);
    A[i * la + j] = a;
  }
  __syncthreads();
  blk_jacobi<KB>(A, la, V, k, k, sh, nullptr, 40);
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < k; ++i) m = fmax(m, A[i * la + i]);
    lmax = m;
  }
  __syncthreads();
  for (int c = tid; c < k; c += NT) {
    const double lam = A[c * la + c];
    dl[c] = (lmax > 0.0 && lam > 1e-24 * lmax) ? 1.0 / sqrt(lam) : 0.0;
  }
  __syncthreads();
  // W = V diag(d) V^T into A
  for (int e = tid; e < k * k; e += NT) {
    const int i = e / k, j = e - (e / k) * k;
    double a = 0.0;
    for (int c = 0; c < k; ++c) a = fma(V[i * k + c] * dl[c], V[j * k + c], a);
    A[i * la + j] = a;
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += NT) {
    const int t = e / k, l = e - (e / k) * k;
    double a = 0.0;
    for (int j = 0; j < k; ++j) a = fma(M[t * k + j], A[j * la + l], a);
    phi[e] = a;
  }
}

// Phi for the next round from the label sums: the literal update leaves it to
// the score kernel (built from `sums`); the Procrustes form computes it here.
// Jacobi item counts (k > 64): (k/2)^2 <= 2 KB NT and k^2/2 <= 4 KB NT.
static const double* nci_phi(const Plan& p, void* ws, const long long* sums, const int32_t* skip, hipStream_t s) {
  // k = 1: every row takes label 0 whatever Phi is
  if (!(p.par.flags & TPO_FLAG_NCI_PROCRUSTES) || p.k == 1) return nullptr;
  double* phi = bufp<double>(p, ws, B_NCI_PHI);
  const int64_t n = static_cast<int64_t>(p.n);
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  double* mg = bufp<double>(p, ws, B_NCI_PM);
  double* vg = bufp<double>(p, ws, B_NCI_PV);
  if (p.k <= 32)
    hipLaunchKernelGGL((k_nci_polar_ns<32, 256>), dim3(1), dim3(256), 0, s, sums, p.k, n, st, phi, skip);
  else if (p.k <= 64)
    hipLaunchKernelGGL((k_nci_polar_ns<64, 256>), dim3(1), dim3(256), 0, s, sums, p.k, n, st, phi, skip);
  else
    hipLaunchKernelGGL((k_nci_polar<kNciWide, 512, 4>), dim3(1), dim3(512), 0, s, sums, p.k, n, st, mg, vg, phi,
                       skip);
  TPO_LAUNCH_CHECK();
  return phi;
}

static void nci_rounds_wide(const Plan& p, void* ws, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  const int k = p.k;
  long long* part = bufp<long long>(p, ws, B_NCI_PART);
  long long* sums = bufp<long long>(p, ws, B_NCI_SUM);
  const int64_t n = static_cast<int64_t>(p.n);
  // the label sums' LDS is sized to k, so up to k = 100 two accumulation
  // workgroups share a CU; 64-row runs per wave
  const size_t acc_lds = static_cast<size_t>(k * k + k) * sizeof(long long);
  // the dynamic-LDS limit is a process-wide attribute: set once, to the
  // largest k's need, so that concurrent callers never race on it
  static std::once_flag once;
  std::call_once(once, [] {
    TPO_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nci_accum_wide),
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      static_cast<int>((kNciWide * kNciWide + kNciWide) * sizeof(long long))));
  });
  const int64_t per_cu = acc_lds <= 80 * 1024 ? 2 : 1;
  const int nb = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>({(n + 63) / 64, 256 * per_cu,
                                                                           static_cast<int64_t>(p.rowpass_blocks)})));
  const int64_t rpb = ((n + nb - 1) / nb + 63) / 64 * 64;
  const float* U = bufp<float>(p, ws, B_UPS);
  int32_t* labels = bufp<int32_t>(p, ws, B_LABELS);
  const int rounds = std::max(p.par.t_g, 1);
  // recheck lists: one counter per round, then the rounds' changed flags
  // (nci_skip), both zeroed here; then one row list
  int32_t* cnt = bufp<int32_t>(p, ws, B_NCI_CHECK);
  int32_t* changed = cnt + kNciMaxRounds;
  int32_t* rows = changed + kNciMaxRounds;
  hipLaunchKernelGGL(k_zero_i32, dim3(ceil_div(2 * kNciMaxRounds, 256)), dim3(256), 0, s, cnt, 2 * kNciMaxRounds);
  TPO_LAUNCH_CHECK();
  for (int t = 1; t <= rounds; ++t) {
    const int32_t* skip = nci_skip(changed, t);
    const long long* sm = t == 1 ? nullptr : sums;
    const double* ph = t == 1 ? nullptr : nci_phi(p, ws, sums, skip, s);
    if (ph) sm = nullptr;
    int32_t* c = cnt + (t - 1);
    const bool acc = t < p.par.t_g;  // the last round's sums are not used
    const int pcols = p.rowpass_blocks + 1;  // partial columns the workspace holds
    int cols = 0;
    switch ((k + 15) / 16) {
      case 3: cols = nci_score_mfma<3>(U, n, k, sm, ph, labels, c, rows, st, skip, t, part, pcols, acc, s); break;
      case 4: cols = nci_score_mfma<4>(U, n, k, sm, ph, labels, c, rows, st, skip, t, part, pcols, acc, s); break;
      case 5: cols = nci_score_mfma<5>(U, n, k, sm, ph, labels, c, rows, st, skip, t, part, pcols, acc, s); break;
      case 6: cols = nci_score_mfma<6>(U, n, k, sm, ph, labels, c, rows, st, skip, t, part, pcols, acc, s); break;
      case 7: cols = nci_score_mfma<7>(U, n, k, sm, ph, labels, c, rows, st, skip, t, part, pcols, acc, s); break;
      case 8: cols = nci_score_mfma<8>(U, n, k, sm, ph, labels, c, rows, st, skip, t, part, pcols, acc, s); break;
      default: throw std::runtime_error("NCI: k outside 33..128 on the two-kernel path");
    }
    if (acc) {
      if (cols == 0) {
        hipLaunchKernelGGL(k_nci_accum_wide, dim3(nb), dim3(1024), acc_lds, s, U, n, k, labels, part, rpb, st, skip);
        TPO_LAUNCH_CHECK();
        cols = nb;
      }
      sum_parts_i64(part, cols, k * k + k, sums, s, skip, t >= 2 ? changed + (t - 1) : nullptr);
    }
  }
}

template <int KT>
static void nci_rounds(const Plan& p, void* ws, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  const int k = p.k;
  long long* part = bufp<long long>(p, ws, B_NCI_PART);
  long long* sums = bufp<long long>(p, ws, B_NCI_SUM);
  const int nb = p.rowpass_blocks;
  const int rpb = static_cast<int>((p.n + nb - 1) / nb);
  const float* U = bufp<float>(p, ws, B_UPS);
  int32_t* labels = bufp<int32_t>(p, ws, B_LABELS);
  const int rounds = std::max(p.par.t_g, 1);
  int32_t* changed = bufp<int32_t>(p, ws, B_NCI_CHECK) + kNciMaxRounds;  // see nci_skip
  hipLaunchKernelGGL(k_zero_i32, dim3(ceil_div(kNciMaxRounds, 256)), dim3(256), 0, s, changed, kNciMaxRounds);
  TPO_LAUNCH_CHECK();
  for (int t = 1; t <= rounds; ++t) {
    // round 1 (and T_g = 0) scores against Phi = I; every round but the last
    // feeds the label sums to the next
    const bool acc = t < p.par.t_g;
    const int32_t* skip = nci_skip(changed, t);
    const double* ph = t == 1 ? nullptr : nci_phi(p, ws, sums, skip, s);
    hipLaunchKernelGGL((k_nci_round<KT>), dim3(nb), dim3(256), 0, s, U, static_cast<int64_t>(p.n), k,
                       (t == 1 || ph) ? nullptr : sums, ph, acc ? part : nullptr, labels, rpb, st, skip, t);
    TPO_LAUNCH_CHECK();
    if (acc) sum_parts_i64(part, nb, k * k + k, sums, s, skip, t >= 2 ? changed + (t - 1) : nullptr);
  }
}

void launch_nci(const Plan& p, void* ws, hipStream_t s) {
  switch ((p.k + 7) / 8) {
    case 1: nci_rounds<8>(p, ws, s); break;
    case 2: nci_rounds<16>(p, ws, s); break;
    case 3: nci_rounds<24>(p, ws, s); break;
    case 4: nci_rounds<32>(p, ws, s); break;
    default: nci_rounds_wide(p, ws, s); break;  // k > 32
  }
}

// ---------------------------------------------------------------------------
// Objective (Eq. obj1 with s ~ R R^T): cluster sums c_l of R rows in fixed
// point, then obj1 = sum_l c_l.(tot - c_l)/|C_l| and sum_l ||c_l||^2/|C_l|.
// ---------------------------------------------------------------------------
// Cluster sums of R rows (fixed point) and label counts for this workgroup's
// rows, over the column range [c0, c0 + cw) of blockIdx.y (the range is split
// so that the k x cw sums fit in LDS); counts by the y = 0 workgroups only.
// Written transposed: entry o (l * twod + j, then k * twod + l for counts) at
// part[o * gridDim.x + blockIdx.x].
constexpr int kObjLdsBytes = 128 * 1024;
constexpr int kObjRows = 8;

__global__ void __launch_bounds__(1024)
k_obj_accum(const float* __restrict__ R, int64_t n, int twod, const int32_t* __restrict__ labels, int k,
            int cw, long long* __restrict__ part, int rows_per_block, const DevStatus* __restrict__ st) {
  __shared__ long long accl[kObjLdsBytes / 8];  // k x cw sums, then k counts
  const int c0 = blockIdx.y * cw;
  const int cn = min(cw, twod - c0);
  long long* cntl = accl + k * cw;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int sft = fixed_point_shift(__uint_as_float(st->maxabs_r_bits), n);
  for (int e = tid; e < k * cw + k; e += blockDim.x) accl[e] = 0;
  __syncthreads();
  const int64_t rb = static_cast<int64_t>(blockIdx.x) * rows_per_block;
  const int64_t re = min(n, rb + rows_per_block);
  // a wave takes kObjRows rows at a time, all their loads issued before the
  // sums (cn <= 2d <= 256: four values of a row per lane)
  const int waves = blockDim.x >> 6;
  for (int64_t r0 = rb + static_cast<int64_t>(w) * kObjRows; r0 < re; r0 += static_cast<int64_t>(waves) * kObjRows) {
    int lab[kObjRows];
    float v[kObjRows][4];
#pragma unroll
    for (int u = 0; u < kObjRows; ++u) {
      const int64_t r = r0 + u;
      lab[u] = r < re ? labels[r] : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = lane + 64 * q;
        v[u][q] = (r < re && j < cn) ? R[r * twod + c0 + j] : 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < kObjRows; ++u) {
      if (r0 + u >= re) break;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = lane + 64 * q;
        if (j < cn)
          atomicAdd(reinterpret_cast<unsigned long long*>(&accl[lab[u] * cw + j]),
                    static_cast<unsigned long long>(to_fixed(v[u][q], sft)));
      }
      if (lane == 0 && blockIdx.y == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&cntl[lab[u]]), 1ull);
    }
  }
  __syncthreads();
  for (int e = tid; e < k * cn; e += blockDim.x) {
    const int l = e / cn, j = e - (e / cn) * cn;
    part[static_cast<int64_t>(l * twod + c0 + j) * gridDim.x + blockIdx.x] = accl[l * cw + j];
  }
  if (blockIdx.y == 0)
    for (int l = tid; l < k; l += blockDim.x)
      part[static_cast<int64_t>(k * twod + l) * gridDim.x + blockIdx.x] = cntl[l];
}

__global__ void __launch_bounds__(1024)
k_obj_final(const long long* __restrict__ acc, int k, int twod, int64_t n, DevStatus* __restrict__ st) {
  const long long* cnt = acc + k * twod;
  __shared__ double red[1024];
  __shared__ double tot[512];
  const int sft = fixed_point_shift(__uint_as_float(st->maxabs_r_bits), n);
  const double inv = ldexp(1.0, -sft);
  for (int j = threadIdx.x; j < twod; j += blockDim.x) {
    long long s = 0;
    for (int l = 0; l < k; ++l) s += acc[l * twod + j];
    tot[j] = static_cast<double>(s) * inv;
  }
  __syncthreads();
  double o = 0.0, t = 0.0;
  for (int idx = threadIdx.x; idx < k * twod; idx += blockDim.x) {
    const int l = idx / twod, j = idx % twod;
    if (cnt[l] <= 0) continue;
    const double c = static_cast<double>(acc[idx]) * inv;
    o += c * (tot[j] - c) / cnt[l];
    t += c * c / cnt[l];
  }
  o = blk_sum(o, red);
  t = blk_sum(t, red);
  if (threadIdx.x == 0) {
    st->objective[0] = o;
    st->objective[1] = t;
  }
}

void launch_objective(const Plan& p, void* ws, hipStream_t s) {
  DevStatus* st = bufp<DevStatus>(p, ws, B_STATUS);
  long long* part = bufp<long long>(p, ws, B_OBJ_PART);
  long long* sums = bufp<long long>(p, ws, B_OBJ_SUM);
  const int k = p.k, twod = p.twod;
  const int nb = p.obj_blocks;
  const int rpb = static_cast<int>((p.n + nb - 1) / nb);
  const int cw = std::min(twod, (kObjLdsBytes / 8 - k) / k);  // columns per LDS pass
  const int ny = (twod + cw - 1) / cw;
  hipLaunchKernelGGL(k_obj_accum, dim3(nb, ny), dim3(1024), 0, s, bufp<float>(p, ws, B_R), static_cast<int64_t>(p.n),
                     twod, bufp<int32_t>(p, ws, B_LABELS), k, cw, part, rpb, st);
  TPO_LAUNCH_CHECK();
  sum_parts_i64(part, nb, k * twod + k, sums, s);
  hipLaunchKernelGGL(k_obj_final, dim3(1), dim3(1024), 0, s, sums, k, twod, static_cast<int64_t>(p.n), st);
  TPO_LAUNCH_CHECK();
}

}  // namespace tpo
