// Internal declarations shared by the host orchestration (tpo_api.cpp) and the
// HIP kernel files: the workspace layout of a plan and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tpo.h"

namespace tpo {

// Edges per hub chunk of the propagation SpMM: rows with more neighbours than
// this are split into chunks whose partial sums are added in chunk order.
constexpr int kHubChunk = 256;
// Workgroups that walk the hub chunks and the hub rows of one SpMM launch
// (grid-stride loops over the counts that ingest finds; 8192 waves fill the
// GPU).
constexpr int kHubBlocks = 2048;
// Radix sort tile: 512 threads x 16 keys (8,192 keys: runs of 32 keys per
// digit on average when a tile is scattered).
constexpr int kSortThreads = 512;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
// Rows per workgroup chunk of the FP64 Gram kernels.
constexpr int kGramRowsPerChunk = 2048;
// Rows per workgroup of the row-pass kernels.
constexpr int kRowPassRows = 1024;
// Hops whose SpMM kernels are bracketed by events when timing is on.
constexpr int kMaxTimedHops = 64;

// Device-side status words (one small block, copied back at the end of a job).
struct DevStatus {
  int32_t err_bits;        // bit 0: edge out of range, bit 1: bad weight,
                           // bit 2: non-finite attribute, bit 3: R'.r <= 0,
                           // bit 4: Cholesky breakdown, bit 5: non-finite value,
                           // bit 6: grid barrier timed out, bit 7: sparse
                           // attribute row starts or columns out of range
  int32_t has_vals;        // CSR carries a value array (weights / duplicates)
  int32_t n_unique;        // distinct (u, v) pairs
  int32_t guard_hits;      // ONMF guards applied
  int32_t iso_u, iso_v;    // isolated nodes
  int32_t hub_chunks_u, hub_rows_u, hub_chunks_v, hub_rows_v;
  uint32_t maxabs_r_bits;  // max |R| as float bits
  uint32_t maxabs_ups_bits;// max |Upsilon| as float bits
  double objective[2];
  int32_t nci_rechecked;   // NCI rows scored again in FP64
  int32_t nci_rounds;      // the last NCI round run (later ones repeat it)
};

// The ingested graph's part of the status block, kept in the workspace
// (B_GSTATUS) so that a later job on the same workspace and edge list can
// skip ingest (tpo_execute_resident).  magic and the shape say that the
// workspace holds a finished ingest of this plan's shape.
constexpr int32_t kGraphMagic = 0x54504F47;
struct GraphStatus {
  int32_t magic;
  int32_t n, m;
  int32_t n_edges;
  int32_t has_vals, n_unique, iso_u, iso_v;
  int32_t hub_chunks_u, hub_rows_u, hub_chunks_v, hub_rows_v;
  int32_t err_bits;  // ingest's bits (edge range, weights)
  int32_t pad;
};

enum Buf {
  B_STATUS, B_GSTATUS,
  // ingest
  B_KEYS_A, B_KEYS_B, B_WV_A, B_WV_B, B_HIST, B_SCAN_AUX, B_UPOS,
  B_ROWPTR_U, B_COL_U, B_VAL_U, B_ROWPTR_V, B_COL_V, B_VAL_V,
  B_DEG_U, B_DEG_V, B_ISQ_U, B_INV_V,
  B_HUBCNT_U, B_HUBCNT_V,         // per-row chunk counts / scans (n+1, m+1)
  B_HUBROW_U, B_HUBROW_V,         // per-row hub index scans (n+1, m+1)
  B_CHUNK_U, B_CHUNK_V,           // int4 {row, begin, end, slot} per chunk
  B_HUBLIST_U, B_HUBLIST_V,       // int4 {row, slot_begin, nchunks, 0} per hub row
  B_PARTIAL,                      // hub chunk partial sums (max chunks x d)
  // reduce
  B_GRAM_PART, B_COLSUM_PART, B_C, B_COLSUM_X, B_MR_A, B_MR_B, B_SMALL_A,
  B_SMALL_B, B_SMALL_C, B_EVAL, B_PSI_D, B_PSI_D32, B_PSI_SPLIT, B_XPRIME,
  // propagate
  B_W0, B_W1, B_T, B_Z,
  // features
  B_G, B_Q, B_QT32, B_R, B_RPART, B_RSUM, B_RCOLSUM,
  // embed
  B_OMEGA, B_K, B_M_A, B_M_B, B_EK_A, B_EK_B, B_EK_C, B_JLOG, B_EEVAL, B_S32,
  B_GAMMA, B_SIGMA, B_PSI, B_OMR,
  // onmf
  B_UPS, B_H, B_H32, B_H_NEW, B_RTU, B_UTU, B_A32, B_ONMF_PART,
  // nci / objective
  B_LABELS, B_NCI_PART, B_NCI_SUM, B_NCI_PHI, B_NCI_PM, B_NCI_PV, B_NCI_CHECK, B_OBJ_PART, B_OBJ_SUM,
  // subspace iteration (reduction and embedding)
  B_SI_M, B_SI_P, B_SI_GRAM, B_SI_PART, B_SI_BAR,
  B_REDTMP,
  // sparse attributes (TPO_X_CSR): column scales and maxima, the FP8 staging
  // tile, the transpose (CSC) and its sort buffers, the column-chunk table
  // and partials, and Y = X M of the refinement step
  B_XS_SCALE, B_XS_COLMAX, B_XS_STAGE, B_XT_KA, B_XT_KB, B_XT_VA, B_XT_VB, B_XT_HIST, B_XT_AUX,
  B_XT_COLPTR, B_XT_ROW, B_XT_CHUNK, B_XT_CINFO, B_XT_CPART, B_XT_Y,
  B_COUNT
};

struct Layout {
  size_t off[B_COUNT];
  size_t bytes[B_COUNT];
  size_t total;
};

struct Plan {
  tpo_problem prob;
  tpo_params par;
  int n, m, du, d, dp, lr, kp, k, twod;
  int64_t E;
  bool reduce;
  bool xbf16;  // X_U is bfloat16
  bool xfp8;   // X_U is FP8 E4M3 with column scales
  bool xcsr;   // X_U is sparse FP32 (CSR)
  int64_t xnnz;        // stored entries of a sparse X_U
  int xsort_blocks;    // radix-sort tiles of the transpose of a sparse X_U
  int xstage_rows;     // rows of the FP8 staging tile
  int64_t xchunks_max; // column chunks of the transpose, upper bound
  int rowbits, colbits;
  int sort_blocks;          // tiles of the radix sort
  int max_chunks_u, max_chunks_v;
  int gram_chunks_x, gram_chunks_r;
  int rowpass_blocks;
  int obj_blocks;  // blocks of the objective accumulation
  std::vector<double> omega_r, g, omega;
  Layout lay;
  std::string last_error;
  tpo_stats stats;
  hipEvent_t ev[10];
  bool events_made;
  bool timing;             // TPO_FLAG_TIMING set
  hipEvent_t kev[4 * kMaxTimedHops];
  bool kev_made;
  // second stream: ingest runs beside the attribute reduction
  hipStream_t side;
  hipEvent_t fork_ev, join_ev;
  bool side_made;
  DevStatus init_status;  // host copy uploaded at the start of a job
  DevStatus host_status;  // last status block read back
};

// the attribute Gram runs on the narrow-type kernel (128 x 128 tile pairs)
inline bool narrow_gram(const Plan& p) { return p.xbf16 || p.xfp8 || p.xcsr; }

// The rotation log of the Jacobi eigensolvers that run without eigenvectors
// (the reduction's Rayleigh-Ritz for l <= 80, the embedding finish for k' in
// 81..128): the (c, s) of every pair of every step run, the steps' indices,
// their count, then the eigenvalue order.
constexpr int kJacobiLogSweeps = 40;
struct JacobiLog {
  double2* rot;
  int* steps;
  int* count;
  int* perm;  // 128
};
int jacobi_log_n(const Plan& p);  // the largest order logged (0: none)
inline size_t jacobi_log_steps(int n) {
  const int np = n + (n & 1);
  return static_cast<size_t>(kJacobiLogSweeps) * static_cast<size_t>(np > 1 ? np - 1 : 1);
}
inline size_t jacobi_log_bytes(int n) {
  const int np = n + (n & 1);
  return sizeof(double2) * jacobi_log_steps(n) * static_cast<size_t>(np / 2 > 0 ? np / 2 : 1) +
         sizeof(int) * (jacobi_log_steps(n) + 1 + 128) + 64;
}

template <typename T>
inline T* bufp(const Plan& p, void* ws, Buf b) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + p.lay.off[b]);
}

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).  All enqueue on `s`.
// ---------------------------------------------------------------------------
// k_ingest.hip
void launch_ingest(const Plan& p, void* ws, const tpo_inputs* in, hipStream_t s);
// sparse attributes: the transpose (CSC) of X_U into B_XT_* (k_ingest.hip)
void xcsr_transpose(const Plan& p, void* ws, const int64_t* rowptr, const int32_t* col, const float* val,
                    hipStream_t s);
// k_xsparse.hip: the column chunks of the transpose (after xcsr_transpose);
// column scales into B_XS_SCALE; rows [r0, r0 + rows) as E4M3 codes into
// B_XS_STAGE (row stride ld, groups staged in row order); out = X B (FP64
// sums, FP32 out, zero columns lb..wo); P = X^T Y (ldp, or no P when NULL)
// and the column sums of X from the transpose; dense rows without the
// reduction.
constexpr int kXMaxDu = 4096;
// row stride (bytes) of the FP8 staging tile of a sparse X_U: 16-byte rows
inline int xcsr_stage_ld(int du) { return (du + 15) / 16 * 16; }
// column tile of the narrow-type (BF16, FP8) Gram partials
constexpr int kNarrowTile = 128;
void xcsc_make_chunks(const Plan& p, void* ws, hipStream_t s);
void xcsr_scales(const Plan& p, void* ws, hipStream_t s);
void xcsr_stage_fp8(const Plan& p, void* ws, int64_t r0, int rows, int ld, hipStream_t s);
void xcsr_rowgather(const Plan& p, const int64_t* rowptr, const int32_t* col, const float* val, const double* B,
                    int lb, int ldb, float* out, int ldo, int wo, hipStream_t s);
void xcsc_colgather(const Plan& p, void* ws, const float* Y, int l, int ldy, double* P, int ldp, double* colsum,
                    hipStream_t s);
void xcsr_dense(const Plan& p, void* ws, const int64_t* rowptr, const int32_t* col, const float* val, float* xp,
                hipStream_t s);
// after ingest: its status fields and the graph's shape into B_GSTATUS; for
// a resident job: those fields back into B_STATUS (k_ingest.hip)
void save_graph_status(const Plan& p, void* ws, hipStream_t s);
void restore_graph_status(const Plan& p, void* ws, hipStream_t s);
// k_spmm.hip
void launch_propagate(const Plan& p, void* ws, const float* xprime, int64_t ldxp,
                      hipStream_t s);
// k_dense.hip
void launch_reduce(const Plan& p, void* ws, const tpo_inputs* in, hipStream_t s);
void launch_features(const Plan& p, void* ws, hipStream_t s);
void launch_embed(const Plan& p, void* ws, hipStream_t s);
// k_smallla.hip (single workgroup, small matrices in LDS, n <= 80)
constexpr int kLdsMaxN = 80;
void cholqr_lds(double* A, int m, int n, int lda, int32_t* err_bits, hipStream_t s);
// n_orth Cholesky-QR steps of subspace iteration on the symmetric N x N A from
// the N x l start omega (l <= 128); m_out = the last basis (omega when
// n_orth = 0), p_out = A m_out.  pa, pb: N x l scratch; gram:
// subspace_gsum_doubles(l) scratch; part: subspace_part_doubles(N, l) scratch.
// bar: two words of scratch for the grid barrier.  One launch.
void subspace_iterate(const double* A, int N, const double* omega, int l, int n_orth, double* pa, double* pb,
                      double* gram, double* part, unsigned* bar, double* m_out, double* p_out, int32_t* err_bits,
                      hipStream_t s);
size_t subspace_part_doubles(int N, int l);
size_t subspace_gsum_doubles(int l);
void rr_reduce_lds(double* M, const double* P, int du, int l, int d, int dp, const double* colsum_x, int64_t n,
                   double* evals, double* psi, float* psi32, JacobiLog jlog, hipStream_t s);
JacobiLog jacobi_log(const Plan& p, void* ws);
void embed_final_lds(double* M, double* P, int twod, int kp, int k, const double* colsum_r, int64_t n, double* S,
                     float* S32, double* sigma, double* psi, double* H, float* H32, int32_t* err_bits,
                     hipStream_t s);
constexpr int kWideMaxN = 128;
// k' in 81..128: the same in three steps, the Jacobi's rotations logged in
// jlog and applied to the rows of M and P afterwards
void embed_final_wide(double* M, double* P, int twod, int kp, int k, const double* colsum_r, int64_t n, double* S,
                      float* S32, double* sigma, double* psi, double* H, float* H32, JacobiLog jlog,
                      int32_t* err_bits, hipStream_t s);
// deterministic two-level sum of nparts rows of length len (k_dense.hip)
void reduce_parts(const double* part, int nparts, int len, double* tmp, double* out, hipStream_t s);
// k_cluster.hip
// emb_out: also written with Upsilon by the last ONMF round (or null)
void launch_onmf(const Plan& p, void* ws, hipStream_t s, float* emb_out = nullptr);
void launch_nci(const Plan& p, void* ws, hipStream_t s);
void launch_objective(const Plan& p, void* ws, hipStream_t s);

}  // namespace tpo

// The opaque plan handle of the C ABI.
struct tpo_plan : public tpo::Plan {};

namespace tpo {
// The body of tpo_execute: validates, runs the whole method for `plan` on `s`
// in the workspace `ws` and synchronises `s`.  no_alloc: everything runs on
// `s` with no plan-owned second stream and no events (plans with
// TPO_FLAG_TIMING are rejected), for callers that must not create runtime
// objects.
tpo_status execute_plan(tpo_plan* plan, const tpo_inputs* in, void* ws, size_t bytes, hipStream_t s,
                        const tpo_outputs* out, bool no_alloc, bool resident = false);
// Records `msg` as the plan's last error and returns `st`.
tpo_status plan_fail(tpo_plan* plan, tpo_status st, const std::string& msg);
}  // namespace tpo
