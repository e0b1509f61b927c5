/*
 * tpo.h - C ABI of the MI355X (gfx950) implementation of TPO, the three-phase
 * k-clustering method for attributed bipartite graphs (ABGs) of
 * "Effective Clustering on Large Attributed Bipartite Graphs" (KDD 2024).
 *
 * One call clusters the target node set U of an ABG G = (U u V, E, X_U) into
 * k disjoint clusters (Definition 1, the k-ABGC problem): edges, attributes,
 * k and the propagation parameters go in; cluster labels, the k-dimensional
 * embedding and the objective of Eq. obj1 come out.
 *
 * Conventions for every entry point:
 *  - Plain pointers and sizes only.  "device" pointers are HIP device
 *    addresses on the current device; "host" pointers are ordinary memory.
 *  - The caller owns every input, output and workspace buffer.  The library
 *    never allocates device memory (no hipMalloc); a plan owns host metadata
 *    only.  (tpo_execute_noalloc uses a fixed device array of the library's
 *    own instead of a caller workspace.)  Inputs are read-only and not
 *    retained after a call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; tpo_execute synchronises it before returning.
 *  - All arguments are validated before the first launch; on error nothing
 *    is written to the outputs and tpo_plan_last_error() explains.  Distinct
 *    plans may be used from different threads; one plan is not reentrant.
 *  - Matrices are row-major.  Sizes are elements unless stated otherwise.
 */
#ifndef TPO_H_
#define TPO_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPO_ABI_VERSION 3

typedef enum tpo_status {
  TPO_OK = 0,
  TPO_EINVAL = 1,   /* bad shape or parameter, ABI version mismatch */
  TPO_ERANGE = 2,   /* edge endpoint out of range, negative/non-finite weight */
  TPO_ENOMEM = 3,   /* workspace smaller than tpo_plan_workspace_bytes() */
  TPO_EDEVICE = 4,  /* HIP runtime error, or no gfx950 device */
  TPO_ENUMERIC = 5  /* non-finite attributes, R'[i].r <= 0 (Eq. Ri), or a
                       Cholesky breakdown in an orthonormalisation */
} tpo_status;

/* Shape of one clustering job: the ABG model of Section 2.1. */
typedef struct tpo_problem {
  int32_t abi_version; /* TPO_ABI_VERSION */
  int32_t n_u;         /* |U| >= 1, the target node set */
  int32_t n_v;         /* |V| >= 1 */
  int32_t d_u;         /* attribute width of X_U, 1..4096 */
  int64_t n_edges;     /* entries of the edge list, 0 <= n_edges < 2^31;
                          a (u, v) pair listed twice adds its weights (B_U[i,j]
                          is the summed weight) */
  int32_t weighted;    /* 1: tpo_inputs.edge_w is given; 0: every w = 1 */
  int32_t x_dtype;     /* element type of tpo_inputs.x_u: TPO_X_F32,
                          TPO_X_BF16 or TPO_X_FP8 (the attribute precision
                          forms: the Gram C = X^T X of Section 3.2.1 on BF16
                          or FP8 MFMA with FP32 accumulation, added up in
                          FP64; the projection reads the narrow type and
                          multiplies in FP32), or TPO_X_CSR (sparse FP32
                          attributes, see below) */
  int64_t x_nnz;       /* TPO_X_CSR: stored entries of X_U, 0 <= x_nnz <
                          2^31; ignored otherwise */
} tpo_problem;

#define TPO_X_F32 0
#define TPO_X_BF16 1 /* bfloat16: the upper 16 bits of an IEEE binary32 */
#define TPO_X_FP8 2  /* OCP FP8 E4M3 (exponent bias 7, no infinities, 0x7F and
                        0xFF are NaN) with one FP32 scale per column: the
                        attribute is decode(x_u[i][j]) * x_scale[j] */
#define TPO_X_CSR 3  /* sparse FP32 attributes in CSR (tpo_inputs.x_rowptr,
                        x_col, and x_u holding the FP32 values), for sparse
                        text attributes such as TF-IDF rows.  With the
                        reduction on, the Gram C = X^T X (Section 3.2.1) is
                        formed on FP8 MFMA: row groups are densified into a
                        staging tile as OCP E4M3 codes of x / s_j with one
                        scale s_j = max_i |x_ij| / 448 per column (round to
                        nearest even), FP32 sums per 64-row slab added in
                        FP64.  FP32 refinement steps follow the subspace
                        iteration on that Gram (tpo_params.x_refine): the
                        Rayleigh-Ritz product, and the power steps before it,
                        are taken with the exact attributes, P = X^T (X M).
                        The projection X' = X Psi_d and
                        the column sums read the exact FP32 values.  Without
                        the reduction the rows are copied densely. */

/* Method parameters: Table 1 of the paper plus the unstated RandomizedSVD
 * details.  Defaults used in the paper: t_f = 5, t_g = 20. */
typedef struct tpo_params {
  int32_t abi_version; /* TPO_ABI_VERSION */
  int32_t k;           /* clusters, 1 <= k <= 128 and k <= 2 d_eff */
  double alpha;        /* balance coefficient of Eq. Z-obj, 0 <= alpha < 1 */
  int32_t gamma;       /* propagation hops of Eq. PX, 0..1000 */
  int32_t d;           /* reduced attribute width of Section 3.2.1; 0 or
                          d >= d_u disables the reduction (d_eff = d_u) */
  int32_t q;           /* power iterations of both randomized SVDs, 0..100 */
  int32_t oversample;  /* p: sketch width k' = min(k + p, 2 d_eff) for
                          RandomizedSVD(R, k), l_r = min(d + p, d_u) for the
                          reduction; 0..64 */
  int32_t t_f;         /* ONMF rounds (Algorithm 2), 0..1000 */
  int32_t t_g;         /* NCI rounds (Algorithm 3), 0..1000 */
  int32_t flags;       /* TPO_FLAG_* */
  uint64_t seed;       /* seeds the Gaussian matrices not given below */
  /* Optional host matrices (row-major float64).  NULL: drawn from `seed`
   * with the library's SplitMix64 + Box-Muller generator, streams 0, 1, 2
   * (see tpo_draw_normals). */
  const double* omega_reduce; /* d_u x l_r sketch of the reduction */
  const double* g;            /* d_eff x d_eff matrix G of Algorithm 1 */
  const double* omega;        /* 2 d_eff x k' sketch of RandomizedSVD(R, k) */
  int32_t x_refine;           /* TPO_X_CSR with the reduction on: refinement
                                 steps with the exact FP32 attributes after
                                 the iteration on the FP8 Gram, 0..8.  Each
                                 step forms P = X^T (X M); the last feeds the
                                 Rayleigh-Ritz step, earlier ones are further
                                 power steps (M <- orth(P)).  0: none, the
                                 Rayleigh-Ritz product is the FP8 Gram's. */
  int32_t reserved;
} tpo_params;

#define TPO_FLAG_TIMING 1 /* record per-stage device times (tpo_plan_stats) */
#define TPO_FLAG_ONE_STREAM 2 /* run everything on the caller's stream: no
                                 plan-owned second stream for ingest (for
                                 callers that overlap many jobs instead) */
#define TPO_FLAG_NCI_PROCRUSTES 4 /* NCI (Algorithm 3) with Phi <- the orthogonal
                                     polar factor of Ups^T Y, the minimiser over
                                     orthogonal Phi of ||Ups Phi - Y||_F that
                                     Section 3.4 describes, instead of the
                                     printed Phi <- Ups^T Y; an empty cluster's
                                     zero column stays zero (the polar factor
                                     of the other columns) */

/* Inputs of one job (device memory unless stated). */
typedef struct tpo_inputs {
  const int32_t* edge_u; /* [n_edges] endpoint in U, 0 <= u < n_u */
  const int32_t* edge_v; /* [n_edges] endpoint in V, 0 <= v < n_v */
  const float* edge_w;   /* [n_edges] weights >= 0, or NULL when unweighted */
  const void* x_u;       /* X_U: n_u rows of ld_x elements of type
                            tpo_problem.x_dtype, first d_u used */
  int64_t ld_x;          /* row stride of x_u in elements, >= d_u */
  const float* x_scale;  /* [d_u] column scales, device memory; required with
                            TPO_X_FP8 (EINVAL if NULL), ignored otherwise */
  const int64_t* x_rowptr; /* TPO_X_CSR: [n_u + 1] row starts, x_rowptr[0] = 0,
                              non-decreasing, x_rowptr[n_u] = x_nnz */
  const int32_t* x_col;    /* TPO_X_CSR: [x_nnz] column of each stored entry,
                              0 <= col < d_u (entries of one row in any order;
                              a column listed twice in a row adds up) */
} tpo_inputs;

/* Outputs of one job. */
typedef struct tpo_outputs {
  int32_t* labels;    /* device [n_u]: cluster of each u, in 0..k-1 */
  float* embedding;   /* device [n_u x k] row-major: Upsilon of Algorithm 2,
                         or NULL */
  double* objective;  /* host [2] or NULL: obj1 of Eq. obj1 with
                         s(u_i,u_j) ~ R[i].R[j], and Tr(Y^T R R^T Y) */
} tpo_outputs;

/* Per-stage device milliseconds of the last tpo_execute with TPO_FLAG_TIMING. */
typedef struct tpo_stats {
  double ms_ingest, ms_reduce, ms_propagate, ms_features, ms_embed, ms_onmf,
      ms_nci, ms_objective, ms_total;
  int64_t n_unique_edges; /* distinct (u, v) pairs after summing duplicates */
  int32_t guard_hits;     /* ONMF guard applications (zero denominators,
                             negative ratios) */
  int32_t isolated_u, isolated_v;
  /* Propagation SpMM row kernels (hub-chunk finalisation excluded), summed
   * over the first min(gamma, 64) hops: V side (T = D_V^-1 B^T W) and U side
   * (Z = X' + alpha D_U^-1/2 B T), milliseconds and launch counts. */
  double ms_spmm_v, ms_spmm_u;
  int32_t n_spmm_v, n_spmm_u;
  /* NCI with k > 32 scores on FP32 MFMA; rows whose two best scores lie
   * within the FP32 error bound are scored again in FP64.  How many, summed
   * over the rounds. */
  int32_t nci_rechecked;
  /* NCI rounds run: T_g, or fewer when the label sums of a round equal those
   * of the round before (Algorithm 3 then repeats that round's labels and
   * Phi in every later round, so the rest are skipped on the device). */
  int32_t nci_rounds;
} tpo_stats;

typedef struct tpo_plan tpo_plan;

/* Validate the job shape and parameters and build a plan (host metadata only:
 * sizes, workspace layout, the Gaussian matrices).  The plan keeps copies of
 * the optional matrices.  Errors: TPO_EINVAL. */
tpo_status tpo_plan_create(const tpo_problem* problem, const tpo_params* params,
                           tpo_plan** out_plan);

/* Bytes of device workspace tpo_execute and the stage calls need (256-byte
 * alignment required for the workspace base). */
tpo_status tpo_plan_workspace_bytes(const tpo_plan* plan, size_t* out_bytes);

/* Run the whole method (Section 3: optional attribute reduction, Algorithms
 * 1, 2 and 3, then Eq. obj1) on `stream`, then synchronise it.
 * `workspace` is device memory of at least tpo_plan_workspace_bytes(); its
 * contents on entry do not matter and on return hold the intermediates
 * described by tpo_plan_buffer.  Errors: TPO_EINVAL (NULL pointers),
 * TPO_ENOMEM, TPO_ERANGE (found on the device; outputs then unspecified),
 * TPO_ENUMERIC, TPO_EDEVICE. */
tpo_status tpo_execute(tpo_plan* plan, const tpo_inputs* in, void* workspace,
                       size_t workspace_bytes, void* stream,
                       const tpo_outputs* out);

/* tpo_execute for a job whose graph is already in `workspace`: the CSR,
 * degrees and hub lists that the last tpo_execute or tpo_stage_ingest of a
 * plan of the same shape built in this workspace are reused, and ingest (S0)
 * is skipped; tpo_inputs' edge arrays are not read.  For serving many jobs
 * on one graph, whose CSR then stays in HBM between jobs.  The caller
 * guarantees that this job's edge list is the one ingested last into the
 * workspace; a workspace without a finished ingest of this plan's shape
 * (n_u, n_v, n_edges) gives TPO_EINVAL.  Other arguments and errors as for
 * tpo_execute. */
tpo_status tpo_execute_resident(tpo_plan* plan, const tpo_inputs* inputs,
                                void* workspace, size_t workspace_bytes,
                                void* stream, const tpo_outputs* outputs);

void tpo_plan_destroy(tpo_plan* plan);
const char* tpo_status_string(tpo_status status);
const char* tpo_plan_last_error(const tpo_plan* plan);
tpo_status tpo_plan_stats(const tpo_plan* plan, tpo_stats* out);

/* The sizes the plan derived: d_eff, the reduction sketch width l_r (0 when
 * no reduction), the embedding sketch width k'. */
tpo_status tpo_plan_dims(const tpo_plan* plan, int32_t* d_eff, int32_t* l_r,
                         int32_t* k_prime);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): tpo_execute
 * with the workspace taken from a device array of TPO_NOALLOC_MAX_BYTES that
 * the library holds on each GPU it runs on until the process ends.  The
 * caller still passes inputs and outputs as for tpo_execute; the kernels are
 * the same.  Calls no hipMalloc/hipFree and creates no stream or event: the
 * plan must not have TPO_FLAG_TIMING (TPO_EINVAL), and everything runs on
 * `stream`, which is synchronised before returning.  A job whose
 * tpo_plan_workspace_bytes() exceeds TPO_NOALLOC_MAX_BYTES gets TPO_ENOMEM
 * before any device work.  All calls on one GPU share that GPU's array,
 * which keeps the last call's contents: calls that overlap on one GPU race
 * and must be serialised by the caller.  Other errors as tpo_execute; after
 * the call, tpo_plan_buffer on the array is not available. */
#define TPO_NOALLOC_MAX_BYTES ((size_t)64 << 20)
tpo_status tpo_execute_noalloc(tpo_plan* plan, const tpo_inputs* in, void* stream,
                               const tpo_outputs* out);

/* ---- Stage entry points -------------------------------------------------
 * tpo_execute is exactly these calls in this order.  Each works on the
 * buffers of `workspace` named by tpo_plan_buffer, so a caller can read an
 * intermediate after a stage, or overwrite a stage's input buffer before
 * calling it.  They enqueue on `stream` and do not synchronise (except
 * tpo_stage_objective, which returns host values). */

/* Section 2.1: CSR of B_U (rows U) and of its transpose (rows V) with
 * duplicates summed and columns ascending, weighted degrees D_U, D_V and the
 * scale vectors of the propagation.  Reads in->edge_*. */
tpo_status tpo_stage_ingest(tpo_plan* plan, const tpo_inputs* in, void* workspace,
                            size_t workspace_bytes, void* stream);
/* Section 3.2.1, Eq. Xd: X' = X Psi_d (top-d right singular vectors of X by
 * randomized subspace iteration on X^T X), or X' = X when d_eff = d_u.
 * Reads in->x_u. */
tpo_status tpo_stage_reduce(tpo_plan* plan, const tpo_inputs* in, void* workspace,
                            size_t workspace_bytes, void* stream);
/* Algorithm 1, Eq. PX: Z = (1-alpha) sum_{r<=gamma} alpha^r
 * (L L^T)^r X' by gamma hops of two CSR SpMMs. */
tpo_status tpo_stage_propagate(tpo_plan* plan, const tpo_inputs* in, void* workspace,
                               size_t workspace_bytes, void* stream);
/* Algorithm 1, Eqs. Z, R-prime, Ri: R from Z and Q = QR(G). */
tpo_status tpo_stage_features(tpo_plan* plan, void* workspace, size_t workspace_bytes,
                              void* stream);
/* Algorithm 2 and Eq. init-HY: RandomizedSVD(R, k) -> Gamma, Sigma,
 * Psi (column sign convention: positive column sums of Gamma). */
tpo_status tpo_stage_embed(tpo_plan* plan, void* workspace, size_t workspace_bytes,
                           void* stream);
/* Algorithm 2, Eqs. update-Q and update-Y: Upsilon, H. */
tpo_status tpo_stage_onmf(tpo_plan* plan, void* workspace, size_t workspace_bytes,
                          void* stream);
/* Algorithm 3: labels from Upsilon (device [n_u], may be the workspace's own
 * label buffer when `labels` is NULL). */
tpo_status tpo_stage_nci(tpo_plan* plan, void* workspace, size_t workspace_bytes,
                         void* stream, int32_t* labels);
/* Eq. obj1 and the trace form for the labels in the workspace; synchronises
 * `stream` and writes objective[0..1] (host). */
tpo_status tpo_stage_objective(tpo_plan* plan, void* workspace, size_t workspace_bytes,
                               void* stream, double* objective);

/* Buffers of the workspace, for stage-by-stage inspection. */
typedef enum tpo_buffer_id {
  TPO_BUF_ROWPTR_U = 0, /* int32 [n_u + 1]  CSR of B_U */
  TPO_BUF_COL_U = 1,    /* int32 [n_edges]  first n_unique entries valid */
  TPO_BUF_VAL_U = 2,    /* float [n_edges]  summed weights (valid when the
                           input is weighted or has duplicates) */
  TPO_BUF_ROWPTR_V = 3, /* int32 [n_v + 1]  CSR of B_U^T */
  TPO_BUF_COL_V = 4,
  TPO_BUF_VAL_V = 5,
  TPO_BUF_DEG_U = 6,    /* float [n_u] D_U */
  TPO_BUF_DEG_V = 7,    /* float [n_v] D_V */
  TPO_BUF_XPRIME = 8,   /* float [n_u x d_pad] X' (d_pad: d_eff rounded up to a
                           power of two >= 16; padding columns are zero) */
  TPO_BUF_PSI_D = 9,    /* double [d_u x d_eff] Psi_d (reduction on) */
  TPO_BUF_Z = 10,       /* float [n_u x d_pad] Z of Eq. PX */
  TPO_BUF_Q = 11,       /* double [d_eff x d_eff] Q of Algorithm 1 */
  TPO_BUF_R = 12,       /* float [n_u x 2 d_eff] R of Eq. Ri */
  TPO_BUF_GAMMA = 13,   /* float [n_u x k] Gamma */
  TPO_BUF_SIGMA = 14,   /* double [k] */
  TPO_BUF_PSI = 15,     /* double [2 d_eff x k] */
  TPO_BUF_UPSILON = 16, /* float [n_u x k] */
  TPO_BUF_H = 17,       /* double [2 d_eff x k] */
  TPO_BUF_LABELS = 18,  /* int32 [n_u] */
  TPO_BUF_T = 19,       /* float [n_v x d_pad] T = D_V^-1 B^T W of the last hop */
  TPO_BUF_W_LAST = 20,  /* float [n_u x d_pad] W = D_U^-1/2 Z that fed the last
                           hop (gamma >= 1) */
  TPO_BUF_SCALE_U = 21, /* float [n_u] D_U^-1/2 (0 for isolated nodes) */
  TPO_BUF_SCALE_V = 22, /* float [n_v] D_V^-1 (0 for isolated nodes) */
  TPO_BUF_RSUM = 23,    /* double [2 d_eff] r = sum_i R'_i (Eq. Ri) */
  TPO_BUF_S = 24,       /* double [2 d_eff x k] S with Gamma = R S */
  TPO_BUF_GRAM_C = 25,  /* double [d_u x d_u] C = X^T X of the reduction
                           (EINVAL when the reduction is off) */
  TPO_BUF_COLSUM_X = 26, /* double [d_u] column sums of X (reduction on) */
  TPO_BUF_COUNT
} tpo_buffer_id;

#define TPO_DTYPE_I32 1
#define TPO_DTYPE_F32 2
#define TPO_DTYPE_F64 3

/* Device address (inside `workspace`), shape and dtype of buffer `which`. */
tpo_status tpo_plan_buffer(const tpo_plan* plan, void* workspace, int32_t which,
                           void** ptr, int64_t* rows, int64_t* cols,
                           int32_t* dtype);

/* The library's Gaussian generator (host): SplitMix64 (Steele, Lea and Flood
 * 2014) from state seed ^ (0x632BE59BD9B4E019 * (stream + 1)), pairs of
 * outputs mapped to 53-bit uniforms on (0, 1] and to two normals by the
 * Box-Muller transform.  Writes `count` doubles to host memory `out`. */
tpo_status tpo_draw_normals(uint64_t seed, int32_t stream, int64_t count, double* out);

/* The OCP FP8 E4M3 (e4m3fn) code the TPO_X_CSR form stages for the value v
 * (x_ij / s_j): round to nearest even, saturating at +-448, 0x7F for NaN.
 * Host function, for reproducing the staged codes. */
uint8_t tpo_e4m3_encode(float v);

int32_t tpo_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TPO_H_ */
