// C ABI of the TPO library: validation, plans, workspace layout, the Gaussian
// generator, and the stage sequence of Section 3 (reduction, Algorithm 1,
// Algorithm 2, Algorithm 3, Eq. obj1) enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>

#include "dev_common.hpp"
#include "tpo_internal.hpp"

using namespace tpo;

namespace {

constexpr int kMaxK = 128;
constexpr int kMaxDEff = 128;
constexpr int kMaxDu = 4096;

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

int bits_for(int64_t n) {
  int b = 1;
  while ((int64_t{1} << b) < n) ++b;
  return b;
}

int next_pow2_at_least(int x, int lo) {
  int p = lo;
  while (p < x) p <<= 1;
  return p;
}

// SplitMix64 (Steele, Lea and Flood 2014).
uint64_t splitmix_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void draw_normals(uint64_t seed, int32_t stream, int64_t count, double* out) {
  uint64_t state = seed ^ (0x632BE59BD9B4E019ull * static_cast<uint64_t>(stream + 1));
  const double scale = 1.0 / 9007199254740992.0;  // 2^-53
  const double two_pi = 2.0 * M_PI;
  for (int64_t i = 0; i < count; i += 2) {
    const uint64_t a = splitmix_next(state);
    const uint64_t b = splitmix_next(state);
    const double u1 = static_cast<double>((a >> 11) + 1) * scale;
    const double u2 = static_cast<double>((b >> 11) + 1) * scale;
    const double rad = std::sqrt(-2.0 * std::log(u1));
    out[i] = rad * std::cos(two_pi * u2);
    if (i + 1 < count) out[i + 1] = rad * std::sin(two_pi * u2);
  }
}

tpo_status fail(Plan* p, tpo_status st, const std::string& msg) {
  if (p) p->last_error = msg;
  return st;
}

void build_layout(Plan& p) {
  Layout& L = p.lay;
  size_t cur = 0;
  auto add = [&](Buf b, size_t bytes) {
    cur = align256(cur);
    L.off[b] = cur;
    L.bytes[b] = bytes;
    cur += std::max<size_t>(bytes, 8);
  };
  const size_t E = static_cast<size_t>(std::max<int64_t>(p.E, 1));
  const size_t n = p.n, m = p.m, du = p.du, d = p.d, dp = p.dp, lr = std::max(p.lr, 1), kp = p.kp, k = p.k,
               twod = p.twod;
  const size_t nb_sort = p.sort_blocks;
  const size_t scan_n = std::max({256 * nb_sort, E, n + 1, m + 1});
  const size_t aux = (scan_n + 2047) / 2048 + 1;
  const size_t maxch = static_cast<size_t>(std::max(p.max_chunks_u, p.max_chunks_v));
  const size_t nbr = p.rowpass_blocks;
  add(B_STATUS, sizeof(DevStatus));
  add(B_GSTATUS, sizeof(GraphStatus));
  add(B_KEYS_A, 8 * E);
  add(B_KEYS_B, 8 * E);
  add(B_WV_A, 4 * E);
  add(B_WV_B, 4 * E);
  add(B_HIST, 4 * 256 * nb_sort);
  add(B_SCAN_AUX, 4 * aux);
  add(B_UPOS, 4 * E);
  add(B_ROWPTR_U, 4 * (n + 1));
  add(B_COL_U, 4 * E);
  add(B_VAL_U, 4 * E);
  add(B_ROWPTR_V, 4 * (m + 1));
  add(B_COL_V, 4 * E);
  add(B_VAL_V, 4 * E);
  add(B_DEG_U, 4 * n);
  add(B_DEG_V, 4 * m);
  add(B_ISQ_U, 4 * n);
  add(B_INV_V, 4 * m);
  add(B_HUBCNT_U, 4 * (n + 1));
  add(B_HUBCNT_V, 4 * (m + 1));
  add(B_HUBROW_U, 4 * (n + 1));
  add(B_HUBROW_V, 4 * (m + 1));
  add(B_CHUNK_U, 16 * static_cast<size_t>(p.max_chunks_u + 1));
  add(B_CHUNK_V, 16 * static_cast<size_t>(p.max_chunks_v + 1));
  add(B_HUBLIST_U, 16 * static_cast<size_t>(p.max_chunks_u + 1));
  add(B_HUBLIST_V, 16 * static_cast<size_t>(p.max_chunks_v + 1));
  add(B_PARTIAL, 4 * dp * (maxch + 1));
  // Gram partials: one tile per (chunk, upper tile pair); 64 x 64 tiles for
  // FP32 X and R, 128 x 128 for the narrow types
  const size_t gt = narrow_gram(p) ? kNarrowTile : 64;
  const size_t tx = (du + gt - 1) / gt, tr = (twod + 63) / 64;
  const size_t gpart_x = p.reduce ? static_cast<size_t>(p.gram_chunks_x) * (tx * (tx + 1) / 2) * gt * gt : 0;
  const size_t gpart_r = static_cast<size_t>(p.gram_chunks_r) * (tr * (tr + 1) / 2) * 4096;
  add(B_GRAM_PART, 8 * std::max(gpart_x, gpart_r));
  add(B_COLSUM_PART, 8 * (p.reduce ? static_cast<size_t>(p.gram_chunks_x) * du : 1));
  add(B_C, 8 * (p.reduce ? du * du : 1));
  add(B_COLSUM_X, 8 * du);
  add(B_MR_A, 8 * du * lr);
  add(B_MR_B, 8 * du * lr);
  add(B_SMALL_A, 8 * std::max(lr * lr, d * d));
  add(B_SMALL_B, 8 * lr * lr);
  add(B_SMALL_C, 8 * lr * lr);
  add(B_EVAL, 8 * std::max(lr, d));
  add(B_PSI_D, 8 * du * d);
  add(B_PSI_D32, 4 * du * dp);
  // narrow attributes: diag(scale) Psi_d split into three bfloat16 parts,
  // transposed (3 x dp x d_u rounded up to 8)
  add(B_PSI_SPLIT, (p.xbf16 || p.xfp8) && p.reduce ? 2 * 3 * dp * ((du + 7) / 8 * 8) : 8);
  add(B_XPRIME, 4 * n * dp);
  add(B_W0, 4 * n * dp);
  add(B_W1, 4 * n * dp);
  add(B_T, 4 * m * dp);
  add(B_Z, 4 * n * dp);
  add(B_G, 8 * d * d);
  add(B_Q, 8 * d * d);
  add(B_QT32, 4 * d * d);
  add(B_R, 4 * n * twod);
  add(B_RPART, 8 * nbr * twod);
  add(B_RSUM, 8 * twod);
  add(B_RCOLSUM, 8 * twod);
  add(B_OMEGA, 8 * twod * kp);
  add(B_K, 8 * twod * twod);
  add(B_M_A, 8 * twod * kp);
  add(B_M_B, 8 * twod * kp);
  add(B_EK_A, 8 * kp * kp);
  add(B_EK_B, 8 * kp * kp);
  add(B_EK_C, 8 * kp * kp);
  add(B_JLOG, jacobi_log_n(p) > 0 ? jacobi_log_bytes(jacobi_log_n(p)) : 8);
  add(B_EEVAL, 8 * twod * kp);
  add(B_S32, 4 * twod * k);
  add(B_GAMMA, 4 * n * k);
  add(B_SIGMA, 8 * k);
  add(B_PSI, 8 * twod * k);
  add(B_OMR, 8 * du * lr);
  add(B_UPS, 4 * n * k);
  add(B_H, 8 * twod * k);
  add(B_H32, 4 * twod * k);
  add(B_H_NEW, 8 * twod * k);
  add(B_RTU, 8 * (twod * k + k * k));
  add(B_UTU, 8);
  add(B_A32, 4 * k * k);
  add(B_ONMF_PART, 8 * nbr * (twod * k + k * k));
  add(B_LABELS, 4 * n);
  add(B_NCI_PART, 8 * (nbr + 1) * (k * k + k));  // partial columns: workgroups, then rechecked rows
  add(B_NCI_SUM, 8 * (k * k + k));
  add(B_NCI_PHI, 8 * k * k);
  add(B_NCI_PM, 8 * k * k);
  add(B_NCI_PV, 8 * k * k);
  add(B_NCI_CHECK, 4 * (2048 + n));  // per-round recheck counters and changed flags, then a row list
  {
    // sparse attributes (TPO_X_CSR)
    const bool xs = p.xcsr;
    const bool xr = p.xcsr && p.reduce;
    const size_t nnz = static_cast<size_t>(std::max<int64_t>(p.xnnz, 1));
    const size_t ldst = static_cast<size_t>(xcsr_stage_ld(static_cast<int>(du)));
    add(B_XS_SCALE, xs ? 4 * du : 8);
    add(B_XS_COLMAX, xs ? 4 * du : 8);
    add(B_XS_STAGE, xr ? ldst * static_cast<size_t>(p.xstage_rows) : 8);
    add(B_XT_KA, xr ? 8 * nnz : 8);
    add(B_XT_KB, xr ? 8 * nnz : 8);
    add(B_XT_VA, xr ? 4 * nnz : 8);
    add(B_XT_VB, xr ? 4 * nnz : 8);
    add(B_XT_HIST, xr ? 4 * 256 * static_cast<size_t>(p.xsort_blocks) : 8);
    // its own scan scratch: ingest may run beside the reduction on a second stream
    add(B_XT_AUX, xr ? 4 * ((256 * static_cast<size_t>(p.xsort_blocks) + 2047) / 2048 + 1) : 8);
    add(B_XT_COLPTR, xr ? 4 * (du + 1) : 8);
    add(B_XT_ROW, xr ? 4 * nnz : 8);
    add(B_XT_CHUNK, xr ? 16 * static_cast<size_t>(p.xchunks_max) : 8);
    add(B_XT_CINFO, xr ? 8 * (du + 1) : 8);
    add(B_XT_CPART, xr ? 8 * static_cast<size_t>(p.xchunks_max) * (lr + 1) : 8);
    add(B_XT_Y, xr ? 4 * n * lr : 8);
  }
  add(B_OBJ_PART, 8 * static_cast<size_t>(p.obj_blocks) * (k * twod + k));
  add(B_OBJ_SUM, 8 * (k * twod + k));
  add(B_REDTMP, 8 * 16 * std::max(twod * k + k * k, twod));
  {
    const bool red_si = p.reduce && p.lr <= kLdsMaxN;
    const bool emb_si = p.kp <= kWideMaxN;
    const size_t mp = std::max(red_si ? du * lr : 0, emb_si ? twod * kp : 0);
    const size_t li = std::max(red_si ? subspace_gsum_doubles(static_cast<int>(lr)) : 0,
                               emb_si ? subspace_gsum_doubles(static_cast<int>(kp)) : 0);
    const size_t pt = std::max(red_si ? subspace_part_doubles(static_cast<int>(du), static_cast<int>(lr)) : 0,
                               emb_si ? subspace_part_doubles(static_cast<int>(twod), static_cast<int>(kp)) : 0);
    add(B_SI_M, 8 * mp);
    add(B_SI_P, 8 * mp);
    add(B_SI_GRAM, 8 * li);
    add(B_SI_PART, 8 * pt);
    add(B_SI_BAR, 8);
  }
  L.total = align256(cur);
}

tpo_status check_ws(tpo_plan* p, void* ws, size_t bytes) {
  if (!ws) return fail(p, TPO_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(p, TPO_EINVAL, "workspace not 256-byte aligned");
  if (bytes < p->lay.total)
    return fail(p, TPO_ENOMEM, "workspace has " + std::to_string(bytes) + " bytes, plan needs " +
                                   std::to_string(p->lay.total));
  return TPO_OK;
}

tpo_status map_bits(tpo_plan* p, int32_t bits) {
  if (bits & 1) return fail(p, TPO_ERANGE, "edge endpoint out of range");
  if (bits & 2) return fail(p, TPO_ERANGE, "negative or non-finite edge weight");
  if (bits & 4) return fail(p, TPO_ENUMERIC, "non-finite attribute value");
  if (bits & 8) return fail(p, TPO_ENUMERIC, "R'[i].r <= 0 or not finite (Eq. Ri)");
  if (bits & 16) return fail(p, TPO_ENUMERIC, "Cholesky breakdown in an orthonormalisation");
  if (bits & 32) return fail(p, TPO_ENUMERIC, "non-finite value in the ONMF updates");
  if (bits & 64) return fail(p, TPO_EDEVICE, "grid barrier of the subspace iteration timed out");
  if (bits & 128) return fail(p, TPO_ERANGE, "sparse attributes: row starts or column ids out of range");
  return TPO_OK;
}

template <typename F>
tpo_status guarded(tpo_plan* p, F&& f) {
  try {
    f();
    return TPO_OK;
  } catch (const std::exception& e) {
    return fail(p, TPO_EDEVICE, e.what());
  }
}

void upload_inputs(tpo_plan* p, void* ws, hipStream_t s) {
  DevStatus& init = p->init_status;
  std::memset(&init, 0, sizeof(init));
  init.has_vals = p->prob.weighted ? 1 : 0;
  TPO_HIP_CHECK(hipMemcpyAsync(bufp<char>(*p, ws, B_STATUS), &init, sizeof(init), hipMemcpyHostToDevice, s));
  if (p->reduce)
    TPO_HIP_CHECK(hipMemcpyAsync(bufp<char>(*p, ws, B_OMR), p->omega_r.data(), sizeof(double) * p->omega_r.size(),
                                 hipMemcpyHostToDevice, s));
  TPO_HIP_CHECK(hipMemcpyAsync(bufp<char>(*p, ws, B_G), p->g.data(), sizeof(double) * p->g.size(),
                               hipMemcpyHostToDevice, s));
  TPO_HIP_CHECK(hipMemcpyAsync(bufp<char>(*p, ws, B_OMEGA), p->omega.data(), sizeof(double) * p->omega.size(),
                               hipMemcpyHostToDevice, s));
}

bool valid_inputs(tpo_plan* p, const tpo_inputs* in, std::string* why, bool need_edges = true) {
  if (!in) {
    *why = "inputs are NULL";
    return false;
  }
  if (need_edges && p->E > 0 && (!in->edge_u || !in->edge_v)) {
    *why = "edge arrays are NULL";
    return false;
  }
  if (need_edges && p->prob.weighted && p->E > 0 && !in->edge_w) {
    *why = "weighted problem without edge_w";
    return false;
  }
  if (p->xcsr) {
    if (!in->x_rowptr || (p->xnnz > 0 && (!in->x_col || !in->x_u))) {
      *why = "x_rowptr, x_col or x_u (the values) is NULL for sparse attributes";
      return false;
    }
    return true;
  }
  if (!in->x_u) {
    *why = "x_u is NULL";
    return false;
  }
  if (in->ld_x < p->du) {
    *why = "ld_x < d_u";
    return false;
  }
  if (p->xfp8 && !in->x_scale) {
    *why = "x_scale is NULL for FP8 attributes";
    return false;
  }
  return true;
}

}  // namespace

tpo_status tpo::execute_plan(tpo_plan* plan, const tpo_inputs* in, void* ws, size_t bytes, hipStream_t s,
                             const tpo_outputs* out, bool no_alloc, bool resident) {
  if (!plan) return TPO_EINVAL;
  tpo_status st = check_ws(plan, ws, bytes);
  if (st != TPO_OK) return st;
  std::string why;
  if (!valid_inputs(plan, in, &why, !resident)) return fail(plan, TPO_EINVAL, why);
  if (resident) {
    // the workspace must hold a finished ingest of a graph of this shape
    GraphStatus g{};
    st = guarded(plan, [&] {
      TPO_HIP_CHECK(hipMemcpyAsync(&g, bufp<char>(*plan, ws, B_GSTATUS), sizeof(g), hipMemcpyDeviceToHost, s));
      TPO_HIP_CHECK(hipStreamSynchronize(s));
    });
    if (st != TPO_OK) return st;
    if (g.magic != kGraphMagic || g.n != plan->n || g.m != plan->m || g.n_edges != static_cast<int32_t>(plan->E))
      return fail(plan, TPO_EINVAL, "the workspace holds no ingested graph of this plan's shape");
  }
  if (!out || !out->labels) return fail(plan, TPO_EINVAL, "outputs or labels are NULL");
  const bool timing = (plan->par.flags & TPO_FLAG_TIMING) != 0;
  if (no_alloc && timing) return fail(plan, TPO_EINVAL, "a plan with TPO_FLAG_TIMING creates events; use one without");
  DevStatus& host = plan->host_status;
  st = guarded(plan, [&] {
    if (timing && !plan->events_made) {
      for (auto& e : plan->ev) TPO_HIP_CHECK(hipEventCreate(&e));
      for (auto& e : plan->kev) TPO_HIP_CHECK(hipEventCreate(&e));
      plan->events_made = true;
      plan->kev_made = true;
    }
    auto mark = [&](int i) {
      if (timing) TPO_HIP_CHECK(hipEventRecord(plan->ev[i], s));
    };
    upload_inputs(plan, ws, s);
    mark(0);
    if (resident) {
      // the graph ingested by an earlier job on this workspace
      restore_graph_status(*plan, ws, s);
      mark(1);
      launch_reduce(*plan, ws, in, s);
      mark(2);
    } else if (timing || no_alloc || (plan->par.flags & TPO_FLAG_ONE_STREAM)) {
      // stage by stage on one stream (timing: so that each stage's time is its own)
      launch_ingest(*plan, ws, in, s);
      mark(1);
      launch_reduce(*plan, ws, in, s);
      mark(2);
    } else {
      // ingest (edges only) and the attribute reduction (X only) are
      // independent: ingest runs on a second stream beside the reduction's
      // chain of small dependent kernels
      if (!plan->side_made) {
        TPO_HIP_CHECK(hipStreamCreateWithFlags(&plan->side, hipStreamNonBlocking));
        TPO_HIP_CHECK(hipEventCreateWithFlags(&plan->fork_ev, hipEventDisableTiming));
        TPO_HIP_CHECK(hipEventCreateWithFlags(&plan->join_ev, hipEventDisableTiming));
        plan->side_made = true;
      }
      TPO_HIP_CHECK(hipEventRecord(plan->fork_ev, s));
      TPO_HIP_CHECK(hipStreamWaitEvent(plan->side, plan->fork_ev, 0));
      // the reduction is enqueued first: its long few-workgroup kernels
      // (subspace iteration, Rayleigh-Ritz) then run beside ingest's
      // whole-GPU sort and scan kernels instead of after them
      launch_reduce(*plan, ws, in, s);
      launch_ingest(*plan, ws, in, plan->side);
      TPO_HIP_CHECK(hipEventRecord(plan->join_ev, plan->side));
      TPO_HIP_CHECK(hipStreamWaitEvent(s, plan->join_ev, 0));
    }
    launch_propagate(*plan, ws, bufp<float>(*plan, ws, B_XPRIME), plan->dp, s);
    mark(3);
    launch_features(*plan, ws, s);
    mark(4);
    launch_embed(*plan, ws, s);
    mark(5);
    // with ONMF rounds to run, the last one writes the output embedding too
    float* emb_direct = plan->par.t_f >= 1 ? static_cast<float*>(out->embedding) : nullptr;
    launch_onmf(*plan, ws, s, emb_direct);
    mark(6);
    launch_nci(*plan, ws, s);
    mark(7);
    launch_objective(*plan, ws, s);
    mark(8);
    TPO_HIP_CHECK(hipMemcpyAsync(out->labels, bufp<int32_t>(*plan, ws, B_LABELS), sizeof(int32_t) * plan->n,
                                 hipMemcpyDeviceToDevice, s));
    if (out->embedding && !emb_direct)
      TPO_HIP_CHECK(hipMemcpyAsync(out->embedding, bufp<float>(*plan, ws, B_UPS),
                                   sizeof(float) * static_cast<size_t>(plan->n) * plan->k, hipMemcpyDeviceToDevice, s));
    TPO_HIP_CHECK(hipMemcpyAsync(&host, bufp<char>(*plan, ws, B_STATUS), sizeof(host), hipMemcpyDeviceToHost, s));
    TPO_HIP_CHECK(hipStreamSynchronize(s));
    if (timing) {
      float ms[8];
      for (int i = 0; i < 8; ++i) TPO_HIP_CHECK(hipEventElapsedTime(&ms[i], plan->ev[i], plan->ev[i + 1]));
      tpo_stats& S = plan->stats;
      S.ms_ingest = ms[0];
      S.ms_reduce = ms[1];
      S.ms_propagate = ms[2];
      S.ms_features = ms[3];
      S.ms_embed = ms[4];
      S.ms_onmf = ms[5];
      S.ms_nci = ms[6];
      S.ms_objective = ms[7];
      float tot;
      TPO_HIP_CHECK(hipEventElapsedTime(&tot, plan->ev[0], plan->ev[8]));
      S.ms_total = tot;
      const int hops = std::min(plan->par.gamma, kMaxTimedHops);
      S.ms_spmm_v = S.ms_spmm_u = 0.0;
      for (int h = 0; h < hops; ++h) {
        float a, b;
        TPO_HIP_CHECK(hipEventElapsedTime(&a, plan->kev[4 * h], plan->kev[4 * h + 1]));
        TPO_HIP_CHECK(hipEventElapsedTime(&b, plan->kev[4 * h + 2], plan->kev[4 * h + 3]));
        S.ms_spmm_v += a;
        S.ms_spmm_u += b;
      }
      S.n_spmm_v = S.n_spmm_u = hops;
    }
  });
  if (st != TPO_OK) return st;
  plan->stats.n_unique_edges = host.n_unique;
  plan->stats.guard_hits = host.guard_hits;
  plan->stats.isolated_u = host.iso_u;
  plan->stats.isolated_v = host.iso_v;
  plan->stats.nci_rechecked = host.nci_rechecked;
  plan->stats.nci_rounds = host.nci_rounds;
  if (out->objective) {
    out->objective[0] = host.objective[0];
    out->objective[1] = host.objective[1];
  }
  return map_bits(plan, host.err_bits);
}


tpo_status tpo::plan_fail(tpo_plan* plan, tpo_status st, const std::string& msg) { return fail(plan, st, msg); }

extern "C" {

int32_t tpo_abi_version(void) { return TPO_ABI_VERSION; }

uint8_t tpo_e4m3_encode(float v) { return tpo::e4m3_encode(v); }

const char* tpo_status_string(tpo_status status) {
  switch (status) {
    case TPO_OK: return "ok";
    case TPO_EINVAL: return "invalid argument";
    case TPO_ERANGE: return "value out of range";
    case TPO_ENOMEM: return "workspace too small";
    case TPO_EDEVICE: return "device error";
    case TPO_ENUMERIC: return "numerical failure";
  }
  return "unknown status";
}

const char* tpo_plan_last_error(const tpo_plan* plan) { return plan ? plan->last_error.c_str() : "no plan"; }

tpo_status tpo_draw_normals(uint64_t seed, int32_t stream, int64_t count, double* out) {
  if (count < 0 || (count > 0 && !out) || stream < 0) return TPO_EINVAL;
  draw_normals(seed, stream, count, out);
  return TPO_OK;
}

tpo_status tpo_plan_create(const tpo_problem* prob, const tpo_params* par, tpo_plan** out_plan) {
  if (!prob || !par || !out_plan) return TPO_EINVAL;
  *out_plan = nullptr;
  if (prob->abi_version != TPO_ABI_VERSION || par->abi_version != TPO_ABI_VERSION) return TPO_EINVAL;
  if (prob->n_u < 1 || prob->n_v < 1 || prob->n_edges < 0 || prob->n_edges >= (int64_t{1} << 31)) return TPO_EINVAL;
  if (prob->d_u < 1 || prob->d_u > kMaxDu) return TPO_EINVAL;
  if (prob->x_dtype != TPO_X_F32 && prob->x_dtype != TPO_X_BF16 && prob->x_dtype != TPO_X_FP8 &&
      prob->x_dtype != TPO_X_CSR)
    return TPO_EINVAL;
  if (prob->x_dtype == TPO_X_CSR && (prob->x_nnz < 0 || prob->x_nnz >= (int64_t{1} << 31))) return TPO_EINVAL;
  if (par->k < 1 || par->k > kMaxK) return TPO_EINVAL;
  if (!(par->alpha >= 0.0 && par->alpha < 1.0)) return TPO_EINVAL;
  if (par->gamma < 0 || par->gamma > 1000 || par->q < 0 || par->q > 100) return TPO_EINVAL;
  if (par->oversample < 0 || par->oversample > 64) return TPO_EINVAL;
  if (par->t_f < 0 || par->t_f > 1000 || par->t_g < 0 || par->t_g > 1000) return TPO_EINVAL;
  if (par->x_refine < 0 || par->x_refine > 8) return TPO_EINVAL;
  const bool reduce = par->d > 0 && par->d < prob->d_u;
  const int d = reduce ? par->d : prob->d_u;
  if (d > kMaxDEff) return TPO_EINVAL;
  if (par->k > 2 * d) return TPO_EINVAL;
  tpo_plan* p = new (std::nothrow) tpo_plan();
  if (!p) return TPO_EINVAL;
  p->prob = *prob;
  p->par = *par;
  p->n = prob->n_u;
  p->m = prob->n_v;
  p->du = prob->d_u;
  p->E = prob->n_edges;
  p->reduce = reduce;
  p->xbf16 = prob->x_dtype == TPO_X_BF16;
  p->xfp8 = prob->x_dtype == TPO_X_FP8;
  p->xcsr = prob->x_dtype == TPO_X_CSR;
  p->xnnz = p->xcsr ? prob->x_nnz : 0;
  p->d = d;
  p->dp = next_pow2_at_least(d, 16);
  p->k = par->k;
  p->twod = 2 * d;
  p->kp = std::min(par->k + par->oversample, 2 * d);
  p->lr = reduce ? std::min(d + par->oversample, prob->d_u) : 0;
  if (p->lr > 256) {
    delete p;
    return TPO_EINVAL;
  }
  // sparse attributes: the sums of the refinement step hold up to 128 sketch
  // columns (two per lane)
  if (p->xcsr && reduce && p->lr > 128) {
    delete p;
    return TPO_EINVAL;
  }
  p->xsort_blocks = static_cast<int>(std::max<int64_t>((p->xnnz + kSortTile - 1) / kSortTile, 1));
  p->xchunks_max = p->xnnz / 8192 + p->du + 1;
  {
    // FP8 staging tile: row groups of about 512 MiB of codes (64-row
    // multiples); each group's Gram launch reads and writes every tile-pair
    // partial once, so fewer, larger groups cost less of that traffic
    const int64_t ld = xcsr_stage_ld(p->du);
    const int64_t g = std::max<int64_t>(64, ((int64_t{512} << 20) / ld) / 64 * 64);
    p->xstage_rows = static_cast<int>(std::min<int64_t>(g, (int64_t{p->n} + 63) / 64 * 64));
  }
  p->rowbits = bits_for(p->n);
  p->colbits = bits_for(p->m);
  p->sort_blocks = static_cast<int>(std::max<int64_t>((p->E + kSortTile - 1) / kSortTile, 1));
  const int64_t maxch = 2 * (p->E / kHubChunk) + 2;
  p->max_chunks_u = static_cast<int>(maxch);
  p->max_chunks_v = static_cast<int>(maxch);
  const int gtx = narrow_gram(*p) ? kNarrowTile : 64;
  const int tiles_x = (p->du + gtx - 1) / gtx, tiles_r = (p->twod + 63) / 64;
  const int pairs_x = tiles_x * (tiles_x + 1) / 2, pairs_r = tiles_r * (tiles_r + 1) / 2;
  // row chunks of the Gram partials: about `blocks` (chunk, pair) workgroups,
  // and a multiple of 8, at least 8, so that the narrow-type kernels (which
  // give each XCD whole chunks) keep all eight XCDs busy
  auto chunks_for = [&](int pairs, int64_t blocks) {
    int64_t want = std::max<int64_t>(8, blocks / pairs);
    want = (want + 7) / 8 * 8;
    int64_t by_rows = std::max<int64_t>(1, (p->n + 255) / 256);
    return static_cast<int>(std::min<int64_t>({want, by_rows, 65535}));
  };
  // the narrow kernel's 512-thread workgroups run one per CU: about eight
  // rounds of them over the 256 CUs
  p->gram_chunks_x = chunks_for(pairs_x, narrow_gram(*p) ? 2048 : 1024);
  p->gram_chunks_r = chunks_for(pairs_r, 1024);
  // row-pass workgroups (ONMF, features, NCI rounds): two per CU at most;
  // measured against caps of 256, 384, 1024 and 2048 on the 4M- and
  // 150M-edge jobs (fewer blocks write fewer FP64 partials per pass)
  p->rowpass_blocks = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((p->n + 31) / 32, 512)));
  p->obj_blocks = std::min(p->rowpass_blocks, 256);
  // Gaussian matrices
  if (reduce) {
    p->omega_r.resize(static_cast<size_t>(p->du) * p->lr);
    if (par->omega_reduce)
      std::memcpy(p->omega_r.data(), par->omega_reduce, sizeof(double) * p->omega_r.size());
    else
      draw_normals(par->seed, 0, static_cast<int64_t>(p->omega_r.size()), p->omega_r.data());
  }
  p->g.resize(static_cast<size_t>(d) * d);
  if (par->g)
    std::memcpy(p->g.data(), par->g, sizeof(double) * p->g.size());
  else
    draw_normals(par->seed, 1, static_cast<int64_t>(p->g.size()), p->g.data());
  p->omega.resize(static_cast<size_t>(p->twod) * p->kp);
  if (par->omega)
    std::memcpy(p->omega.data(), par->omega, sizeof(double) * p->omega.size());
  else
    draw_normals(par->seed, 2, static_cast<int64_t>(p->omega.size()), p->omega.data());
  p->par.omega_reduce = nullptr;
  p->par.g = nullptr;
  p->par.omega = nullptr;
  build_layout(*p);
  std::memset(&p->stats, 0, sizeof(p->stats));
  p->events_made = false;
  p->kev_made = false;
  p->side = nullptr;
  p->side_made = false;
  p->timing = (par->flags & TPO_FLAG_TIMING) != 0;
  *out_plan = p;
  return TPO_OK;
}

void tpo_plan_destroy(tpo_plan* plan) {
  if (!plan) return;
  if (plan->events_made)
    for (auto& e : plan->ev) (void)hipEventDestroy(e);
  if (plan->kev_made)
    for (auto& e : plan->kev) (void)hipEventDestroy(e);
  if (plan->side_made) {
    (void)hipStreamSynchronize(plan->side);
    (void)hipEventDestroy(plan->fork_ev);
    (void)hipEventDestroy(plan->join_ev);
    (void)hipStreamDestroy(plan->side);
  }
  delete plan;
}

tpo_status tpo_plan_workspace_bytes(const tpo_plan* plan, size_t* out_bytes) {
  if (!plan || !out_bytes) return TPO_EINVAL;
  *out_bytes = plan->lay.total;
  return TPO_OK;
}

tpo_status tpo_plan_dims(const tpo_plan* plan, int32_t* d_eff, int32_t* l_r, int32_t* k_prime) {
  if (!plan) return TPO_EINVAL;
  if (d_eff) *d_eff = plan->d;
  if (l_r) *l_r = plan->lr;
  if (k_prime) *k_prime = plan->kp;
  return TPO_OK;
}

tpo_status tpo_plan_stats(const tpo_plan* plan, tpo_stats* out) {
  if (!plan || !out) return TPO_EINVAL;
  *out = plan->stats;
  return TPO_OK;
}

tpo_status tpo_plan_buffer(const tpo_plan* plan, void* ws, int32_t which, void** ptr, int64_t* rows, int64_t* cols,
                           int32_t* dtype) {
  if (!plan || !ws || !ptr) return TPO_EINVAL;
  const Plan& p = *plan;
  Buf b;
  int64_t r = 0, c = 1;
  int32_t dt = TPO_DTYPE_F32;
  switch (which) {
    case TPO_BUF_ROWPTR_U: b = B_ROWPTR_U; r = p.n + 1; dt = TPO_DTYPE_I32; break;
    case TPO_BUF_COL_U: b = B_COL_U; r = p.E; dt = TPO_DTYPE_I32; break;
    case TPO_BUF_VAL_U: b = B_VAL_U; r = p.E; break;
    case TPO_BUF_ROWPTR_V: b = B_ROWPTR_V; r = p.m + 1; dt = TPO_DTYPE_I32; break;
    case TPO_BUF_COL_V: b = B_COL_V; r = p.E; dt = TPO_DTYPE_I32; break;
    case TPO_BUF_VAL_V: b = B_VAL_V; r = p.E; break;
    case TPO_BUF_DEG_U: b = B_DEG_U; r = p.n; break;
    case TPO_BUF_DEG_V: b = B_DEG_V; r = p.m; break;
    case TPO_BUF_XPRIME: b = B_XPRIME; r = p.n; c = p.dp; break;
    case TPO_BUF_PSI_D: b = B_PSI_D; r = p.du; c = p.d; dt = TPO_DTYPE_F64; break;
    case TPO_BUF_Z: b = B_Z; r = p.n; c = p.dp; break;
    case TPO_BUF_Q: b = B_Q; r = p.d; c = p.d; dt = TPO_DTYPE_F64; break;
    case TPO_BUF_R: b = B_R; r = p.n; c = p.twod; break;
    case TPO_BUF_GAMMA: b = B_GAMMA; r = p.n; c = p.k; break;
    case TPO_BUF_SIGMA: b = B_SIGMA; r = p.k; dt = TPO_DTYPE_F64; break;
    case TPO_BUF_PSI: b = B_PSI; r = p.twod; c = p.k; dt = TPO_DTYPE_F64; break;
    case TPO_BUF_UPSILON: b = B_UPS; r = p.n; c = p.k; break;
    case TPO_BUF_H: b = B_H; r = p.twod; c = p.k; dt = TPO_DTYPE_F64; break;
    case TPO_BUF_LABELS: b = B_LABELS; r = p.n; dt = TPO_DTYPE_I32; break;
    case TPO_BUF_T: b = B_T; r = p.m; c = p.dp; break;
    case TPO_BUF_W_LAST:
      if (p.par.gamma < 1) return TPO_EINVAL;
      b = ((p.par.gamma - 1) % 2 == 0) ? B_W0 : B_W1;  // the hops alternate between the two
      r = p.n;
      c = p.dp;
      break;
    case TPO_BUF_SCALE_U: b = B_ISQ_U; r = p.n; break;
    case TPO_BUF_SCALE_V: b = B_INV_V; r = p.m; break;
    case TPO_BUF_RSUM: b = B_RSUM; r = p.twod; dt = TPO_DTYPE_F64; break;
    case TPO_BUF_S: b = B_EEVAL; r = p.twod; c = p.k; dt = TPO_DTYPE_F64; break;
    case TPO_BUF_GRAM_C:
      if (!p.reduce) return TPO_EINVAL;
      b = B_C;
      r = p.du;
      c = p.du;
      dt = TPO_DTYPE_F64;
      break;
    case TPO_BUF_COLSUM_X:
      if (!p.reduce) return TPO_EINVAL;
      b = B_COLSUM_X;
      r = p.du;
      dt = TPO_DTYPE_F64;
      break;
    default: return TPO_EINVAL;
  }
  *ptr = bufp<char>(p, ws, b);
  if (rows) *rows = r;
  if (cols) *cols = c;
  if (dtype) *dtype = dt;
  return TPO_OK;
}

tpo_status tpo_stage_ingest(tpo_plan* plan, const tpo_inputs* in, void* ws, size_t bytes, void* stream) {
  if (!plan) return TPO_EINVAL;
  tpo_status st = check_ws(plan, ws, bytes);
  if (st != TPO_OK) return st;
  std::string why;
  if (!valid_inputs(plan, in, &why)) return fail(plan, TPO_EINVAL, why);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded(plan, [&] {
    upload_inputs(plan, ws, s);
    launch_ingest(*plan, ws, in, s);
  });
}

tpo_status tpo_stage_reduce(tpo_plan* plan, const tpo_inputs* in, void* ws, size_t bytes, void* stream) {
  if (!plan) return TPO_EINVAL;
  tpo_status st = check_ws(plan, ws, bytes);
  if (st != TPO_OK) return st;
  std::string why;
  if (!valid_inputs(plan, in, &why)) return fail(plan, TPO_EINVAL, why);
  return guarded(plan, [&] { launch_reduce(*plan, ws, in, static_cast<hipStream_t>(stream)); });
}

tpo_status tpo_stage_propagate(tpo_plan* plan, const tpo_inputs* in, void* ws, size_t bytes, void* stream) {
  (void)in;
  if (!plan) return TPO_EINVAL;
  tpo_status st = check_ws(plan, ws, bytes);
  if (st != TPO_OK) return st;
  return guarded(plan, [&] {
    launch_propagate(*plan, ws, bufp<float>(*plan, ws, B_XPRIME), plan->dp, static_cast<hipStream_t>(stream));
  });
}

tpo_status tpo_stage_features(tpo_plan* plan, void* ws, size_t bytes, void* stream) {
  if (!plan) return TPO_EINVAL;
  tpo_status st = check_ws(plan, ws, bytes);
  if (st != TPO_OK) return st;
  return guarded(plan, [&] { launch_features(*plan, ws, static_cast<hipStream_t>(stream)); });
}

tpo_status tpo_stage_embed(tpo_plan* plan, void* ws, size_t bytes, void* stream) {
  if (!plan) return TPO_EINVAL;
  tpo_status st = check_ws(plan, ws, bytes);
  if (st != TPO_OK) return st;
  return guarded(plan, [&] { launch_embed(*plan, ws, static_cast<hipStream_t>(stream)); });
}

tpo_status tpo_stage_onmf(tpo_plan* plan, void* ws, size_t bytes, void* stream) {
  if (!plan) return TPO_EINVAL;
  tpo_status st = check_ws(plan, ws, bytes);
  if (st != TPO_OK) return st;
  return guarded(plan, [&] { launch_onmf(*plan, ws, static_cast<hipStream_t>(stream)); });
}

tpo_status tpo_stage_nci(tpo_plan* plan, void* ws, size_t bytes, void* stream, int32_t* labels) {
  if (!plan) return TPO_EINVAL;
  tpo_status st = check_ws(plan, ws, bytes);
  if (st != TPO_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded(plan, [&] {
    launch_nci(*plan, ws, s);
    if (labels)
      TPO_HIP_CHECK(hipMemcpyAsync(labels, bufp<int32_t>(*plan, ws, B_LABELS), sizeof(int32_t) * plan->n,
                                   hipMemcpyDeviceToDevice, s));
  });
}

tpo_status tpo_stage_objective(tpo_plan* plan, void* ws, size_t bytes, void* stream, double* objective) {
  if (!plan) return TPO_EINVAL;
  tpo_status st = check_ws(plan, ws, bytes);
  if (st != TPO_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevStatus& host = plan->host_status;
  st = guarded(plan, [&] {
    launch_objective(*plan, ws, s);
    TPO_HIP_CHECK(hipMemcpyAsync(&host, bufp<char>(*plan, ws, B_STATUS), sizeof(host), hipMemcpyDeviceToHost, s));
    TPO_HIP_CHECK(hipStreamSynchronize(s));
  });
  if (st != TPO_OK) return st;
  if (objective) {
    objective[0] = host.objective[0];
    objective[1] = host.objective[1];
  }
  return map_bits(plan, host.err_bits);
}

tpo_status tpo_execute(tpo_plan* plan, const tpo_inputs* in, void* ws, size_t bytes, void* stream,
                       const tpo_outputs* out) {
  return execute_plan(plan, in, ws, bytes, static_cast<hipStream_t>(stream), out, false);
}

tpo_status tpo_execute_resident(tpo_plan* plan, const tpo_inputs* in, void* ws, size_t bytes, void* stream,
                                const tpo_outputs* out) {
  return execute_plan(plan, in, ws, bytes, static_cast<hipStream_t>(stream), out, false, true);
}

}  // extern "C"
