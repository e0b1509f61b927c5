#!/usr/bin/env python
"""Throughput of TPO clustering on one MI355X.

One step = one whole clustering job (ingest -> attribute reduction ->
propagation -> random features -> RandomizedSVD -> ONMF -> NCI -> objective)
through tpo_execute on inputs already resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--config large|mid_fp32|fp8_tfidf|serve] [--cpu-baseline on|off]

The default workload is the 150M-edge job in the attribute precision form
(X_U as bfloat16), timed beside the plain FP32 job on the same input; the
mid-size FP32 workload is reported under "mid".

Only one GPU is used: --gpus N with N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GEdge-hop/s + clusterings/s vs plain FP32 GPU; p50/p99 job latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmm_u_bytes(n, m, e, d, has_vals):
    """Algorithmic HBM bytes of one U-side SpMM launch (rows of B):
    column ids + row pointers + each gathered T row once + X' rows read +
    output rows written + the per-row scale (+ values when weighted)."""
    return 4 * e + 4 * (n + 1) + 4 * m * d + 4 * n * d + 4 * n * d + 4 * n + (4 * e if has_vals else 0)


def spmm_v_bytes(n, m, e, d, has_vals):
    """Algorithmic HBM bytes of one V-side SpMM launch (rows of B^T)."""
    return 4 * e + 4 * (m + 1) + 4 * n * d + 4 * m * d + 4 * m + (4 * e if has_vals else 0)


def counted_traffic(config: str, side: str):
    """HBM bytes per launch of the SpMM side ('U' or 'V') from the rocprofv3
    FETCH_SIZE / WRITE_SIZE runs recorded under profiles/, scaled by the
    counters' readings for a copy of known size; None when no record exists
    for this workload or the kernel source has changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"spmm_traffic_{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, rec["source"])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    k = rec["kernels"][side]
    return int(1024 * (k["fetch_kib"] * rec["fetch_factor"] + k["write_kib"] * rec["write_factor"]))


def run_serve(args) -> int:
    """The serving workload: a Poisson stream of independent jobs of random
    shape served with continuous batching (paper_2405_11922_amd.serve), each
    pool graph's CSR resident in HBM between its jobs, attributes in
    bfloat16; beside it the same stream with FP32 attributes, and with FP32
    attributes on the plain path (one job at a time, every job ingesting)."""
    import torch

    import abg_synth as synth
    from paper_2405_11922_amd import serve

    dev = torch.device("cuda:0")
    shapes, reqs = synth.serving_stream(args.serve_jobs, args.serve_rate, args.serve_pool, seed=args.seed)
    t0 = time.time()
    graphs = []
    for n_u, n_v, n_edges, k, d_u, gseed in shapes:
        eu, ev, x, _, _ = synth.planted_abg_device(n_u, n_v, n_edges, k, d_u, device=dev, zipf_a=2.0, seed=gseed)
        graphs.append((eu, ev, x, n_v))
    torch.cuda.synchronize()
    log(f"[serve] {len(shapes)} pool graphs (|U| {min(s[0] for s in shapes)}..{max(s[0] for s in shapes)}, "
        f"{sum(s[2] for s in shapes)} edges in all) drawn on the GPU in {time.time() - t0:.1f}s")

    def stream_of(dtype):
        xs = [g[2].to(dtype) for g in graphs]
        jobs = [serve.Job(i, r.arrival, graphs[r.graph][0], graphs[r.graph][1], xs[r.graph], graphs[r.graph][3],
                          r.params, graph_key=r.graph) for i, r in enumerate(reqs)]
        warm = [serve.Job(-1 - i, 0.0, graphs[g][0], graphs[g][1], xs[g], graphs[g][3], reqs[0].params | dict(k=2))
                for i, g in enumerate(range(min(4, len(graphs))))]
        return jobs, warm

    def serve_once(tag, dtype, workers, resident):
        jobs, warm = stream_of(dtype)
        srv = serve.Server(device=dev, hbm_budget=args.serve_hbm_gb << 30, workers=workers, resident=resident)
        srv.run(warm, realtime=False)
        torch.cuda.synchronize()
        t1 = time.time()
        res = srv.run(jobs, realtime=True)
        torch.cuda.synchronize()
        wall = time.time() - t1
        summ = serve.summarize(res)
        log(f"[serve] {tag}: {summ['jobs']} jobs ({summ['failed']} failed, {summ.get('resident_jobs', 0)} on a resident "
            f"graph) in {wall:.2f}s: {summ.get('jobs_per_s', 0):.1f} jobs/s, p50 {summ.get('p50_ms', 0):.2f} ms, "
            f"p99 {summ.get('p99_ms', 0):.2f} ms; queueing p50 {summ.get('queue_p50_ms', 0):.2f} ms, inside "
            f"tpo_execute p50 {summ.get('exec_p50_ms', 0):.2f} ms (mean {summ.get('exec_mean_ms', 0):.2f})")
        return summ

    summ = serve_once("bf16, resident graphs", torch.bfloat16, args.serve_workers, True)
    f32 = serve_once("f32, resident graphs", torch.float32, args.serve_workers, True)
    plain = serve_once("f32, plain path (one job at a time, every job ingests)", torch.float32, 1, False)

    def brief(x):
        return {"jobs_per_s": round(x["jobs_per_s"], 3) if x.get("jobs_per_s") else None,
                "p50_ms": round(x["p50_ms"], 4), "p99_ms": round(x["p99_ms"], 4),
                "exec_p50_ms": round(x["exec_p50_ms"], 4), "failed": x["failed"]}

    result = {
        "metric": "clusterings/s served (continuous batching) and p50/p99 job latency",
        "value": round(summ["jobs_per_s"], 3) if summ.get("jobs_per_s") else None,
        "unit": "clusterings/s",
        "n_gpus": 1,
        "steps": summ["jobs"],
        "warmup": 4,
        "ms_per_step": round(1e3 / summ["jobs_per_s"], 4) if summ.get("jobs_per_s") else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 attributes, f32 path",
        "data": "synthetic",
        "config": {
            "workload": f"serve: Poisson arrivals at {args.serve_rate} jobs/s, {args.serve_jobs} jobs drawn from "
                        f"{args.serve_pool} planted-partition graphs, |U| log-uniform in [1e3, 5e5], |V| = 1.5|U|, "
                        f"average degree 10-30, k in [2, 64], d_U in {{32, 128, 256}} bfloat16 -> min(d_U, 64), "
                        f"gamma 5, alpha 0.5; {args.serve_workers} concurrent jobs, "
                        f"{args.serve_hbm_gb} GiB workspace budget, each graph's CSR resident between its jobs",
        },
        "latency_ms": {"p50": round(summ["p50_ms"], 4), "p99": round(summ["p99_ms"], 4),
                       "mean": round(summ["mean_ms"], 4), "max": round(summ["max_ms"], 4)},
        "resident_jobs": summ.get("resident_jobs", 0),
        "failed": summ["failed"],
        "vs_f32_same_server": brief(f32),
        "vs_plain_fp32": brief(plain),
    }
    print(json.dumps(result), flush=True)
    return 0 if summ["failed"] == 0 else 1


def mfma_util(config: str):
    """MFMA utilisation of the attribute Gram (S1), the random features (S3)
    and the embedding (S4) kernels from the rocprofv3 counter run recorded
    under profiles/ for this workload, or None when no record exists or a
    kernel source has changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"mfma_util_{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    for src, sha in rec["sources"].items():
        with open(os.path.join(ROOT, src), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != sha:
                return None
    return {"busy_pct": rec["busy_pct"], "profile": os.path.relpath(path, ROOT)}


def make_input(args, config, dev):
    """Seeded synthetic input of one workload, resident in HBM."""
    import torch

    import abg_synth as synth

    shape = synth.CONFIGS[config]
    x_scale = None  # column scales of FP8 attributes
    t0 = time.time()
    on_device = shape.n_edges > 20_000_000  # the host generator is too slow beyond this
    if on_device:
        tfidf = config == "fp8_tfidf"
        eu, ev, x, truth, _ = synth.planted_abg_device(shape.n_u, shape.n_v, shape.n_edges, shape.k,
                                                       1 if tfidf else shape.d_u,
                                                       device=dev, zipf_a=shape.zipf_a, sigma=shape.sigma,
                                                       in_out_ratio=shape.in_out_ratio, max_degree=shape.max_degree,
                                                       seed=args.seed)
        if tfidf:
            # the attributes: sparse TF-IDF rows in FP32 CSR (the library stages
            # them as FP8 E4M3 codes with column scales for the Gram)
            import paper_2405_11922_amd as tpo

            del x
            rowptr, col, val = synth.tfidf_csr(truth, shape.d_u, device=dev, seed=args.seed)
            x = tpo.CsrX(rowptr, col, val, shape.d_u)
        torch.cuda.synchronize()
        truth = truth.cpu().numpy()
        abg = None
    else:
        abg = synth.config_abg(shape, seed=args.seed)
        eu = torch.from_numpy(abg.edge_u).to(dev)
        ev = torch.from_numpy(abg.edge_v).to(dev)
        x = torch.from_numpy(abg.x_u).to(dev)
        truth = abg.labels_u
    log(f"[bench] generated {config} ({'on the GPU' if on_device else 'on the host'}): n_u={shape.n_u} "
        f"n_v={shape.n_v} E={shape.n_edges} d_u={shape.d_u} in {time.time() - t0:.1f}s")
    return dict(shape=shape, eu=eu, ev=ev, x=x, x_scale=x_scale, truth=truth, abg=abg, on_device=on_device)


def time_jobs(args, inp, x, x_dtype, dev, steps, warmup, instrument=True):
    """W untimed and K timed whole jobs (tpo_execute) of one input; then, with
    an instrumented plan, the stage split and the SpMM launch times."""
    import numpy as np
    import torch

    import paper_2405_11922_amd as tpo

    shape = inp["shape"]
    kw = dict(k=shape.k, alpha=shape.alpha, gamma=shape.gamma, d=shape.d, q=shape.q,
              oversample=shape.oversample, t_f=shape.t_f, t_g=shape.t_g, seed=args.seed, x_dtype=x_dtype,
              nci=args.nci)
    eu, ev, xs = inp["eu"], inp["ev"], inp["x_scale"]
    if x_dtype == "csr":
        kw["x_nnz"] = x.nnz
    plan = tpo.Plan.create(shape.n_u, shape.n_v, shape.n_edges, shape.d_u, device=dev, timing=False, **kw)
    labels = torch.empty(shape.n_u, dtype=torch.int32, device=dev)
    emb = torch.empty(shape.n_u, shape.k, dtype=torch.float32, device=dev)
    dims = tpo.tpo_plan_dims(plan.handle)
    for _ in range(warmup):
        tpo.tpo_execute(plan.handle, eu, ev, x, plan.workspace, labels, emb, x_scale=xs)
    torch.cuda.synchronize()
    step_ms = []
    t_start = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        obj = tpo.tpo_execute(plan.handle, eu, ev, x, plan.workspace, labels, emb, x_scale=xs)
        step_ms.append((time.perf_counter() - s0) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    plan.close()
    del plan
    res = dict(value=steps / elapsed, ms_per_step=elapsed * 1e3 / steps, obj=obj, labels=labels, emb=emb,
               dims=dims, p50=float(np.percentile(step_ms, 50)), p99=float(np.percentile(step_ms, 99)))
    log(f"[bench] {x_dtype}: {steps} steps in {elapsed:.3f}s ({res['ms_per_step']:.3f} ms/step)")
    if not instrument:
        return res
    plan_t = tpo.Plan.create(shape.n_u, shape.n_v, shape.n_edges, shape.d_u, device=dev, timing=True, **kw)
    stats = []
    for _ in range(3):
        tpo.tpo_execute(plan_t.handle, eu, ev, x, plan_t.workspace, labels, emb, x_scale=xs)
        stats.append(tpo.tpo_plan_stats(plan_t.handle))
    st = {key: statistics.median(s[key] for s in stats) for key in stats[0]}
    log(f"[bench] {x_dtype} stages ms: " + " ".join(f"{k[3:]}={st[k]:.3f}" for k in st if k.startswith("ms_")))
    res.update(stats=st, plan_t=plan_t)
    return res


def spmm_roofline(config, shape, st, d_eff):
    """Roofline of the dominant SpMM launch from the instrumented plan's HIP
    events (the larger of the U- and V-side average launch times)."""
    e_u = int(st["n_unique_edges"])
    has_vals = e_u < shape.n_edges
    u_avg = st["ms_spmm_u"] / max(st["n_spmm_u"], 1)
    v_avg = st["ms_spmm_v"] / max(st["n_spmm_v"], 1)
    if u_avg >= v_avg:
        side, kern, per, avg = "U", "k_spmm_rowgroup<64,U> (Z = X' + alpha D_U^-1/2 B T)", spmm_u_bytes(
            shape.n_u, shape.n_v, e_u, d_eff, has_vals), u_avg
    else:
        side, kern, per, avg = "V", "k_spmm_rowgroup<64,V> (T = D_V^-1 B^T W)", spmm_v_bytes(
            shape.n_u, shape.n_v, e_u, d_eff, has_vals), v_avg
    achieved = per / (avg * 1e-3) / 1e9
    return {"kernel": kern, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counted_traffic(config, side),
            "bytes_per_launch": per, "avg_launch_ms": round(avg, 5),
            "spmm_u_avg_ms": round(u_avg, 5), "spmm_v_avg_ms": round(v_avg, 5)}


def best_match_agreement(a, b, k):
    """Fraction of rows whose labels agree under the best one-to-one relabelling."""
    import numpy as np
    from scipy.optimize import linear_sum_assignment

    a, b = a.astype(np.int64), b.astype(np.int64)
    table = np.zeros((k, k), np.int64)
    np.add.at(table, (a, b), 1)
    r, c = linear_sum_assignment(-table)
    return float(table[r, c].sum() / a.size)


def sin_theta_device(a, b):
    """Largest principal-angle sine between the column spaces of two n x k
    device matrices (FP64 Grams on the GPU, eigen step on the host)."""
    import numpy as np
    import torch

    def orth(m):
        g = torch.zeros(m.shape[1], m.shape[1], dtype=torch.float64, device=m.device)
        for r0 in range(0, m.shape[0], 500_000):
            blk = m[r0:r0 + 500_000].double()
            g += blk.T @ blk
        w, v = np.linalg.eigh(g.cpu().numpy())
        w = np.maximum(w, 1e-300)
        return torch.from_numpy(v / np.sqrt(w)[None, :]).to(m.device)

    ia, ib = orth(a), orth(b)
    c = torch.zeros(a.shape[1], b.shape[1], dtype=torch.float64, device=a.device)
    for r0 in range(0, a.shape[0], 500_000):
        c += a[r0:r0 + 500_000].double().T @ b[r0:r0 + 500_000].double()
    s = np.linalg.svd((ia.T @ c @ ib).cpu().numpy(), compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - min(1.0, float(s.min())) ** 2)))


def cpu_baseline_sample(inp, shape, rows_frac=10):
    """The FP64 oracle's propagation timed on the host: one Horner hop
    (both products of L L^T) over the subgraph of the first |U|/rows_frac
    target rows (all their edges, every V node), at the workload's width d.
    Returns its rate in GEdge-hop/s (edges of the subgraph per second)."""
    import numpy as np

    import oracle

    nu = shape.n_u // rows_frac
    eu = inp["eu"].cpu().numpy()
    keep = eu < nu
    eu = eu[keep]
    ev = inp["ev"].cpu().numpy()[keep]
    del keep
    b = oracle.bipartite_adjacency(nu, shape.n_v, eu, ev)
    del eu, ev
    x = np.random.default_rng(0).standard_normal((nu, shape.d))
    t0 = time.perf_counter()
    oracle.propagate(b, x, shape.alpha, 1)
    t1 = time.perf_counter()
    oracle.propagate(b, x, shape.alpha, 2)
    t2 = time.perf_counter()
    hop = (t2 - t1) - (t1 - t0)  # the second hop alone (each call also builds L)
    rate = b.nnz / hop / 1e9
    # scipy's sparse-times-dense product runs on one thread
    return {"value": round(rate, 6), "unit": "GEdge-hop/s", "cores": 1, "kind": "oracle",
            "sample": f"one Horner hop of the oracle's propagation (oracle.propagate, scipy sparse products, "
                      f"single-threaded) over the subgraph of the first {nu} of {shape.n_u} target rows "
                      f"({b.nnz} edges, all {shape.n_v} V nodes, d={shape.d}): the time of gamma=2 minus gamma=1, "
                      f"{hop:.2f} s; rate = subgraph edges per second",
            "oracle_hop_s": round(hop, 3)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="large",
                    help="large (default), mid_fp32, fp8_tfidf, cpu_scale, serve, or copy (one 256 MiB device copy, the kernel of known traffic that scales the hardware byte counters)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-baseline", default="on", choices=["on", "off"])
    ap.add_argument("--serve-jobs", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-pool", type=int, default=32)
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-hbm-gb", type=int, default=64)
    ap.add_argument("--nci", default="literal", choices=["literal", "procrustes"],
                    help="NCI Phi update: the printed Ups^T Y, or its orthogonal polar factor")
    ap.add_argument("--x-dtype", default="auto", choices=["auto", "f32", "bf16"],
                    help="attribute storage: auto = bf16 for the large precision form, f32 otherwise")
    ap.add_argument("--compare-f32", default="on", choices=["on", "off"],
                    help="with bf16 attributes, also time the plain FP32 job on the same graph (the metric's "
                         "'vs plain FP32 GPU') and report how far the results differ")
    ap.add_argument("--mid", default="on", choices=["on", "off"],
                    help="with --config large, also time the mid-size FP32 workload (reported under 'mid')")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent jobs shard by job across GPUs; see the design notes)", file=sys.stderr)
        return 2
    if args.config == "serve":
        # one hardware queue per worker stream, so that concurrent jobs do not
        # wait behind each other in a shared queue (read when HIP starts)
        os.environ["GPU_MAX_HW_QUEUES"] = str(max(4, min(16, args.serve_workers)))

    import torch

    import paper_2405_11922_amd as tpo
    from paper_2405_11922_amd import quality

    tpo.load_library()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.config == "serve":
        return run_serve(args)
    dev = torch.device("cuda:0")
    if args.config == "copy":
        # one device copy of 256 MiB and nothing else: the kernel of known
        # traffic that scales the hardware byte counters
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"metric": "calibration copy", "bytes_read": src.numel() * 4,
                          "bytes_written": dst.numel() * 4}), flush=True)
        return 0
    inp = make_input(args, args.config, dev)
    shape = inp["shape"]
    x_dtype = args.x_dtype if args.x_dtype != "auto" else {"large": "bf16", "fp8_tfidf": "csr"}.get(args.config, "f32")
    if (x_dtype == "csr") != (args.config == "fp8_tfidf"):
        print("sparse FP8-staged attributes go with --config fp8_tfidf (and only there)", file=sys.stderr)
        return 2
    x_f32 = inp["x"]
    x = x_f32.to(torch.bfloat16) if x_dtype == "bf16" else x_f32
    compare = x_dtype == "bf16" and args.compare_f32 == "on"
    if x_dtype == "bf16" and not compare:
        del x_f32
        x_f32 = None
        inp["x"] = None

    res = time_jobs(args, inp, x, x_dtype, dev, args.steps, args.warmup)
    st = res["stats"]
    d_eff, l_r, kp = res["dims"]
    labels_np = res["labels"].cpu().numpy()
    gedge_hops = shape.gamma * int(st["n_unique_edges"]) / (st["ms_propagate"] * 1e-3) / 1e9 \
        if st["ms_propagate"] > 0 else None
    result = {
        "metric": METRIC,
        "value": round(res["value"], 4),
        "unit": "clusterings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16 attributes (BF16 MFMA Gram, FP32 accumulation), f32 path",
                  "csr": "sparse f32 attributes staged as fp8 e4m3 with column scales (FP8 MFMA Gram, FP32 "
                         "accumulation, one FP32 refinement step), f32 path"}[x_dtype],
        "data": "synthetic",
        "config": {
            "workload": f"{args.config}: planted degree-corrected bipartite SBM, |U|={shape.n_u}, "
                        f"|V|={shape.n_v}, {shape.n_edges} edges, k={shape.k}, Zipf({shape.zipf_a}) degrees"
                        + (f" (largest expected degree {shape.max_degree})" if shape.max_degree else "")
                        + f", d_U={shape.d_u} -> d={d_eff}, gamma={shape.gamma}, alpha={shape.alpha}, "
                          f"q={shape.q}, T_f={shape.t_f}, T_g={shape.t_g}"
                        + (", X_U stored as bfloat16" if x_dtype == "bf16" else "")
                        + (", sparse TF-IDF attributes (2% of the words drawn per row, abg_synth.tfidf_csr) in "
                           "FP32 CSR, densified per row group to FP8 E4M3 with column scales for the Gram"
                           if args.config == "fp8_tfidf" else ""),
            "n_u": shape.n_u, "n_v": shape.n_v, "n_edges": shape.n_edges, "k": shape.k, "d_u": shape.d_u,
            "d": d_eff, "k_prime": kp, "l_r": l_r, "gamma": shape.gamma, "x_dtype": x_dtype, "nci": args.nci,
        },
        "gedge_hop_per_s": round(gedge_hops, 3) if gedge_hops else None,
        "latency_ms": {"p50": round(res["p50"], 4), "p99": round(res["p99"], 4)},
        "stage_ms": {k[3:]: round(v, 4) for k, v in st.items() if k.startswith("ms_")},
        # NCI rounds run of T_g (a round repeating the previous one's label
        # sums ends them: the later rounds would repeat it exactly)
        "nci_rounds": int(st["nci_rounds"]),
        "roofline": spmm_roofline(args.config, shape, st, d_eff),
        "mfma_util": mfma_util(args.config + ("_bf16" if x_dtype == "bf16" else "")),
        "objective": res["obj"][0],
        # recovery of the planted clusters (ACC, NMI, ARI of the paper's quality tables)
        "quality": {key: round(v, 6) for key, v in quality.report(inp["truth"], labels_np).items()},
    }
    log(f"[bench] planted clusters recovered: {result['quality']}")
    plan_t = res["plan_t"]

    if x_dtype == "csr":
        # error of the form against FP64 on the exact attributes, for the
        # reduction (the full-size job is beyond the oracle): the exact Gram
        # in FP64 (torch, on the GPU, from the CSR rows densified in chunks),
        # the oracle's basis from it, and X' on sampled rows
        import numpy as np

        import abg_synth as synth
        import oracle

        def plan_t_buf(name):
            return tpo.tpo_plan_buffer(plan_t.handle, plan_t.workspace, name)

        rp, cl, vl = x.rowptr, x.col, x.val
        c_ex = torch.zeros(shape.d_u, shape.d_u, dtype=torch.float64, device=dev)
        colsum = torch.zeros(shape.d_u, dtype=torch.float64, device=dev)
        for r0 in range(0, shape.n_u, 100_000):
            r1 = min(shape.n_u, r0 + 100_000)
            b0, b1 = int(rp[r0]), int(rp[r1])
            rows = torch.repeat_interleave(torch.arange(r1 - r0, device=dev), (rp[r0 + 1:r1 + 1] - rp[r0:r1]))
            xd = torch.zeros(r1 - r0, shape.d_u, dtype=torch.float64, device=dev)
            xd.index_put_((rows, cl[b0:b1].long()), vl[b0:b1].double(), accumulate=True)
            c_ex += xd.T @ xd
            colsum += xd.sum(0)
            del xd, rows
        c_dev = plan_t_buf("gram_c")
        gram_rel = float((c_dev - c_ex).norm() / c_ex.norm())
        mm = synth.method_matrices(args.seed, shape.d_u, shape.d, shape.k, shape.oversample)
        psi_ref, _ = oracle.top_d_gram_basis(c_ex.cpu().numpy(), colsum.cpu().numpy(), shape.n_u, shape.d,
                                             mm.omega_reduce, shape.q)
        psi_d = plan_t_buf("psi_d").cpu().numpy()
        sin_psi = oracle.subspace_sin_theta(psi_d, psi_ref)
        idx = np.sort(np.random.default_rng(1).choice(shape.n_u, 2000, replace=False))
        xs_rows = torch.zeros(len(idx), shape.d_u, dtype=torch.float64, device=dev)
        for i, r in enumerate(idx):
            b0, b1 = int(rp[r]), int(rp[r + 1])
            xs_rows[i].index_put_((cl[b0:b1].long(),), vl[b0:b1].double(), accumulate=True)
        ref = (xs_rows @ torch.from_numpy(psi_d).to(dev)).cpu().numpy()
        got = plan_t_buf("xprime")[torch.from_numpy(idx).to(dev)][:, :shape.d].double().cpu().numpy()
        xp_rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        result["vs_fp64"] = {"gram_rel_err_vs_exact": gram_rel, "psi_d_sin_theta_vs_exact_iteration": sin_psi,
                             "xprime_rel_err_sampled_rows": xp_rel}
        log(f"[bench] sparse FP8-staged form vs FP64 on the exact attributes: Gram rel err {gram_rel:.2e} "
            f"(Frobenius), Psi_d sin theta vs the oracle's basis from the exact Gram {sin_psi:.2e}, X' rel err on "
            f"2,000 sampled rows {xp_rel:.2e}")
    plan_t.close()
    del plan_t, res["plan_t"]

    if compare:
        # the plain FP32 job on the same graph (X not rounded), timed the same
        # way: the metric's "vs plain FP32 GPU", and how far the precision form
        # moves the result
        r32 = time_jobs(args, inp, x_f32, "f32", dev, args.steps, args.warmup, instrument=False)
        agree = best_match_agreement(labels_np, r32["labels"].cpu().numpy(), shape.k)
        sin_t = sin_theta_device(res["emb"], r32["emb"])
        result["vs_plain_fp32"] = {
            "value": round(r32["value"], 4), "ms_per_step": round(r32["ms_per_step"], 4),
            "speedup": round(res["value"] / r32["value"], 4),
            "latency_ms": {"p50": round(r32["p50"], 4), "p99": round(r32["p99"], 4)},
            "label_agreement": round(agree, 6),
            "objective_rel_diff": abs(res["obj"][0] - r32["obj"][0]) / abs(r32["obj"][0]),
            "embedding_sin_theta": sin_t,
        }
        log(f"[bench] plain FP32 job on the same graph: {r32['ms_per_step']:.3f} ms/step "
            f"(bf16 speedup {result['vs_plain_fp32']['speedup']:.3f}); labels agree on {agree:.4%} of the rows, "
            f"objective rel diff {result['vs_plain_fp32']['objective_rel_diff']:.2e}, embedding sin theta {sin_t:.2e}")
        del r32

    if args.cpu_baseline == "on" and inp["on_device"]:
        # a bounded sample: the oracle's propagation hop on a tenth of the target rows
        c0 = time.perf_counter()
        result["cpu_baseline"] = cpu_baseline_sample(inp, shape)
        log(f"[bench] oracle sample {result['cpu_baseline']['value']:.5f} GEdge-hop/s "
            f"({time.perf_counter() - c0:.1f} s with its set-up)")
    if args.cpu_baseline == "on" and not inp["on_device"]:
        import oracle
        import abg_synth as synth
        from threadpoolctl import threadpool_info

        abg = inp["abg"]
        mm = synth.method_matrices(args.seed, abg.d_u, shape.d, shape.k, shape.oversample)
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        # whole jobs, repeated until about 10 s of CPU work (at most 3 jobs)
        c0 = time.perf_counter()
        jobs = 0
        while True:
            ref = oracle.tpo(abg.n_u, abg.n_v, abg.edge_u, abg.edge_v, abg.x_u, k=shape.k,
                             alpha=shape.alpha, gamma=shape.gamma, g=mm.g, omega=mm.omega,
                             omega_r=mm.omega_reduce, d=shape.d, q=shape.q, t_f=shape.t_f,
                             t_g=shape.t_g, nci_variant=args.nci)
            jobs += 1
            if time.perf_counter() - c0 >= 10.0 or jobs >= 3:
                break
        c_el = time.perf_counter() - c0
        result["cpu_baseline"] = {
            "value": round(jobs / c_el, 5), "unit": "clusterings/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{jobs} whole {args.config} job(s), same input (the FP64 numpy/scipy oracle, "
                      f"{c_el:.1f} s; sparse products single-threaded, dense BLAS on the stated threads)",
        }
        result["parity"] = {
            "labels_match_oracle": bool(oracle.labels_match_up_to_permutation(labels_np, ref.labels)),
            "objective_rel_err": abs(res["obj"][0] - ref.objective) / abs(ref.objective),
            "embedding_sin_theta": float(oracle.subspace_sin_theta(res["emb"].cpu().numpy(), ref.ups)),
        }
        log(f"[bench] oracle {c_el:.1f}s on {threads} threads; parity {result['parity']}")

    if args.config == "large" and args.mid == "on":
        # the mid-size FP32 workload, beside the headline
        del inp, x, x_f32
        torch.cuda.empty_cache()
        inp_m = make_input(args, "mid_fp32", dev)
        rm = time_jobs(args, inp_m, inp_m["x"], "f32", dev, 20, 3)
        stm = rm["stats"]
        rm["plan_t"].close()
        shm = inp_m["shape"]
        result["mid"] = {
            "workload": f"mid_fp32: |U|={shm.n_u}, |V|={shm.n_v}, {shm.n_edges} edges, k={shm.k}, "
                        f"d_U={shm.d_u} -> d={shm.d}, FP32",
            "value": round(rm["value"], 3), "unit": "clusterings/s", "ms_per_step": round(rm["ms_per_step"], 4),
            "steps": 20, "warmup": 3,
            "gedge_hop_per_s": round(shm.gamma * int(stm["n_unique_edges"]) / (stm["ms_propagate"] * 1e-3) / 1e9, 3),
            "latency_ms": {"p50": round(rm["p50"], 4), "p99": round(rm["p99"], 4)},
            "stage_ms": {k[3:]: round(v, 4) for k, v in stm.items() if k.startswith("ms_")},
            "nci_rounds": int(stm["nci_rounds"]),
            "roofline": spmm_roofline("mid_fp32", shm, stm, rm["dims"][0]),
            "mfma_util": mfma_util("mid_fp32"),
        }
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
