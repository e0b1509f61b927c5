"""Shared helpers for the GPU tests, smoke() and bench.py: run one job
through the C ABI stage by stage and pull intermediates back to the host,
and run the oracle on the same seeded inputs.  Test infrastructure only."""
from __future__ import annotations

import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(abg, *, k, alpha, gamma, d, q=20, oversample=10, t_f=5, t_g=20, seed=0,
            mm=None, stages=True, device="cuda:0", x_bf16=False, nci="literal", x_fp8=None):
    """Runs the job on the GPU.  Returns a dict of numpy intermediates.
    x_bf16: hand X over as bfloat16 (its values must be representable).
    x_fp8: (codes uint8, column scales float32) handed over as FP8 E4M3 in
    place of abg.x_u (which then holds the encoded values, for the oracle)."""
    import torch

    import paper_2405_11922_amd as tpo

    dev = torch.device(device)
    eu = torch.from_numpy(np.ascontiguousarray(abg.edge_u, dtype=np.int32)).to(dev)
    ev = torch.from_numpy(np.ascontiguousarray(abg.edge_v, dtype=np.int32)).to(dev)
    x = torch.from_numpy(np.ascontiguousarray(abg.x_u, dtype=np.float32)).to(dev)
    if x_bf16:
        xb = x.to(torch.bfloat16)
        assert torch.equal(xb.float(), x), "X is not representable in bfloat16"
        x = xb
    xs = None
    if x_fp8 is not None:
        x = torch.from_numpy(np.ascontiguousarray(x_fp8[0], dtype=np.uint8)).to(dev).view(torch.float8_e4m3fn)
        xs = torch.from_numpy(np.ascontiguousarray(x_fp8[1], dtype=np.float32)).to(dev)
    ew = None
    if abg.edge_w is not None:
        ew = torch.from_numpy(np.ascontiguousarray(abg.edge_w, dtype=np.float32)).to(dev)
    kw = {}
    if mm is not None:
        kw = dict(omega_reduce=mm.omega_reduce, g=mm.g, omega=mm.omega)
    plan = tpo.Plan.create(abg.n_u, abg.n_v, abg.n_edges, abg.d_u, device=dev, k=k, alpha=alpha,
                           gamma=gamma, d=d, q=q, oversample=oversample, t_f=t_f, t_g=t_g,
                           seed=seed, weighted=ew is not None, timing=True,
                           x_dtype="fp8" if x_fp8 is not None else "bf16" if x_bf16 else "f32", nci=nci, **kw)
    out = {}
    try:
        h, ws = plan.handle, plan.workspace
        d_eff, l_r, kp = tpo.tpo_plan_dims(h)
        out["dims"] = (d_eff, l_r, kp)
        labels = torch.empty(abg.n_u, dtype=torch.int32, device=dev)
        emb = torch.empty(abg.n_u, k, dtype=torch.float32, device=dev)
        if stages:
            tpo.tpo_stage_ingest(h, eu, ev, x, ws, edge_w=ew, x_scale=xs)
            tpo.tpo_stage_reduce(h, eu, ev, x, ws, edge_w=ew, x_scale=xs)
            tpo.tpo_stage_propagate(h, ws)
            tpo.tpo_stage_features(h, ws)
            tpo.tpo_stage_embed(h, ws)
            tpo.tpo_stage_onmf(h, ws)
            tpo.tpo_stage_nci(h, ws, labels)
            out["objective"] = tpo.tpo_stage_objective(h, ws)
            emb.copy_(plan.buffer("upsilon"))
        else:
            out["objective"] = tpo.tpo_execute(h, eu, ev, x, ws, labels, emb, edge_w=ew, x_scale=xs)
            out["stats"] = tpo.tpo_plan_stats(h)
        torch.cuda.synchronize()
        out["labels"] = labels.cpu().numpy()
        out["embedding"] = emb.cpu().numpy()
        for name in ("rowptr_u", "col_u", "val_u", "rowptr_v", "col_v", "val_v", "deg_u", "deg_v",
                     "xprime", "z", "q", "r", "gamma", "sigma", "psi", "upsilon", "h"):
            out[name] = plan.buffer(name).cpu().numpy()
        if l_r > 0:
            out["psi_d"] = plan.buffer("psi_d").cpu().numpy()
        out["xprime"] = out["xprime"][:, :d_eff] if out["xprime"].ndim == 2 else out["xprime"]
        out["z"] = out["z"][:, :d_eff] if out["z"].ndim == 2 else out["z"]
    finally:
        plan.close()
    return out


def oracle_run(abg, *, k, alpha, gamma, d, q=20, oversample=10, t_f=5, t_g=20, seed=0, mm=None,
               nci="literal"):
    import abg_synth as synth
    import oracle

    if mm is None:
        mm = synth.method_matrices(seed, abg.d_u, d, k, oversample)
    return oracle.tpo(abg.n_u, abg.n_v, abg.edge_u, abg.edge_v, abg.x_u, k=k, alpha=alpha,
                      gamma=gamma, g=mm.g, omega=mm.omega, omega_r=mm.omega_reduce, d=d, q=q,
                      t_f=t_f, t_g=t_g, edge_w=abg.edge_w, nci_variant=nci)


def rel_fro(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def row_rel_max(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    den = np.where(den > 0, den, 1.0)
    return float(np.max(num / den)) if a.shape[0] else 0.0


def top2_margin(ups, phi_labels_fn=None):
    """FP64 score margin of each row's argmax in the final NCI round."""
    s = np.sort(ups, axis=1)
    return s[:, -1] - s[:, -2]
