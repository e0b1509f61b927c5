"""Python binding of libtpo (the MI355X implementation of TPO clustering).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI declared in include/tpo.h.  The functions keep the C names
(tpo_plan_create, tpo_execute, tpo_stage_*, ...).  PyTorch supplies device
memory and the stream.  There is no CPU fallback: loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

__all__ = [
    "TPO_ABI_VERSION", "TpoError", "load_library", "lib_path",
    "TpoProblem", "TpoParams", "TpoInputs", "TpoOutputs", "TpoStats",
    "tpo_plan_create", "tpo_plan_destroy", "tpo_plan_workspace_bytes", "tpo_plan_dims",
    "tpo_execute", "tpo_stage_ingest", "tpo_stage_reduce", "tpo_stage_propagate",
    "tpo_stage_features", "tpo_stage_embed", "tpo_stage_onmf", "tpo_stage_nci",
    "tpo_stage_objective", "tpo_plan_buffer", "tpo_plan_stats", "tpo_draw_normals",
    "tpo_status_string", "BUF", "Plan", "cluster", "tpo_execute_noalloc", "TPO_NOALLOC_MAX_BYTES", "CsrX",
    "tpo_e4m3_encode", "tpo_execute_resident",
]

TPO_ABI_VERSION = 3
TPO_FLAG_TIMING = 1
TPO_FLAG_ONE_STREAM = 2
TPO_FLAG_NCI_PROCRUSTES = 4
TPO_NOALLOC_MAX_BYTES = 64 << 20  # the device array behind tpo_execute_noalloc
NCI_VARIANTS = ("literal", "procrustes")
_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libtpo.so")

STATUS = {0: "TPO_OK", 1: "TPO_EINVAL", 2: "TPO_ERANGE", 3: "TPO_ENOMEM", 4: "TPO_EDEVICE", 5: "TPO_ENUMERIC"}

BUF = {
    "rowptr_u": 0, "col_u": 1, "val_u": 2, "rowptr_v": 3, "col_v": 4, "val_v": 5,
    "deg_u": 6, "deg_v": 7, "xprime": 8, "psi_d": 9, "z": 10, "q": 11, "r": 12,
    "gamma": 13, "sigma": 14, "psi": 15, "upsilon": 16, "h": 17, "labels": 18,
    "t": 19, "w_last": 20, "scale_u": 21, "scale_v": 22, "rsum": 23, "s": 24, "gram_c": 25, "colsum_x": 26,
}
_MATRICES = {"xprime", "psi_d", "z", "q", "r", "gamma", "psi", "upsilon", "h", "t", "w_last", "s", "gram_c"}
EXPORTED = [
    "tpo_plan_create", "tpo_plan_workspace_bytes", "tpo_execute", "tpo_plan_destroy",
    "tpo_status_string", "tpo_plan_last_error", "tpo_plan_stats", "tpo_plan_dims",
    "tpo_stage_ingest", "tpo_stage_reduce", "tpo_stage_propagate", "tpo_stage_features",
    "tpo_stage_embed", "tpo_stage_onmf", "tpo_stage_nci", "tpo_stage_objective",
    "tpo_plan_buffer", "tpo_draw_normals", "tpo_abi_version", "tpo_execute_noalloc", "tpo_e4m3_encode",
    "tpo_execute_resident",
]


class TpoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class TpoProblem(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("n_u", C.c_int32), ("n_v", C.c_int32),
                ("d_u", C.c_int32), ("n_edges", C.c_int64), ("weighted", C.c_int32),
                ("x_dtype", C.c_int32), ("x_nnz", C.c_int64)]


class TpoParams(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("k", C.c_int32), ("alpha", C.c_double),
                ("gamma", C.c_int32), ("d", C.c_int32), ("q", C.c_int32),
                ("oversample", C.c_int32), ("t_f", C.c_int32), ("t_g", C.c_int32),
                ("flags", C.c_int32), ("seed", C.c_uint64),
                ("omega_reduce", C.POINTER(C.c_double)), ("g", C.POINTER(C.c_double)),
                ("omega", C.POINTER(C.c_double)), ("x_refine", C.c_int32), ("reserved", C.c_int32)]


class TpoInputs(C.Structure):
    _fields_ = [("edge_u", C.c_void_p), ("edge_v", C.c_void_p), ("edge_w", C.c_void_p),
                ("x_u", C.c_void_p), ("ld_x", C.c_int64), ("x_scale", C.c_void_p),
                ("x_rowptr", C.c_void_p), ("x_col", C.c_void_p)]


class CsrX:
    """Sparse attributes X_U (TPO_X_CSR): device tensors rowptr (int64,
    n_u + 1), col (int32, nnz) and val (float32, nnz), d_u columns."""

    def __init__(self, rowptr, col, val, d_u):
        self.rowptr, self.col, self.val, self.d_u = rowptr, col, val, int(d_u)
        self.dtype = "csr"

    @property
    def nnz(self) -> int:
        return int(self.col.numel())


class TpoOutputs(C.Structure):
    _fields_ = [("labels", C.c_void_p), ("embedding", C.c_void_p),
                ("objective", C.POINTER(C.c_double))]


class TpoStats(C.Structure):
    _fields_ = [("ms_ingest", C.c_double), ("ms_reduce", C.c_double), ("ms_propagate", C.c_double),
                ("ms_features", C.c_double), ("ms_embed", C.c_double), ("ms_onmf", C.c_double),
                ("ms_nci", C.c_double), ("ms_objective", C.c_double), ("ms_total", C.c_double),
                ("n_unique_edges", C.c_int64), ("guard_hits", C.c_int32),
                ("isolated_u", C.c_int32), ("isolated_v", C.c_int32),
                ("ms_spmm_v", C.c_double), ("ms_spmm_u", C.c_double),
                ("n_spmm_v", C.c_int32), ("n_spmm_u", C.c_int32),
                ("nci_rechecked", C.c_int32), ("nci_rounds", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_LIB = None


def load_library() -> C.CDLL:
    """Load the in-tree libtpo.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(lib_path):
        raise ImportError(f"{lib_path} is missing: build it with python -m paper_2405_11922_amd.build")
    lib = C.CDLL(lib_path)
    vp, sz = C.c_void_p, C.c_size_t
    i32 = C.c_int32
    lib.tpo_plan_create.argtypes = [C.POINTER(TpoProblem), C.POINTER(TpoParams), C.POINTER(vp)]
    lib.tpo_plan_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
    lib.tpo_plan_dims.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.tpo_execute.argtypes = [vp, C.POINTER(TpoInputs), vp, sz, vp, C.POINTER(TpoOutputs)]
    lib.tpo_execute_noalloc.argtypes = [vp, C.POINTER(TpoInputs), vp, C.POINTER(TpoOutputs)]
    lib.tpo_execute_resident.argtypes = [vp, C.POINTER(TpoInputs), vp, sz, vp, C.POINTER(TpoOutputs)]
    lib.tpo_plan_destroy.argtypes = [vp]
    lib.tpo_plan_destroy.restype = None
    lib.tpo_status_string.argtypes = [C.c_int]
    lib.tpo_status_string.restype = C.c_char_p
    lib.tpo_plan_last_error.argtypes = [vp]
    lib.tpo_plan_last_error.restype = C.c_char_p
    lib.tpo_plan_stats.argtypes = [vp, C.POINTER(TpoStats)]
    for name in ("tpo_stage_ingest", "tpo_stage_reduce", "tpo_stage_propagate"):
        getattr(lib, name).argtypes = [vp, C.POINTER(TpoInputs), vp, sz, vp]
    for name in ("tpo_stage_features", "tpo_stage_embed", "tpo_stage_onmf"):
        getattr(lib, name).argtypes = [vp, vp, sz, vp]
    lib.tpo_stage_nci.argtypes = [vp, vp, sz, vp, vp]
    lib.tpo_stage_objective.argtypes = [vp, vp, sz, vp, C.POINTER(C.c_double)]
    lib.tpo_plan_buffer.argtypes = [vp, vp, i32, C.POINTER(vp), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64), C.POINTER(i32)]
    lib.tpo_draw_normals.argtypes = [C.c_uint64, i32, C.c_int64, C.POINTER(C.c_double)]
    lib.tpo_e4m3_encode.argtypes = [C.c_float]
    lib.tpo_e4m3_encode.restype = C.c_uint8
    lib.tpo_abi_version.restype = i32
    for name in EXPORTED:
        if name not in ("tpo_plan_destroy", "tpo_status_string", "tpo_plan_last_error", "tpo_abi_version"):
            getattr(lib, name).restype = C.c_int
    if lib.tpo_abi_version() != TPO_ABI_VERSION:
        raise ImportError("libtpo ABI version mismatch")
    _LIB = lib
    return lib


def tpo_status_string(status: int) -> str:
    return load_library().tpo_status_string(status).decode()


def _check(status: int, plan=None):
    if status != 0:
        msg = ""
        if plan:
            msg = load_library().tpo_plan_last_error(plan).decode()
        raise TpoError(status, msg or tpo_status_string(status))


def _dptr(arr):
    import numpy as np
    if arr is None:
        return None
    a = np.ascontiguousarray(arr, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


X_DTYPES = {"f32": 0, "bf16": 1, "fp8": 2, "csr": 3}  # TPO_X_F32, TPO_X_BF16, TPO_X_FP8, TPO_X_CSR
_TORCH_XDT = {"torch.float32": "f32", "torch.bfloat16": "bf16", "torch.float8_e4m3fn": "fp8"}
_PLAN_XDT = {}  # plan handle -> x_dtype name, to check the tensors handed over


def tpo_plan_create(n_u, n_v, n_edges, d_u, *, k, alpha, gamma, d=0, q=20, oversample=10,
                    t_f=5, t_g=20, seed=0, weighted=False, timing=False, one_stream=False,
                    omega_reduce=None, g=None, omega=None, x_dtype="f32", nci="literal", x_nnz=0,
                    x_refine=1):
    """Returns an opaque plan handle (int).  x_dtype: "f32", "bf16", "fp8" or
    "csr" (X_U's element type; "csr": sparse FP32 rows with x_nnz stored
    entries, x_refine FP32 refinement steps after the FP8-Gram iteration)."""
    lib = load_library()
    if x_dtype not in X_DTYPES:
        raise TpoError(1, f"x_dtype must be one of {sorted(X_DTYPES)}")
    prob = TpoProblem(TPO_ABI_VERSION, int(n_u), int(n_v), int(d_u), int(n_edges), int(bool(weighted)),
                      X_DTYPES[x_dtype], int(x_nnz))
    keep = [_dptr(omega_reduce), _dptr(g), _dptr(omega)]
    flags = _flags(timing, one_stream, nci)
    par = TpoParams(TPO_ABI_VERSION, int(k), float(alpha), int(gamma), int(d), int(q), int(oversample),
                    int(t_f), int(t_g), flags, int(seed) & ((1 << 64) - 1),
                    keep[0][1] if keep[0] else None, keep[1][1] if keep[1] else None,
                    keep[2][1] if keep[2] else None, int(x_refine), 0)
    h = C.c_void_p()
    _check(lib.tpo_plan_create(C.byref(prob), C.byref(par), C.byref(h)))
    _PLAN_XDT[h.value] = x_dtype
    return h.value


def _flags(timing, one_stream, nci) -> int:
    if nci not in NCI_VARIANTS:
        raise ValueError(f"nci must be one of {NCI_VARIANTS}")
    return ((TPO_FLAG_TIMING if timing else 0) | (TPO_FLAG_ONE_STREAM if one_stream else 0)
            | (TPO_FLAG_NCI_PROCRUSTES if nci == "procrustes" else 0))


def tpo_e4m3_encode(v: float) -> int:
    """The E4M3 code the sparse-attribute form stages for the value v."""
    return int(load_library().tpo_e4m3_encode(float(v)))


def tpo_plan_destroy(plan) -> None:
    _PLAN_XDT.pop(plan, None)
    load_library().tpo_plan_destroy(plan)


def tpo_plan_workspace_bytes(plan) -> int:
    out = C.c_size_t()
    _check(load_library().tpo_plan_workspace_bytes(plan, C.byref(out)), plan)
    return int(out.value)


def tpo_plan_dims(plan):
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(load_library().tpo_plan_dims(plan, C.byref(a), C.byref(b), C.byref(c)), plan)
    return a.value, b.value, c.value


def _inputs(edge_u, edge_v, x_u, edge_w=None, plan=None, x_scale=None):
    if isinstance(x_u, CsrX):
        if plan in _PLAN_XDT and _PLAN_XDT[plan] != "csr":
            raise TpoError(1, f"sparse attributes given, the plan expects {_PLAN_XDT[plan]}")
        for t, dt in ((x_u.rowptr, "torch.int64"), (x_u.col, "torch.int32"), (x_u.val, "torch.float32")):
            if str(t.dtype) != dt or not t.is_contiguous():
                raise TpoError(1, "CsrX needs contiguous int64 rowptr, int32 col and float32 val tensors")
        return TpoInputs(edge_u.data_ptr() if edge_u is not None else None,
                         edge_v.data_ptr() if edge_v is not None else None,
                         edge_w.data_ptr() if edge_w is not None else None,
                         x_u.val.data_ptr(), 0, None, x_u.rowptr.data_ptr(), x_u.col.data_ptr())
    if plan in _PLAN_XDT and _PLAN_XDT[plan] == "csr":
        raise TpoError(1, "the plan expects sparse attributes (CsrX)")
    if x_u is not None and plan in _PLAN_XDT:
        want = _PLAN_XDT[plan]
        have = _TORCH_XDT.get(str(x_u.dtype))
        if have != want:
            raise TpoError(1, f"x_u is {x_u.dtype}, the plan expects {want}")
        if want == "fp8" and (x_scale is None or str(x_scale.dtype) != "torch.float32"
                              or x_scale.numel() != x_u.shape[1] or not x_scale.is_contiguous()):
            raise TpoError(1, "FP8 attributes need x_scale: a contiguous float32 tensor of d_u column scales")
    ld = x_u.stride(0) if x_u is not None else 0
    return TpoInputs(edge_u.data_ptr() if edge_u is not None else None,
                     edge_v.data_ptr() if edge_v is not None else None,
                     edge_w.data_ptr() if edge_w is not None else None,
                     x_u.data_ptr(), ld, x_scale.data_ptr() if x_scale is not None else None, None, None)


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream


def tpo_execute(plan, edge_u, edge_v, x_u, workspace, labels, embedding=None, edge_w=None,
                stream=None, x_scale=None):
    """Runs the whole method; returns (obj1, trace form).  x_scale: the
    column scales of FP8 attributes."""
    lib = load_library()
    inp = _inputs(edge_u, edge_v, x_u, edge_w, plan, x_scale)
    obj = (C.c_double * 2)()
    out = TpoOutputs(labels.data_ptr(), embedding.data_ptr() if embedding is not None else None,
                     C.cast(obj, C.POINTER(C.c_double)))
    _check(lib.tpo_execute(plan, C.byref(inp), workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                           _stream(stream), C.byref(out)), plan)
    return float(obj[0]), float(obj[1])


def tpo_execute_resident(plan, x_u, workspace, labels, embedding=None, stream=None, x_scale=None):
    """tpo_execute on the graph a previous job ingested into `workspace`
    (ingest skipped, the CSR reused); returns (obj1, trace form)."""
    lib = load_library()
    inp = _inputs(None, None, x_u, None, plan, x_scale)
    obj = (C.c_double * 2)()
    out = TpoOutputs(labels.data_ptr(), embedding.data_ptr() if embedding is not None else None,
                     C.cast(obj, C.POINTER(C.c_double)))
    _check(lib.tpo_execute_resident(plan, C.byref(inp), workspace.data_ptr(),
                                    workspace.numel() * workspace.element_size(), _stream(stream), C.byref(out)), plan)
    return float(obj[0]), float(obj[1])


def tpo_execute_noalloc(plan, edge_u, edge_v, x_u, labels, embedding=None, edge_w=None,
                        stream=None, x_scale=None):
    """tpo_execute with the library's own device array as the workspace (no
    allocation anywhere in the call); returns (obj1, trace form)."""
    lib = load_library()
    inp = _inputs(edge_u, edge_v, x_u, edge_w, plan, x_scale)
    obj = (C.c_double * 2)()
    out = TpoOutputs(labels.data_ptr() if labels is not None else None,
                     embedding.data_ptr() if embedding is not None else None,
                     C.cast(obj, C.POINTER(C.c_double)))
    _check(lib.tpo_execute_noalloc(plan, C.byref(inp), _stream(stream), C.byref(out)), plan)
    return float(obj[0]), float(obj[1])


def _ws(workspace):
    return workspace.data_ptr(), workspace.numel() * workspace.element_size()


def tpo_stage_ingest(plan, edge_u, edge_v, x_u, workspace, edge_w=None, stream=None, x_scale=None):
    inp = _inputs(edge_u, edge_v, x_u, edge_w, plan, x_scale)
    _check(load_library().tpo_stage_ingest(plan, C.byref(inp), *_ws(workspace), _stream(stream)), plan)


def tpo_stage_reduce(plan, edge_u, edge_v, x_u, workspace, edge_w=None, stream=None, x_scale=None):
    inp = _inputs(edge_u, edge_v, x_u, edge_w, plan, x_scale)
    _check(load_library().tpo_stage_reduce(plan, C.byref(inp), *_ws(workspace), _stream(stream)), plan)


def tpo_stage_propagate(plan, workspace, stream=None):
    _check(load_library().tpo_stage_propagate(plan, None, *_ws(workspace), _stream(stream)), plan)


def tpo_stage_features(plan, workspace, stream=None):
    _check(load_library().tpo_stage_features(plan, *_ws(workspace), _stream(stream)), plan)


def tpo_stage_embed(plan, workspace, stream=None):
    _check(load_library().tpo_stage_embed(plan, *_ws(workspace), _stream(stream)), plan)


def tpo_stage_onmf(plan, workspace, stream=None):
    _check(load_library().tpo_stage_onmf(plan, *_ws(workspace), _stream(stream)), plan)


def tpo_stage_nci(plan, workspace, labels=None, stream=None):
    _check(load_library().tpo_stage_nci(plan, *_ws(workspace), _stream(stream),
                                        labels.data_ptr() if labels is not None else None), plan)


def tpo_stage_objective(plan, workspace, stream=None):
    obj = (C.c_double * 2)()
    _check(load_library().tpo_stage_objective(plan, *_ws(workspace), _stream(stream),
                                              C.cast(obj, C.POINTER(C.c_double))), plan)
    return float(obj[0]), float(obj[1])


def tpo_plan_buffer(plan, workspace, name):
    """A torch view of workspace buffer `name` (see BUF)."""
    import torch
    ptr, rows, cols, dt = C.c_void_p(), C.c_int64(), C.c_int64(), C.c_int32()
    _check(load_library().tpo_plan_buffer(plan, workspace.data_ptr(), BUF[name], C.byref(ptr), C.byref(rows),
                                          C.byref(cols), C.byref(dt)), plan)
    dtype = {1: torch.int32, 2: torch.float32, 3: torch.float64}[dt.value]
    esz = torch.empty((), dtype=dtype).element_size()
    off = ptr.value - workspace.data_ptr()
    assert off % esz == 0
    n = rows.value * cols.value
    flat = workspace.view(torch.uint8)[off: off + n * esz].view(dtype)
    return flat.view(rows.value, cols.value) if name in _MATRICES else flat


def tpo_plan_stats(plan) -> dict:
    st = TpoStats()
    _check(load_library().tpo_plan_stats(plan, C.byref(st)), plan)
    return st.as_dict()


def tpo_draw_normals(seed: int, stream: int, count: int):
    import numpy as np
    out = np.empty(count, dtype=np.float64)
    _check(load_library().tpo_draw_normals(int(seed) & ((1 << 64) - 1), int(stream), int(count),
                                           out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


@dataclass
class Plan:
    """RAII holder of a plan handle plus its device workspace (torch)."""

    handle: int
    workspace: object
    n_u: int
    k: int

    @classmethod
    def create(cls, n_u, n_v, n_edges, d_u, device="cuda", **params):
        """params: those of tpo_plan_create (x_dtype "f32" or "bf16" included)."""
        import torch
        h = tpo_plan_create(n_u, n_v, n_edges, d_u, **params)
        nbytes = tpo_plan_workspace_bytes(h)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        ws = ws[off: off + nbytes]
        return cls(h, ws, int(n_u), int(params["k"]))

    def buffer(self, name):
        return tpo_plan_buffer(self.handle, self.workspace, name)

    def close(self):
        if self.handle:
            tpo_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cluster(edge_u, edge_v, x_u, *, n_v, k, **kw):
    """Cluster the target nodes of one ABG given as device tensors
    (edge_u/edge_v int32 [E], x_u float32 or bfloat16 [n_u, d_u], optional edge_w float32).
    Returns (labels int32 [n_u], embedding float32 [n_u, k], (obj1, trace), stats)."""
    return cluster_sized(edge_u, edge_v, x_u, n_v=n_v, k=k, **kw)


def cluster_target_v(edge_u, edge_v, x_v, *, n_u, k, **kw):
    """Cluster the nodes of V instead of U: the same graph read from the
    other side (edge (u, v) taken as (v, u)), with x_v [n_v, d_V] as the
    target's attributes.  The call passes edge_v as the target side's column
    and edge_u as the other side's; nothing is copied.  Returns what cluster
    returns, for the n_v nodes of V."""
    return cluster_sized(edge_v, edge_u, x_v, n_v=n_u, k=k, **kw)


def cluster_sized(edge_u, edge_v, x_u, *, n_v, k, alpha=0.5, gamma=5, d=0, q=20, oversample=10,
                  t_f=5, t_g=20, seed=0, edge_w=None, omega_reduce=None, g=None, omega=None,
                  timing=False, nci="literal", x_scale=None):
    import torch
    n_u, d_u = x_u.shape
    xdt = _TORCH_XDT.get(str(x_u.dtype), "f32")
    plan = Plan.create(n_u, n_v, edge_u.numel(), d_u, device=x_u.device, k=k, alpha=alpha,
                       gamma=gamma, d=d, q=q, oversample=oversample, t_f=t_f, t_g=t_g, seed=seed,
                       weighted=edge_w is not None, timing=timing, omega_reduce=omega_reduce,
                       g=g, omega=omega, x_dtype=xdt, nci=nci)
    try:
        labels = torch.empty(n_u, dtype=torch.int32, device=x_u.device)
        emb = torch.empty(n_u, k, dtype=torch.float32, device=x_u.device)
        obj = tpo_execute(plan.handle, edge_u, edge_v, x_u, plan.workspace, labels, emb, edge_w, x_scale=x_scale)
        stats = tpo_plan_stats(plan.handle)
    finally:
        plan.close()
    return labels, emb, obj, stats
