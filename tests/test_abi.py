"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every entry point include/tpo.h declares, validates arguments, and its
Gaussian generator reproduces the seeded input generator bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import abg_synth as synth
import paper_2405_11922_amd as tpo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    with open(os.path.join(ROOT, "include", "tpo.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tpo_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = tpo.load_library()
    syms = _declared_symbols()
    assert "tpo_execute" in syms and "tpo_plan_create" in syms and len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(tpo.EXPORTED)


def test_abi_version():
    assert tpo.load_library().tpo_abi_version() == tpo.TPO_ABI_VERSION


@pytest.mark.parametrize("seed,stream,count", [(0, 0, 1001), (12345, 1, 64 * 64), (2**63 + 7, 2, 4000)])
def test_native_generator_matches_input_generator(seed, stream, count):
    a = tpo.tpo_draw_normals(seed, stream, count)
    b = synth.splitmix64_normals(seed, stream, count)
    assert np.array_equal(a, b)


def test_plan_dims_and_workspace():
    h = tpo.tpo_plan_create(200_000, 400_000, 4_000_000, 256, k=20, alpha=0.5, gamma=10, d=64)
    try:
        assert tpo.tpo_plan_dims(h) == synth.sketch_widths(256, 64, 20, 10)
        ws = tpo.tpo_plan_workspace_bytes(h)
        assert 100e6 < ws < 8e9
    finally:
        tpo.tpo_plan_destroy(h)
    h = tpo.tpo_plan_create(2000, 3000, 20_000, 64, k=5, alpha=0.5, gamma=5, d=0)
    try:
        assert tpo.tpo_plan_dims(h) == (64, 0, 15)
    finally:
        tpo.tpo_plan_destroy(h)


@pytest.mark.parametrize("kw", [
    dict(k=0), dict(k=65), dict(alpha=1.0), dict(alpha=-0.1), dict(gamma=-1), dict(q=-1),
    dict(t_f=-1), dict(t_g=-2), dict(oversample=-1), dict(k=40, d=16),
])
def test_plan_create_rejects_bad_parameters(kw):
    base = dict(k=5, alpha=0.5, gamma=3, d=0)
    base.update(kw)
    with pytest.raises(tpo.TpoError) as e:
        h = tpo.tpo_plan_create(100, 100, 500, 32, **base)
        tpo.tpo_plan_destroy(h)
    assert e.value.status == 1


@pytest.mark.parametrize("shape", [(0, 10, 5, 8), (10, 0, 5, 8), (10, 10, -1, 8), (10, 10, 5, 0),
                                   (10, 10, 2**31, 8), (10, 10, 5, 200)])
def test_plan_create_rejects_bad_shapes(shape):
    with pytest.raises(tpo.TpoError):
        h = tpo.tpo_plan_create(*shape, k=2, alpha=0.5, gamma=2)
        tpo.tpo_plan_destroy(h)


def test_status_strings():
    assert tpo.tpo_status_string(0) == "ok"
    assert tpo.tpo_status_string(3) == "workspace too small"


def test_attribute_dtype_checked():
    """x_dtype must be TPO_X_F32 (0), TPO_X_BF16 (1) or TPO_X_FP8 (2); the
    binding refuses other names, a tensor whose dtype is not the plan's, and
    FP8 attributes without their column scales."""
    import ctypes as C

    import torch

    lib = tpo.load_library()
    par = tpo.TpoParams(tpo.TPO_ABI_VERSION, 5, 0.5, 3, 0, 20, 10, 5, 20, 0, 0, None, None, None)
    for xdt, nnz, want in ((0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 800, 0), (3, -1, 1), (3, 1 << 31, 1), (4, 0, 1),
                           (-1, 0, 1)):
        prob = tpo.TpoProblem(tpo.TPO_ABI_VERSION, 100, 100, 32, 500, 0, xdt, nnz)
        h = C.c_void_p()
        st = lib.tpo_plan_create(C.byref(prob), C.byref(par), C.byref(h))
        assert st == want, (xdt, nnz, st)
        if st == 0:
            lib.tpo_plan_destroy(h)
    with pytest.raises(tpo.TpoError) as e:
        tpo.tpo_plan_create(100, 100, 500, 32, k=5, alpha=0.5, gamma=3, x_dtype="fp4")
    assert e.value.status == 1
    h = tpo.tpo_plan_create(100, 100, 500, 32, k=5, alpha=0.5, gamma=3, x_dtype="bf16")
    try:
        with pytest.raises(tpo.TpoError) as e:
            tpo.tpo_stage_reduce(h, None, None, torch.zeros(100, 32, dtype=torch.float32), None)
        assert e.value.status == 1
    finally:
        tpo.tpo_plan_destroy(h)
    h = tpo.tpo_plan_create(100, 100, 500, 32, k=5, alpha=0.5, gamma=3, x_dtype="fp8")
    try:
        x8 = torch.zeros(100, 32, dtype=torch.float8_e4m3fn)
        for bad in (None, torch.ones(31), torch.ones(32, dtype=torch.float64)):
            with pytest.raises(tpo.TpoError) as e:
                tpo.tpo_stage_reduce(h, None, None, x8, None, x_scale=bad)
            assert e.value.status == 1
    finally:
        tpo.tpo_plan_destroy(h)
    # the C ABI refuses FP8 inputs without scales before touching any memory
    prob = tpo.TpoProblem(tpo.TPO_ABI_VERSION, 100, 100, 32, 0, 0, 2)
    h = C.c_void_p()
    assert lib.tpo_plan_create(C.byref(prob), C.byref(par), C.byref(h)) == 0
    try:
        inp = tpo.TpoInputs(None, None, None, 4096, 32, None)
        ws = C.c_void_p(1 << 20)  # never dereferenced: the inputs are rejected first
        nbytes = C.c_size_t()
        lib.tpo_plan_workspace_bytes(h, C.byref(nbytes))
        assert lib.tpo_stage_reduce(h, C.byref(inp), ws, nbytes.value, None) == 1
        assert b"x_scale" in lib.tpo_plan_last_error(h)
    finally:
        lib.tpo_plan_destroy(h)


def test_serving_stream_recipe():
    """The serving workload's generator: Poisson arrivals in order, shapes
    within the recipe's ranges, k <= 2 d_eff for every request."""
    shapes, reqs = synth.serving_stream(500, 200.0, 16, seed=3)
    assert len(shapes) == 16 and len(reqs) == 500
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0)
    assert 1.5 < arr[-1] < 3.5  # 500 arrivals at 200/s
    for n_u, n_v, e, k, d_u, _ in shapes:
        assert 1_000 <= n_u <= 500_000 and n_v == round(1.5 * n_u)
        assert 10 * n_u - 1 <= e <= 30 * n_u + 1
        assert 2 <= k <= 64 and d_u in (32, 128, 256)
    for r in reqs:
        d_eff = r.d
        assert r.k <= 2 * d_eff


def test_serving_worker_cap():
    from paper_2405_11922_amd import serve

    with pytest.raises(ValueError):
        serve.Server(device="cpu", workers=serve.MAX_WORKERS + 1).run([], realtime=False)


def test_serving_pool_and_summary():
    """The serving workspace pool (first fit, 256-byte aligned, merged on
    release) and the latency summary, on the host."""
    from paper_2405_11922_amd import serve

    p = serve._Pool(10_000)
    a, b, c = p.take(1000), p.take(3000), p.take(5000)
    assert (a, b, c) == (0, 1024, 4096)
    assert p.take(1000) is None  # 784 bytes left
    p.give(b, 3000)
    assert p.take(2000) == 1024
    p.give(a, 1000)
    p.give(c, 5000)
    p.give(1024, 2000)
    assert p.free == [(0, 10_000)]
    res = [serve.Result(i, 0.1 * i, 0.1 * i, 0.1 * i + 0.02 + 0.001 * i, started=0.1 * i, exec_s=0.02)
           for i in range(10)]
    res.append(serve.Result(10, 1.0, 1.0, 1.0, error="workspace above the HBM budget"))
    s = serve.summarize(res)
    assert s["jobs"] == 10 and s["failed"] == 1
    assert abs(s["p50_ms"] - 24.5) < 1e-6 and abs(s["exec_p50_ms"] - 20.0) < 1e-9
    assert abs(s["jobs_per_s"] - 10 / (0.9 + 0.029)) < 1e-9


def test_noalloc_entry_point_rejects_jobs_beyond_its_array():
    """The no-allocation entry point refuses, before any device work, a job
    whose workspace exceeds its fixed array, and says why."""
    with open(os.path.join(ROOT, "include", "tpo.h")) as f:
        m = re.search(r"#define TPO_NOALLOC_MAX_BYTES \(\(size_t\)(\d+) << (\d+)\)", f.read())
    assert m and int(m.group(1)) << int(m.group(2)) == tpo.TPO_NOALLOC_MAX_BYTES
    lib = tpo.load_library()
    h = tpo.tpo_plan_create(200_000, 400_000, 4_000_000, 256, k=20, alpha=0.5, gamma=10, d=64)
    try:
        assert tpo.tpo_plan_workspace_bytes(h) > tpo.TPO_NOALLOC_MAX_BYTES
        inp = tpo.TpoInputs(None, None, None, None, 256, None)
        out = tpo.TpoOutputs(None, None, None)
        st = lib.tpo_execute_noalloc(h, ctypes.byref(inp), None, ctypes.byref(out))
        assert st == 3  # TPO_ENOMEM
        assert b"no-allocation" in lib.tpo_plan_last_error(h)
    finally:
        tpo.tpo_plan_destroy(h)
    h = tpo.tpo_plan_create(2000, 3000, 20_000, 64, k=5, alpha=0.5, gamma=5, timing=True)
    try:
        assert tpo.tpo_plan_workspace_bytes(h) <= tpo.TPO_NOALLOC_MAX_BYTES
        st = lib.tpo_execute_noalloc(h, ctypes.byref(inp), None, ctypes.byref(out))
        assert st == 1  # TPO_EINVAL: a timing plan would create events
    finally:
        tpo.tpo_plan_destroy(h)
