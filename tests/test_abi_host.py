"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a GPU."""
import ctypes
import glob
import os
import re

import pytest

from paper_1708_01135_amd import ewald as ew
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(ewald_\w+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = ew.library()
    names = header_functions()
    assert len(names) >= 26
    assert "ewald_server_submit" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    for st in (0, -1, -2, -3, -4, -5, -6, -7):
        assert ew.status_string(st)
    assert "unknown" in ew.status_string(7)
    assert "scratch" in ew.status_string(ew.ERR_SCRATCH)


BAD = [
    dict(n_max=0), dict(n_max=(1 << 25) + 1), dict(box_L=0.0), dict(box_L=-1.0), dict(box_L=float("nan")), dict(alpha=0.0),
    dict(alpha=float("inf")), dict(r_c=0.0), dict(r_c=8.5), dict(k_max=0), dict(k_max=ew.K_MAX_LIMIT + 1),
    dict(precision=2), dict(device=-1), dict(flags=32), dict(flags=-1),
]


@pytest.mark.parametrize("bad", BAD)
def test_invalid_parameters_rejected_without_gpu(bad):
    kw = dict(n_max=512, box_L=8.0, alpha=0.9, r_c=4.0, k_max=8, precision=0, device=0, flags=0)
    kw.update(bad)
    p = ew.make_params(**kw)
    assert ew.validate(p) == ew.ERR_INVALID_ARG
    assert ew.workspace_bytes(p) == 0
    h = ctypes.c_void_p(123)
    assert ew.library().ewald_plan(ctypes.byref(p), ctypes.byref(h)) == ew.ERR_INVALID_ARG
    assert h.value is None  # *out cleared on failure


def test_vector_alu_and_graph_flags_are_valid():
    for f in (ew.FLAG_VALU_GATHER, ew.FLAG_VALU_SK, ew.FLAG_VALU_GATHER | ew.FLAG_VALU_SK, ew.FLAG_NO_GRAPH,
              ew.FLAG_VALU_GATHER | ew.FLAG_VALU_SK | ew.FLAG_NO_GRAPH):
        assert ew.validate(ew.make_params(512, 8.0, 0.9, 4.0, 8, flags=f)) == ew.OK
    p = ew.make_params(512, 8.0, 0.9, 4.0, 8, flags=ew.FLAG_VALU_GATHER)
    assert ew.workspace_bytes(p) == ew.workspace_bytes(ew.make_params(512, 8.0, 0.9, 4.0, 8))


def test_null_handling():
    lib = ew.library()
    p = ew.make_params(512, 8.0, 0.9, 4.0, 8)
    assert ew.validate(p) == ew.OK
    assert lib.ewald_plan(ctypes.byref(p), None) == ew.ERR_INVALID_ARG
    lib.ewald_release(None)  # no-op
    assert lib.ewald_energy_forces(None, 10, 1, 1, 1, None, None) == ew.ERR_INVALID_ARG
    assert lib.ewald_plan_status(None) == ew.ERR_INVALID_ARG
    assert lib.ewald_plan_kcount(None) == 0
    assert lib.ewald_plan_set_stream(None, None) == ew.ERR_INVALID_ARG
    assert lib.ewald_debug_copy_sk(None, None, None) == ew.ERR_INVALID_ARG
    assert lib.ewald_profile_enable(None, 1) == ew.ERR_INVALID_ARG
    # batches: count outside 1 .. EWALD_BATCH_MAX, or NULL arrays and plans
    vp = ctypes.c_void_p
    one = (vp * 1)(None)
    n1 = (ctypes.c_int64 * 1)(10)
    for count in (0, -1, ew.BATCH_MAX + 1):
        assert lib.ewald_energy_forces_batch(count, one, n1, one, one, one, None, None, None, None,
                                             None) == ew.ERR_INVALID_ARG
    assert lib.ewald_energy_forces_batch(1, None, n1, one, one, one, None, None, None, None, None) == ew.ERR_INVALID_ARG
    assert lib.ewald_energy_forces_batch(1, one, n1, one, one, one, None, None, None, None, None) == ew.ERR_INVALID_ARG


def test_workspace_bytes_scale_with_capacity():
    small = ew.workspace_bytes(ew.make_params(1000, 8.0, 0.9, 4.0, 8))
    big = ew.workspace_bytes(ew.make_params(100000, 8.0, 0.9, 4.0, 8))
    mixed = ew.workspace_bytes(ew.make_params(100000, 8.0, 0.9, 4.0, 8, precision="mixed"))
    assert 0 < small < big
    assert mixed < big  # FP32 gather coefficients


@pytest.mark.parametrize("K", [1, 2, 8, 13, 20, 40])
def test_kset_size_matches_oracle(K):
    assert ew.kset_size(K) == len(oracle.kset(K, half=True))


def test_plan_without_gpu_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except Exception:
        pass
    p = ew.make_params(64, 4.0, 1.0, 2.0, 4)
    h = ctypes.c_void_p()
    st = ew.library().ewald_plan(ctypes.byref(p), ctypes.byref(h))
    assert st == ew.ERR_DEVICE and h.value is None


@pytest.mark.parametrize("bad", [dict(n_streams=0), dict(n_streams=17), dict(precision=3), dict(flags=4),
                                 dict(device=-1)])
def test_server_rejects_bad_parameters_without_gpu(bad):
    kw = dict(device=0, n_streams=4, precision=ew.MIXED, flags=0, hbm_budget=0)
    kw.update(bad)
    prm = ew.ServerParams(kw["device"], kw["n_streams"], kw["precision"], kw["flags"], kw["hbm_budget"])
    h = ctypes.c_void_p(123)
    assert ew.library().ewald_server_create(ctypes.byref(prm), ctypes.byref(h)) == ew.ERR_INVALID_ARG
    assert h.value is None


def test_server_null_handling_and_clock():
    import time
    lib = ew.library()
    assert lib.ewald_server_create(None, None) == ew.ERR_INVALID_ARG
    lib.ewald_server_destroy(None)
    t = ctypes.c_int64()
    assert lib.ewald_server_submit(None, 0, 1, 1, 1, 1, None, None, ctypes.byref(t)) == ew.ERR_INVALID_ARG
    assert lib.ewald_server_wait(None, 0, None, None) == ew.ERR_INVALID_ARG
    assert lib.ewald_server_drain(None) == ew.ERR_INVALID_ARG
    # the server clock is CLOCK_MONOTONIC, the clock of time.perf_counter on Linux
    a = time.perf_counter()
    c = ew.Server.clock()
    b = time.perf_counter()
    assert a - 1e-3 <= c <= b + 1e-3


@pytest.mark.skipif(__import__("torch").cuda.is_available(), reason="checks the no-GPU error path")
def test_server_without_gpu_reports_device_error():
    prm = ew.ServerParams(0, 4, ew.MIXED, 0, 0)
    h = ctypes.c_void_p()
    assert ew.library().ewald_server_create(ctypes.byref(prm), ctypes.byref(h)) == ew.ERR_DEVICE


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and r.stdout == ""


def test_binding_rejects_mis_shaped_outputs_without_gpu():
    # caller-given outputs are checked before any pointer reaches the library
    import torch
    n = 10
    e = torch.empty(5, dtype=torch.float64)  # host tensor: not a device tensor
    with pytest.raises(ValueError):
        ew._check_outputs((e, None, None), n)
    with pytest.raises(ValueError):
        ew._check_outputs((torch.empty(4, dtype=torch.float64), None, None), n)
