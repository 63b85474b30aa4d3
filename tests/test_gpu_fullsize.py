"""Full-size parity: the 64^3 rock-salt lattice and the 10^6-ion electrolyte,
in the launch configuration the benchmark uses (one plan sized to N).

Expected values come from ``tests/golden/oracle_*.json``, written by
``tests/golden/make_golden.py`` with the FP64 oracle: every energy part, S(k)
at 4096 sampled k vectors, and forces / dE/dq on 4096 particles stratified
over the box (one from each block of a 16^3 grid).  Forces and dE/dq are
checked by relative norm and per element (max deviation over the RMS of the
reference); the net force is checked over all particles.
"""
import functools
import json
import os

import numpy as np
import pytest

from paper_1708_01135_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = {"fp64": 1e-10, "mixed": 1e-6}
TOL_ELEM = {"fp64": 1e-9, "mixed": 1e-5}


@functools.lru_cache(maxsize=None)
def golden(name):
    with open(os.path.join(GOLDEN, f"oracle_{name}_s0.json")) as f:
        return json.load(f)


@functools.lru_cache(maxsize=None)
def system(name):
    s = wl.make_config(name, 0)
    ck = golden(name)["input_checksum"]
    got = {"sum_pos": np.sum(s.pos), "sum_pos2": np.sum(s.pos * s.pos), "sum_q": np.sum(s.q),
           "sum_qx": np.sum(s.q * s.pos[:, 0])}
    for k, v in ck.items():
        assert abs(got[k] - v) <= 1e-12 * max(1.0, abs(v)), f"generated input differs from the golden one ({k})"
    return s


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["rocksalt64", "electrolyte1m"])
def test_fullsize_against_oracle(name, precision):
    import torch
    from paper_1708_01135_amd import ewald as ew
    g = golden(name)
    s = system(name)
    dev = torch.device("cuda:0")
    pos = torch.tensor(s.pos, device=dev)
    q = torch.tensor(s.q, device=dev)
    with ew.Plan(s.n, s.box_L, s.alpha, s.r_c, s.k_max, precision) as p:
        e, f, dq = p.energy_forces(pos, q, True, True)
        torch.cuda.synchronize()
        assert p.status() == ew.OK
        kv = p.kset()
        sk = p.structure_factor()
    e, f, dq = e.cpu().numpy(), f.cpu().numpy(), dq.cpu().numpy()
    tol = TOL[precision]
    eref = np.array(g["energy"])
    scale = np.abs(eref[1:4]).max()
    rel_e = abs(e[0] - eref[0]) / abs(eref[0])
    parts = [abs(e[i] - eref[i]) / max(abs(eref[i]), 1e-12 * scale) for i in range(1, 5)]
    t = np.array(g["targets"])
    fref, dref = np.array(g["forces"]), np.array(g["dEdq"])
    rel_f = np.linalg.norm(f[t] - fref) / np.linalg.norm(fref)
    rel_d = np.linalg.norm(dq[t] - dref) / np.linalg.norm(dref)
    elem_f = np.abs(f[t] - fref).max() / np.sqrt(np.mean(fref * fref))
    elem_d = np.abs(dq[t] - dref).max() / np.sqrt(np.mean(dref * dref))
    lookup = {tuple(v): i for i, v in enumerate(kv.tolist())}
    idx = np.array([lookup[tuple(v)] for v in g["k_samples"]])
    sref = np.array(g["sk_re"]) + 1j * np.array(g["sk_im"])
    s_err = np.abs(sk[idx] - sref).max() / np.sqrt(s.n)
    net = np.abs(f.sum(axis=0)).max() / np.abs(f).sum()
    print(f"{name} {precision}: rel_E={rel_e:.2e} parts={['%.1e' % x for x in parts]} rel_F={rel_f:.2e} "
          f"rel_dEdq={rel_d:.2e} elem_F={elem_f:.2e} elem_dEdq={elem_d:.2e} S_err/sqrtN={s_err:.2e} "
          f"net={net:.1e} samples={len(t)}", flush=True)
    assert len(t) >= 4096
    assert rel_e <= tol and max(parts) <= tol
    assert rel_f <= tol and rel_d <= tol
    assert elem_f <= TOL_ELEM[precision] and elem_d <= TOL_ELEM[precision]
    assert s_err <= 1e-12  # S(k) is FP64 in both precisions
    assert net <= (1e-12 if precision == "fp64" else 1e-7)
