"""Adjoint (autograd) of the Ewald energy: dL/dpos = -g F, dL/dq = g dE/dq.

Checked against the FP64 oracle's forces and dE/dq, and against central
finite differences of the library's own FP64 energy (h = 1e-4, 64 random
particles of the 64^3 lattice).  Finite-difference components for which the
moved particle has a pair within h of the cutoff are skipped: the truncated
real-space energy is discontinuous there (a pair entering or leaving r_c).
"""
import functools
import json
import os

import numpy as np
import pytest

import oracle
from paper_1708_01135_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@functools.lru_cache(maxsize=None)
def golden(name):
    with open(os.path.join(GOLDEN, f"oracle_{name}_s0.json")) as f:
        return json.load(f)


def grads(s, precision, scale=1.0):
    import torch
    from paper_1708_01135_amd import ewald as ew
    dev = torch.device("cuda:0")
    pos = torch.tensor(s.pos, device=dev, requires_grad=True)
    q = torch.tensor(s.q, device=dev, requires_grad=True)
    plan = ew.Plan(s.n, s.box_L, s.alpha, s.r_c, s.k_max, precision)
    e = ew.ewald_energy(pos, q, plan)
    (scale * e).backward()
    torch.cuda.synchronize()
    assert plan.status() == ew.OK
    out = float(e.item()), pos.grad.cpu().numpy(), q.grad.cpu().numpy()
    plan.release()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adjoint_matches_oracle_small(precision):
    s = wl.make_config("rocksalt8", 2)
    en, f, dq = oracle.energy_forces(s.pos, s.q, s.box_L, s.alpha, s.r_c, s.k_max, oracle.FAST)
    e, gp, gq = grads(s, precision, scale=2.5)
    tol = 1e-10 if precision == "fp64" else 1e-6
    assert abs(e - en[0]) <= tol * abs(en[0])
    assert np.linalg.norm(gp - (-2.5 * f)) <= tol * 2.5 * np.linalg.norm(f)
    assert np.linalg.norm(gq - 2.5 * dq) <= tol * 2.5 * np.linalg.norm(dq)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adjoint_rocksalt64_oracle_and_finite_differences(precision):
    import torch
    from paper_1708_01135_amd import ewald as ew
    g = golden("rocksalt64")
    s = wl.make_config("rocksalt64", 0)
    e, gp, gq = grads(s, precision)
    t = np.array(g["targets"])
    tol = 1e-10 if precision == "fp64" else 1e-6
    fref, dref = np.array(g["forces"]), np.array(g["dEdq"])
    rel_f = np.linalg.norm(-gp[t] - fref) / np.linalg.norm(fref)
    rel_q = np.linalg.norm(gq[t] - dref) / np.linalg.norm(dref)
    print(f"adjoint rocksalt64 {precision}: rel_F={rel_f:.2e} rel_dEdq={rel_q:.2e}", flush=True)
    assert rel_f <= tol and rel_q <= tol

    # central differences of the FP64 energy on 64 random particles
    dev = torch.device("cuda:0")
    pos0 = torch.tensor(s.pos, device=dev)
    q0 = torch.tensor(s.q, device=dev)
    h = 1e-4
    rng = np.random.default_rng(7)
    sel = rng.choice(s.n, 64, replace=False)
    L, rc = s.box_L, s.r_c
    with ew.Plan(s.n, s.box_L, s.alpha, s.r_c, s.k_max, "fp64") as p:
        def energy(pos, q):
            return p.energy(pos, q)[0].item()
        worst_f, worst_q, checked = 0.0, 0.0, 0
        frms = np.sqrt(np.mean(gp ** 2))
        for i in sel:
            d = s.pos - s.pos[i]
            d -= L * np.round(d / L)
            r = np.sqrt(np.einsum("jk,jk->j", d, d))
            for ax in range(3):
                # skip if any pair distance can cross r_c within the step
                if np.any(np.abs(r - rc) <= 2 * h):
                    continue
                pp, pm = pos0.clone(), pos0.clone()
                pp[i, ax] += h
                pm[i, ax] -= h
                fd = (energy(pp, q0) - energy(pm, q0)) / (2 * h)
                worst_f = max(worst_f, abs(fd - gp[i, ax]) / frms)
                checked += 1
            qp, qm = q0.clone(), q0.clone()
            qp[i] += h
            qm[i] -= h
            fdq = (energy(pos0, qp) - energy(pos0, qm)) / (2 * h)
            worst_q = max(worst_q, abs(fdq - gq[i]) / np.sqrt(np.mean(gq ** 2)))
    print(f"  finite differences: {checked} position components, worst |fd-grad|/rms: F {worst_f:.2e}, "
          f"dEdq {worst_q:.2e}", flush=True)
    assert checked >= 150
    # FD truncation O(h^2) plus FP64 cancellation eps*|E|/h (|E| ~ 2e5): ~1e-6 of the rms force
    assert worst_f <= 2e-5 and worst_q <= 2e-5
