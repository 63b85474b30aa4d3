"""The allocation-free evaluation (ewald_energy_forces_noalloc): per-evaluation
buffers in the library's static device scratch instead of a plan workspace.

Checked through the C ABI against ewald_energy_forces on the same inputs (the
same kernels and launch shapes, so bitwise equal) and against the FP64 oracle
to the parity bars, on two calls in a row of which the second has fewer
particles in another box (the scratch keeps the first call's contents, so
what must start at zero has to be cleared by the call itself).
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1708_01135_amd import workloads as wl

from gpu_helpers import compare

pytestmark = pytest.mark.gpu


def _cases():
    s = wl.make_config("rocksalt8", 0)
    big = (s.pos, s.q, s.box_L, s.alpha, s.r_c, s.k_max)
    pos, q = wl.random_neutral(300, 7.0, 5)
    small = (pos, q, 7.0, 0.9, 3.5, 8)
    return big, small


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_existing_entry_point(precision):
    import torch
    from paper_1708_01135_amd import ewald as ew
    dev = torch.device("cuda:0")
    for step, (pos, q, L, a, rc, K) in enumerate(_cases()):
        n = len(q)
        print(f"noalloc {precision} call {step}: n={n} L={L} K={K}", flush=True)
        tp = torch.tensor(pos, dtype=torch.float64, device=dev)
        tq = torch.tensor(q, dtype=torch.float64, device=dev)
        out = (torch.full((5,), np.nan, dtype=torch.float64, device=dev),
               torch.full((n, 3), np.nan, dtype=torch.float64, device=dev),
               torch.full((n,), np.nan, dtype=torch.float64, device=dev))
        with ew.Plan(512, L, a, rc, K, precision) as ref_plan, \
                ew.Plan(512, L, a, rc, K, precision, flags=ew.FLAG_NO_WORKSPACE) as plan:
            e, f, g = plan.energy_forces_noalloc(tp, tq, out)
            er, fr, gr = ref_plan.energy_forces(tp, tq, True, True)
            torch.cuda.synchronize()
            assert plan.status() == ew.OK and ref_plan.status() == ew.OK
            # a plan without workspace takes no other evaluation
            st = ew.library().ewald_energy_forces(plan.handle, n, tp.data_ptr(), tq.data_ptr(),
                                                  out[0].data_ptr(), None, None)
            assert st == ew.ERR_INVALID_ARG
            got = (e.cpu().numpy(), f.cpu().numpy(), g.cpu().numpy())
            ref = (er.cpu().numpy(), fr.cpu().numpy(), gr.cpu().numpy())
        for a_, b_ in zip(got, ref):
            assert np.array_equal(a_, b_), f"call {step}: not bitwise equal to ewald_energy_forces"
        want = oracle.energy_forces(pos, q, L, a, rc, K, oracle.FAST)
        compare((*got, 0), want, precision, f"noalloc call {step}")


def test_noalloc_rejects_what_does_not_fit():
    import torch
    from paper_1708_01135_amd import ewald as ew
    dev = torch.device("cuda:0")
    s = wl.make_config("rocksalt32", 0)
    n = len(s.q)
    tp = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    tq = torch.tensor(s.q, dtype=torch.float64, device=dev)
    e = torch.full((5,), 7.0, dtype=torch.float64, device=dev)
    with ew.Plan(n, s.box_L, s.alpha, s.r_c, s.k_max, "mixed", flags=ew.FLAG_NO_WORKSPACE) as plan:
        lib = ew.library()
        st = lib.ewald_energy_forces_noalloc(plan.handle, n, tp.data_ptr(), tq.data_ptr(), e.data_ptr(), None, None)
        assert st == ew.ERR_SCRATCH
        assert lib.ewald_energy_forces_noalloc(plan.handle, n + 1, tp.data_ptr(), tq.data_ptr(), e.data_ptr(),
                                               None, None) == ew.ERR_CAPACITY
        torch.cuda.synchronize()
    assert torch.all(e == 7.0).item()  # nothing was enqueued
