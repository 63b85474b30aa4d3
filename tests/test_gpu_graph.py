"""Graph replay of repeated evaluations.

A plan records its launch sequence into a HIP graph on the second evaluation
with the same n, buffers and kind (one of its last four keys), and launches
that graph afterwards.  Every
replay must equal, bit for bit, the kernel-by-kernel evaluation of the same
inputs by a plan made with EWALD_FLAG_NO_GRAPH.  The replays are interleaved
with other device work and host synchronisations, the inputs change in place
between replays (the graph reads the buffers, not captured values), and a
call with other buffers falls back to kernel-by-kernel launches.
"""
import numpy as np
import pytest

from paper_1708_01135_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _system(n, seed):
    L = 14.0
    pos, q = wl.random_neutral(n, L, seed)
    return pos, q, L, 0.8, 4.5, 10


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_replays_bitwise_equal_kernel_by_kernel(precision):
    import torch
    from paper_1708_01135_amd import ewald as ew
    dev = torch.device("cuda:0")
    pos_h, q_h, L, alpha, rc, K = _system(2500, 7)
    n = q_h.shape[0]
    pos = torch.tensor(pos_h, device=dev)
    q = torch.tensor(q_h, device=dev)
    g = ew.Plan(n, L, alpha, rc, K, precision)
    r = ew.Plan(n, L, alpha, rc, K, precision, flags=ew.FLAG_NO_GRAPH)
    out = (torch.empty(5, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64, device=dev),
           torch.empty(n, dtype=torch.float64, device=dev))
    rng = np.random.default_rng(3)
    for it in range(7):
        if it in (3, 5):  # new coordinates and charges in the same buffers
            pos += torch.tensor(rng.normal(0.0, 0.05, size=(n, 3)), device=dev)
            q.mul_(1.0 + 0.01 * it)
        e, f, d = g.energy_forces(pos, q, True, True, out=out)
        er, fr, dr = r.energy_forces(pos, q, True, True)
        # unrelated device work between evaluations
        x = torch.randn(4096, device=dev)
        _ = (x * x).sum().item()
        torch.cuda.synchronize()
        assert torch.equal(e, er), it
        assert torch.equal(f, fr), it
        assert torch.equal(d, dr), it
    assert g.status() == ew.OK and r.status() == ew.OK
    # other buffers: kernel by kernel again, same results
    out2 = tuple(torch.empty_like(t) for t in out)
    e2, f2, d2 = g.energy_forces(pos, q, True, True, out=out2)
    torch.cuda.synchronize()
    assert torch.equal(e2, er) and torch.equal(f2, fr) and torch.equal(d2, dr)


def test_energy_only_and_backward_replays():
    import torch
    from paper_1708_01135_amd import ewald as ew
    dev = torch.device("cuda:0")
    pos_h, q_h, L, alpha, rc, K = _system(1800, 9)
    n = q_h.shape[0]
    pos = torch.tensor(pos_h, device=dev)
    q = torch.tensor(q_h, device=dev)
    g = ew.Plan(n, L, alpha, rc, K, "mixed")
    r = ew.Plan(n, L, alpha, rc, K, "mixed", flags=ew.FLAG_NO_GRAPH)
    lib = ew.library()
    e = torch.empty(5, dtype=torch.float64, device=dev)
    er = torch.empty(5, dtype=torch.float64, device=dev)
    gs = torch.tensor([0.75], dtype=torch.float64, device=dev)
    gp = torch.empty((n, 3), dtype=torch.float64, device=dev)
    gq = torch.empty(n, dtype=torch.float64, device=dev)
    gpr = torch.empty_like(gp)
    gqr = torch.empty_like(gq)
    for it in range(5):
        stream = ew._stream_handle()
        assert lib.ewald_plan_set_stream(g.handle, stream) == ew.OK
        assert lib.ewald_plan_set_stream(r.handle, stream) == ew.OK
        assert lib.ewald_energy(g.handle, n, pos.data_ptr(), q.data_ptr(), e.data_ptr()) == ew.OK
        assert lib.ewald_energy(r.handle, n, pos.data_ptr(), q.data_ptr(), er.data_ptr()) == ew.OK
        torch.cuda.synchronize()
        assert torch.equal(e, er), it
        assert lib.ewald_energy_backward(g.handle, n, pos.data_ptr(), q.data_ptr(), gs.data_ptr(), e.data_ptr(),
                                         gp.data_ptr(), gq.data_ptr()) == ew.OK
        assert lib.ewald_energy_backward(r.handle, n, pos.data_ptr(), q.data_ptr(), gs.data_ptr(), er.data_ptr(),
                                         gpr.data_ptr(), gqr.data_ptr()) == ew.OK
        torch.cuda.synchronize()
        assert torch.equal(gp, gpr) and torch.equal(gq, gqr) and torch.equal(e, er), it
        gs.mul_(1.5)  # the upstream gradient changes in place
    assert g.status() == ew.OK


def test_two_plans_on_side_streams_replay():
    """Two plans on two non-default streams, evaluated alternately many times
    (graph replay on both), each equal to its kernel-by-kernel reference."""
    import torch
    from paper_1708_01135_amd import ewald as ew
    dev = torch.device("cuda:0")
    systems = [_system(1500, 21), _system(2200, 22)]
    streams = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]  # default priority
    plans, refs, bufs, outs = [], [], [], []
    for (pos_h, q_h, L, alpha, rc, K), st in zip(systems, streams):
        n = q_h.shape[0]
        pos = torch.tensor(pos_h, device=dev)
        q = torch.tensor(q_h, device=dev)
        r = ew.Plan(n, L, alpha, rc, K, "mixed", flags=ew.FLAG_NO_GRAPH)
        e, f, d = r.energy_forces(pos, q, True, True)
        torch.cuda.synchronize()
        refs.append((e.clone(), f.clone(), d.clone()))
        with torch.cuda.stream(st):
            plans.append(ew.Plan(n, L, alpha, rc, K, "mixed"))
        bufs.append((pos, q))
        outs.append((torch.empty(5, dtype=torch.float64, device=dev),
                     torch.empty((n, 3), dtype=torch.float64, device=dev),
                     torch.empty(n, dtype=torch.float64, device=dev)))
    torch.cuda.synchronize()
    for it in range(6):
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                plans[k].energy_forces(bufs[k][0], bufs[k][1], True, True, out=outs[k])
        if it % 2:
            torch.cuda.synchronize()
            for k in range(2):
                for a, b in zip(outs[k], refs[k]):
                    assert torch.equal(a, b), (it, k)
    torch.cuda.synchronize()
    for k in range(2):
        for a, b in zip(outs[k], refs[k]):
            assert torch.equal(a, b), k
        assert plans[k].status() == ew.OK
