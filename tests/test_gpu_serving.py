"""Request server: many independent systems of different N, L and K in flight
together on one GPU.

Every result served in a mix must equal, bit for bit, the result of a
stand-alone plan with the same parameters (the kernels use fixed-order
reductions, so neither the stream nor the neighbours in the mix may change a
bit), and the FP64 results must match the oracle.
"""
import time

import numpy as np
import pytest

import oracle
from paper_1708_01135_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _mix(n_systems, n_hi, seed):
    return wl.serving_mix(n_systems, seed=seed, n_lo=500, n_hi=n_hi)


def _to_dev(mix):
    import torch
    dev = torch.device("cuda:0")
    for it in mix:
        it["pos_d"] = torch.tensor(it["pos"], device=dev)
        it["q_d"] = torch.tensor(it["q"], device=dev)
    torch.cuda.synchronize()


def _standalone(it, precision):
    import torch
    from paper_1708_01135_amd import ewald as ew
    with ew.Plan(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"], precision) as p:
        e, f, g = p.energy_forces(it["pos_d"], it["q_d"], True, True)
        torch.cuda.synchronize()
        assert p.status() == ew.OK
        return e.cpu().numpy(), f.cpu().numpy(), g.cpu().numpy()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_mix_results_bitwise_equal_to_standalone(precision):
    from paper_1708_01135_amd import ewald as ew
    mix = _mix(10, 6000, seed=3)
    _to_dev(mix)
    ref = [_standalone(it, precision) for it in mix]
    with ew.Server(n_streams=4, precision=precision) as srv:
        ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
        tickets = []
        for rep in range(3):  # interleaved: every system three times, in a rotating order
            order = np.roll(np.arange(len(mix)), rep * 3)
            for s in order:
                tickets.append((s, srv.submit(ids[s], mix[s]["pos_d"], mix[s]["q_d"], True, True)))
        for s, t in tickets:
            (e, f, g), ts, td = srv.wait(t)
            assert td >= ts
            assert np.array_equal(e.cpu().numpy(), ref[s][0]), (s, "energy")
            assert np.array_equal(f.cpu().numpy(), ref[s][1]), (s, "forces")
            assert np.array_equal(g.cpu().numpy(), ref[s][2]), (s, "dEdq")
        st = srv.stats()
        assert st["submitted"] == st["completed"] == 30 and st["in_flight"] == 0
        for i in ids:
            assert srv.system_status(i) == ew.OK


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_express_requests_batched_bitwise_equal_to_standalone(precision):
    # a burst of small requests: those that wait together for the express
    # stream go out as batched launch sequences; every result must still equal
    # the stand-alone plan's bit for bit, with batching on or off
    from paper_1708_01135_amd import ewald as ew
    mix = _mix(24, 2500, seed=8)
    _to_dev(mix)
    ref = [_standalone(it, precision) for it in mix]
    for batching in (True, False):
        with ew.Server(n_streams=4, precision=precision, batching=batching) as srv:
            ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
            tickets = [(s, srv.submit(ids[s], mix[s]["pos_d"], mix[s]["q_d"], True, True))
                       for rep in range(2) for s in range(len(mix))]
            for s, t in tickets:
                (e, f, g), _, _ = srv.wait(t)
                assert np.array_equal(e.cpu().numpy(), ref[s][0]), (batching, s, "energy")
                assert np.array_equal(f.cpu().numpy(), ref[s][1]), (batching, s, "forces")
                assert np.array_equal(g.cpu().numpy(), ref[s][2]), (batching, s, "dEdq")
            st = srv.stats()
            print(f"batching={batching}: {st['batches']} batches carried {st['batched']} of "
                  f"{st['completed']} requests", flush=True)
            assert st["completed"] == 2 * len(mix) and st["in_flight"] == 0 and st["used"] == 0
            if batching:
                assert st["batches"] >= 1 and st["batched"] >= 2
            else:
                assert st["batches"] == 0
            for i in ids:
                assert srv.system_status(i) == ew.OK


@pytest.mark.timeout(600)
def test_served_fp64_matches_oracle():
    from paper_1708_01135_amd import ewald as ew
    mix = _mix(4, 3000, seed=5)
    _to_dev(mix)
    with ew.Server(n_streams=2, precision="fp64") as srv:
        ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
        tickets = [srv.submit(i, it["pos_d"], it["q_d"], True, True) for i, it in zip(ids, mix)]
        for it, t in zip(mix, tickets):
            (e, f, g), _, _ = srv.wait(t)
            en, fo, dq = oracle.energy_forces(it["pos"], it["q"], it["box_L"], it["alpha"], it["r_c"],
                                              it["k_max"], oracle.FAST)
            e, f, g = e.cpu().numpy(), f.cpu().numpy(), g.cpu().numpy()
            print(f"n={it['n']} K={it['k_max']} rel_E={abs(e[0] - en[0]) / abs(en[0]):.2e} "
                  f"rel_F={np.linalg.norm(f - fo) / np.linalg.norm(fo):.2e}", flush=True)
            assert abs(e[0] - en[0]) <= 1e-10 * abs(en[0])
            assert np.linalg.norm(f - fo) <= 1e-10 * np.linalg.norm(fo)
            assert np.linalg.norm(g - dq) <= 1e-10 * np.linalg.norm(dq)


def _ws_bytes(params, n):
    from paper_1708_01135_amd import ewald as ew
    with ew.Plan(params["n_max"], params["box_L"], params["alpha"], params["r_c"], params["k_max"], "mixed",
                 flags=ew.FLAG_NO_WORKSPACE) as p:
        return p.eval_workspace_bytes(n)


def test_admission_capacity_and_removal():
    import torch
    from paper_1708_01135_amd import ewald as ew
    a = dict(n_max=2000, box_L=13.57, alpha=0.711, r_c=4.5, k_max=14)
    b = dict(n_max=4000, box_L=17.1, alpha=0.711, r_c=4.5, k_max=18)
    big = dict(n_max=40000, box_L=36.8, alpha=0.711, r_c=4.5, k_max=38)
    wa, wb = _ws_bytes(a, 2000), _ws_bytes(b, 4000)
    assert 0 < wa < wb < _ws_bytes(big, 40000)
    with ew.Server(n_streams=2, precision="mixed", hbm_budget=wb + wa // 2) as srv:
        ia = srv.add_system(**a)
        ib = srv.add_system(**b)
        assert srv.stats()["used"] == 0 and srv.stats()["systems"] == 2
        with pytest.raises(ew.EwaldError) as ex:  # a request of n_max could never fit
            srv.add_system(**big)
        assert ex.value.status == ew.ERR_ADMISSION
        assert srv.stats()["systems"] == 2
        pos, q = wl.random_neutral(2001, a["box_L"], 1)
        pd = torch.tensor(pos, device="cuda:0")
        qd = torch.tensor(q, device="cuda:0")
        with pytest.raises(ew.EwaldError) as ex:
            srv.submit(ia, pd, qd)
        assert ex.value.status == ew.ERR_CAPACITY
        t = srv.submit(ia, pd[:1000].contiguous(), qd[:1000].contiguous())
        srv.wait(t)
        assert srv.stats()["used"] == 0 and srv.stats()["peak_used"] > 0
        srv.remove_system(ia)
        with pytest.raises(ew.EwaldError) as ex:
            srv.submit(ia, pd[:10].contiguous(), qd[:10].contiguous())
        assert ex.value.status == ew.ERR_INVALID_ARG
        assert srv.stats()["systems"] == 1 and ib != ia


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_request_held_until_memory_frees(precision):
    """Two systems whose requests each need most of the arena: the second
    request is held until the first one's buffers return, then runs; both
    results equal, bit for bit, those of stand-alone plans."""
    from paper_1708_01135_amd import ewald as ew
    mix = [wl.serving_mix(1, seed=40, n_lo=5000, n_hi=5001)[0], wl.serving_mix(1, seed=41, n_lo=5000, n_hi=5001)[0]]
    _to_dev(mix)
    ref = [_standalone(it, precision) for it in mix]
    ws = [_ws_bytes(dict(n_max=it["n"], box_L=it["box_L"], alpha=it["alpha"], r_c=it["r_c"], k_max=it["k_max"]),
                    it["n"]) for it in mix]
    budget = max(ws) + min(ws) // 2  # one request at a time
    with ew.Server(n_streams=2, precision=precision, hbm_budget=budget) as srv:
        ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
        tickets = [srv.submit(i, it["pos_d"], it["q_d"], True, True) for i, it in zip(ids, mix)]
        done = []
        for s, t in enumerate(tickets):
            (e, f, g), ts, td = srv.wait(t)
            done.append(td)
            assert np.array_equal(e.cpu().numpy(), ref[s][0]), (s, "energy")
            assert np.array_equal(f.cpu().numpy(), ref[s][1]), (s, "forces")
            assert np.array_equal(g.cpu().numpy(), ref[s][2]), (s, "dEdq")
        st = srv.stats()
        print(f"held {st['held_total']} peak {st['peak_used']} budget {st['budget']}", flush=True)
        assert st["held_total"] >= 1 and st["held"] == 0
        assert st["peak_used"] <= budget and st["used"] == 0


def test_nonfinite_request_is_isolated():
    import torch
    from paper_1708_01135_amd import ewald as ew
    mix = _mix(2, 2000, seed=8)
    _to_dev(mix)
    ref = _standalone(mix[1], "mixed")
    bad = mix[0]["pos_d"].clone()
    bad[7, 1] = float("nan")
    torch.cuda.synchronize()
    with ew.Server(n_streams=2, precision="mixed") as srv:
        i0 = srv.add_system(mix[0]["n"], mix[0]["box_L"], mix[0]["alpha"], mix[0]["r_c"], mix[0]["k_max"])
        i1 = srv.add_system(mix[1]["n"], mix[1]["box_L"], mix[1]["alpha"], mix[1]["r_c"], mix[1]["k_max"])
        t0 = srv.submit(i0, bad, mix[0]["q_d"])
        t1 = srv.submit(i1, mix[1]["pos_d"], mix[1]["q_d"], True, True)
        (e0, _, _), _, _ = srv.wait(t0)
        (e1, f1, g1), _, _ = srv.wait(t1)
        assert np.isnan(e0.cpu().numpy()[0])
        assert srv.system_status(i0) == ew.ERR_NONFINITE
        assert srv.system_status(i0) == ew.OK  # status cleared on read
        assert srv.system_status(i1) == ew.OK
        assert np.array_equal(e1.cpu().numpy(), ref[0]) and np.array_equal(f1.cpu().numpy(), ref[1])
        # the system serves again after the bad request
        t2 = srv.submit(i0, mix[0]["pos_d"], mix[0]["q_d"])
        (e2, _, _), _, _ = srv.wait(t2)
        assert np.isfinite(e2.cpu().numpy()[0])


@pytest.mark.timeout(600)
def test_poisson_arrivals_all_served():
    from paper_1708_01135_amd import ewald as ew
    mix = _mix(24, 8000, seed=11)
    _to_dev(mix)
    rng = np.random.default_rng(1000)
    with ew.Server(n_streams=4, precision="mixed") as srv:
        ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
        # warm-up pass, then 3 passes at Poisson arrivals of 2 kHz
        for i, it in zip(ids, mix):
            srv.wait(srv.submit(i, it["pos_d"], it["q_d"]))
        seq = np.concatenate([rng.permutation(len(mix)) for _ in range(3)])
        arrive = np.cumsum(rng.exponential(1.0 / 2000.0, size=seq.size))
        t0 = ew.Server.clock()
        tickets = []
        for s, ta in zip(seq, arrive):
            while ew.Server.clock() - t0 < ta:
                pass
            tickets.append((t0 + ta, srv.submit(ids[s], mix[s]["pos_d"], mix[s]["q_d"])))
        lat = []
        for ta, t in tickets:
            (e, _, _), ts, td = srv.wait(t)
            assert ts >= ta - 1e-6 and td >= ts
            assert np.isfinite(e.cpu().numpy()[0])
            lat.append(td - ta)
        lat = np.sort(np.array(lat)) * 1e3
        print(f"served {lat.size} requests: p50 {lat[lat.size // 2]:.3f} ms, "
              f"p99 {lat[int(np.ceil(0.99 * lat.size)) - 1]:.3f} ms, max {lat[-1]:.3f} ms", flush=True)
        assert srv.stats()["in_flight"] == 0


@pytest.mark.skip(reason="the CU-masked express lane (EWALD_SERVER_FLAG_EXPRESS_CUS) is opt-in: a sibling "
                         "configuration with four express CUs per XCD went silent on the GPU once, cause not "
                         "known, so the round-end suite does not run CU-masked streams")
def test_express_cus_results_bitwise_equal_to_standalone():
    from paper_1708_01135_amd import ewald as ew
    mix = _mix(6, 8000, seed=31)
    _to_dev(mix)
    ref = [_standalone(it, "mixed") for it in mix]
    with ew.Server(n_streams=4, precision="mixed", express_cus=True) as srv:
        ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
        tickets = [(s, srv.submit(ids[s], mix[s]["pos_d"], mix[s]["q_d"], True, True)) for s in range(len(mix))]
        for s, t in tickets:
            (e, f, g), _, _ = srv.wait(t)
            assert np.array_equal(e.cpu().numpy(), ref[s][0]) and np.array_equal(f.cpu().numpy(), ref[s][1])
