"""Benchmark: Ewald energy + forces throughput on one MI355X.

Headline workload: rock-salt lattice of 32^3 sites (N = 32768, L = 32, spacing
1, charges +-1, jitter U(-0.1, 0.1)), alpha = 0.7, r_c = 4.5, k_max = 20 -- the
32^3 NaCl crystal of the paper's strong-scaling study (section 4.2) in reduced
units.  One step = one complete ewald_energy_forces call (binning, cell list,
real-space pairs, phase tables, structure factor, reduction, force gather,
totals) with inputs resident in HBM.

Prints one JSON line: the mixed-precision throughput as ``value`` (particle
evaluations per second), the plain-FP64 throughput beside it, p50/p99 latency,
errors of both paths against the FP64 CPU oracle, the roofline of the dominant
kernel (per-kernel HIP-event timing on the streams the kernels run on) and the
oracle's own throughput on this host.  Beside the headline:

* ``configs``: the 8^3 lattice (latency), the 64^3 lattice and the 10^6-ion
  electrolyte (throughput, p50/p99 latency, per-kernel times and rooflines,
  errors against the oracle's stored values on 4096 sampled particles);
* ``rooflines_all``: for every kernel class of the reciprocal space and for the
  real-space chain, the algorithmic rate (direct-evaluation flop counts) and,
  for the matrix-core kernels, the rate of the matrix instructions they
  actually execute, each against its pipe's peak;
* ``cpu_baselines``: the FP64 oracle on this host's cores at every config
  (median of 3 runs where that stays short, one run for the 10^6-ion system)
  and single-threaded at the two smallest, with the CPU model;
* ``batch``: 64 small systems (500-5000 ions) evaluated one by one and in
  one batched launch sequence (ewald_energy_forces_batch);
* ``serving``: the request server on a mix of 256 independent electrolyte
  systems (N = 500 ... 50000, K = 9 ... 41): its saturation throughput with
  small requests batched and one by one (and of the systems below 5,000 ions
  alone), and p50/p99 latency under Poisson arrivals.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Ewald E+F particle-evals/s, mixed vs FP64 at 1e-6 rel force err; p99 latency"
WORKLOAD = "rocksalt32"

# Algorithmic flops per unit, counted for a direct evaluation: structure factor
# 10 per (particle, k in the half space): complex phase product 6 and
# charge-weighted complex accumulate 4; force gather 20 per (particle, k):
# phase 6, Re/Im of exp(i k.r) conj(G) 6, force accumulate 6, potential 2; the
# real-space pair loop 30 per ordered pair inside the cutoff (plus three special
# functions): displacement 3, |d|^2 5, |d| 1, sqrt(alpha)|d| 1, alpha|d|^2 1,
# erfc combination 3, q q/r 2, energy 2, force scalar 5, force accumulate 6.
FLOPS_PER_UNIT = {"sk": 10.0, "gather": 20.0, "realspace": 30.0}
# Peaks (MI355X, dense): FP64 matrix cores 78.6 TFLOP/s, FP32 matrix cores
# 157.3; vector ALU 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz =
# 78.6 TFLOP/s for FP64 and for unpacked FP32 (packed dual-FP32 issue is
# compiled out; the published 157.3 FP32 vector figure counts it).
PEAK_VALU = 78.6
PEAK_MFMA = {"fp64": 78.6, "fp32": 157.3}
# The real-space chain is the neighbour-list build followed by the pair loop.
REALSPACE = ("pair_list", "pair")


def kernel_bound(kernel, precision, stats):
    """(bound, peak TFLOP/s) of a hot kernel in the plan that ran."""
    if kernel == "sk":
        return ("mfma", PEAK_MFMA["fp64"]) if stats.get("sk_matrix_cores") else ("alu", PEAK_VALU)
    if kernel == "gather":
        if stats.get("gather_matrix_cores"):
            return "mfma", PEAK_MFMA["fp32" if precision == "mixed" else "fp64"]
        return "alu", PEAK_VALU
    return "alu", PEAK_VALU


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-calls", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-large", action="store_true",
                    help="skip the oracle timings of the 64^3 lattice and the 10^6-ion electrolyte")
    ap.add_argument("--no-configs", action="store_true", help="headline workload only")
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-server measurement")
    ap.add_argument("--no-graph", action="store_true",
                    help="plans launch kernel by kernel (no graph replay of repeated evaluations)")
    ap.add_argument("--serving-systems", type=int, default=256)
    ap.add_argument("--serving-passes", type=int, default=3)
    ap.add_argument("--serving-express-cus", action="store_true",
                    help="request server whose express stream has compute units of its own")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    return ap.parse_args()


# Kernel-source files whose hash is stored with the counter-based traffic figures;
# a changed source invalidates them.
KERNEL_SOURCES = {"gather": "paper_1708_01135_amd/csrc/k_gather_mfma.hip",
                  "sk": "paper_1708_01135_amd/csrc/k_sk_mfma.hip", "pair": "paper_1708_01135_amd/csrc/k_pair.hip",
                  "pair_list": "paper_1708_01135_amd/csrc/k_pair.hip"}


def source_hash(kernel):
    with open(os.path.join(ROOT, KERNEL_SOURCES[kernel]), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_bytes(kernel, workload, precision):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, calibrated against a plain copy), or None when absent or taken
    on a different kernel source.  The real-space chain sums its two kernels."""
    if kernel == "realspace":
        parts = [traffic_bytes(k, workload, precision) for k in REALSPACE]
        return None if any(p is None for p in parts) else sum(parts)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    for e in tab.get("entries", []):
        if (e["kernel"], e["workload"], e["precision"]) == (kernel, workload, precision):
            if e.get("source_sha256_16") != source_hash(kernel):
                return None
            return (e["fetch_kib"] * tab["fetch_factor"] + e["write_kib"] * tab["write_factor"]) * 1024.0
    return None


def issue_busy(kernel, workload, precision):
    """(VALU busy, matrix busy) fractions of SIMD-cycles from the committed
    counter summary, or None when absent or taken on a different kernel source.
    The real-space chain weights its two kernels by their durations."""
    path = os.path.join(ROOT, "profiles", "issue.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    names = REALSPACE if kernel == "realspace" else (kernel,)
    got = []
    for name in names:
        hit = [e for e in tab.get("entries", [])
               if (e["kernel"], e["workload"], e["precision"]) == (name, workload, precision)]
        if not hit or hit[0].get("source_sha256_16") != source_hash(name):
            return None
        got.append(hit[0])
    w = sum(e["duration_us"] for e in got)
    return {"valu_busy": sum(e["valu_busy"] * e["duration_us"] for e in got) / w,
            "matrix_busy": sum(e["matrix_busy"] * e["duration_us"] for e in got) / w,
            "source": "profiles/issue.json (kernel alone, rocprofv3 counters)"}


def calib_copy(mib):
    import torch
    n = mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": n * 4}), flush=True)


def time_steps(plan, pos, q, out, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.energy_forces(pos, q, True, False, out=out)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(s)
    for _ in range(steps):
        plan.energy_forces(pos, q, True, False, out=out)
    t1.record(s)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def kernel_profile(plan, pos, q, out, steps):
    """Average duration of every kernel class: HIP events around each launch on
    the stream it is launched on (the reciprocal kernels run on the plan's
    second stream, concurrently with the real-space ones)."""
    import torch
    plan.profile_reset()
    plan.profile(True)
    for _ in range(steps):
        plan.energy_forces(pos, q, True, False, out=out)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    return {k: {"avg_ms": (v[0] / v[1]) if v[1] else 0.0, "launches": v[1]} for k, v in prof.items()}


def pct(sorted_ms, p):
    return sorted_ms[min(len(sorted_ms) - 1, max(0, int(math.ceil(p * len(sorted_ms))) - 1))]


def latencies(plan, pos, q, out, calls):
    """Synchronised single calls (host wall time), after three warm-up calls."""
    import torch
    for _ in range(3):
        plan.energy_forces(pos, q, True, False, out=out)
    torch.cuda.synchronize()
    lat = []
    for _ in range(calls):
        t = time.perf_counter()
        plan.energy_forces(pos, q, True, False, out=out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    lat.sort()
    return {"p50_ms": pct(lat, 0.5), "p99_ms": pct(lat, 0.99), "calls": calls}


def rooflines(n, nk, prec, kern, stats, workload):
    """Per kernel class: algorithmic rate (direct-evaluation flops per launch /
    average duration) and, for matrix-core kernels, the rate of the matrix
    instructions executed, each against its pipe's peak."""
    out = {}
    units = {"sk": n * nk, "gather": n * nk, "realspace": stats["listed_pairs"]}
    for k in ("sk", "gather", "realspace"):
        if k == "realspace":
            if not all(kern.get(c, {}).get("launches") for c in REALSPACE):
                continue
            ms = sum(kern[c]["avg_ms"] for c in REALSPACE)
        else:
            if not kern.get(k, {}).get("launches"):
                continue
            ms = kern[k]["avg_ms"]
        flops = FLOPS_PER_UNIT[k] * units[k]
        ach = flops / (ms * 1e-3) / 1e12
        bound, peak = kernel_bound(k, prec, stats)
        r = {"bound": bound, "kernel": k if k != "realspace" else "pair_list+pair", "achieved": ach, "peak": peak,
             "unit": "TFLOP/s", "frac": ach / peak, "traffic": traffic_bytes(k, workload, prec), "avg_ms": ms,
             "algorithmic_flops_per_launch": flops, "issue": issue_busy(k, workload, prec)}
        exe = {"sk": stats.get("sk_mfma_flops", 0), "gather": stats.get("gather_mfma_flops", 0)}.get(k, 0)
        if exe:
            r["executed_flops_per_launch"] = exe
            r["executed_tflops"] = exe / (ms * 1e-3) / 1e12
            r["executed_frac"] = r["executed_tflops"] / peak
        out[k] = r
    return out


def golden(name):
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{name}_s0.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def measure(sysm, prec, steps, warmup, latency_calls, no_graph, want_forces=False):
    """Throughput, latency, per-kernel profile and branch statistics of one
    workload in one precision, on a plan sized to its N."""
    import torch
    from paper_1708_01135_amd import ewald
    n = sysm.n
    dev = torch.device("cuda:0")
    pos = torch.tensor(sysm.pos, dtype=torch.float64, device=dev)
    q = torch.tensor(sysm.q, dtype=torch.float64, device=dev)
    with ewald.Plan(n, sysm.box_L, sysm.alpha, sysm.r_c, sysm.k_max, prec,
                    flags=ewald.FLAG_NO_GRAPH if no_graph else 0) as plan:
        out = (torch.empty(5, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64, device=dev),
               torch.empty(n, dtype=torch.float64, device=dev))
        e, f, g = plan.energy_forces(pos, q, True, True)
        torch.cuda.synchronize()
        assert plan.status() == ewald.OK
        stats = plan.debug_stats(n)
        res = dict(energy=e.cpu().numpy(), stats=stats)
        if want_forces:
            res["forces"], res["dEdq"] = f.cpu().numpy(), g.cpu().numpy()
        # latency and per-kernel timings first: the throughput window below then
        # starts on a GPU that is already at its working clocks
        res["latency"] = latencies(plan, pos, q, out, latency_calls)
        res["kernels"] = kernel_profile(plan, pos, q, out, max(10, min(steps, 100)))
        ms = time_steps(plan, pos, q, out, steps, warmup)
        res["ms"], res["pe_s"] = ms, n / (ms * 1e-3)
    return res


def errors_vs(ref_e, ref_f, got_e, got_f, idx=None):
    import numpy as np
    ff = got_f if idx is None else got_f[idx]
    return {"rel_E": abs(got_e[0] - ref_e[0]) / abs(ref_e[0]),
            "rel_F": float(np.linalg.norm(ff - ref_f) / np.linalg.norm(ref_f))}


def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def time_oracle(sysm, runs, threads=None):
    """Wall times of `runs` full FP64 oracle evaluations (energy, forces,
    dE/dq); returns (median seconds, threads used, last result)."""
    import oracle
    prev = oracle.num_threads()
    if threads:
        oracle.set_num_threads(threads)
    try:
        used = oracle.num_threads()
        ts, ref = [], None
        for _ in range(runs):
            t = time.perf_counter()
            ref = oracle.energy_forces(sysm.pos, sysm.q, sysm.box_L, sysm.alpha, sysm.r_c, sysm.k_max, oracle.FAST)
            ts.append(time.perf_counter() - t)
    finally:
        oracle.set_num_threads(prev)
    ts.sort()
    return ts[len(ts) // 2], used, ref


def cpu_line(sysm, sec, threads, runs):
    return {"value": sysm.n / sec, "unit": "particle-evals/s", "cores": threads, "kind": "oracle",
            "seconds": sec, "sample": f"median of {runs} full FP64 oracle evaluation(s) of the {sysm.n}-ion "
                                     f"{sysm.name} workload" if runs > 1 else
            f"one full FP64 oracle evaluation of the {sysm.n}-ion {sysm.name} workload"}


def batched(n_systems=64):
    """Many small systems (electrolytes of 500-5000 ions from the serving mix's
    recipe) evaluated one by one through their plans against one
    ewald_energy_forces_batch call: median wall time of 10 repetitions each."""
    import torch

    from paper_1708_01135_amd import ewald, workloads
    mix = workloads.serving_mix(n_systems, seed=21, n_lo=500, n_hi=5000)
    dev = torch.device("cuda:0")
    res = {"systems": n_systems, "n_total": int(sum(it["n"] for it in mix)),
           "n_range": [min(it["n"] for it in mix), max(it["n"] for it in mix)]}
    for prec in ("mixed", "fp64"):
        plans = [ewald.Plan(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"], prec) for it in mix]
        items = [(p, torch.tensor(it["pos"], device=dev), torch.tensor(it["q"], device=dev),
                  (torch.empty(5, dtype=torch.float64, device=dev),
                   torch.empty((it["n"], 3), dtype=torch.float64, device=dev), None)) for p, it in zip(plans, mix)]

        def one_by_one():
            for p, a, b, o in items:
                p.energy_forces(a, b, True, False, out=o)

        def together():
            ewald.energy_forces_batch(items)

        out = {}
        for name, fn in (("one_by_one_ms", one_by_one), ("batched_ms", together)):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(10):
                t = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            out[name] = sorted(ts)[len(ts) // 2] * 1e3
        out["batched_systems_per_s"] = n_systems / (out["batched_ms"] * 1e-3)
        out["speedup"] = out["one_by_one_ms"] / out["batched_ms"]
        res[prec] = out
        for p in plans:
            p.release()
    return res


def serving(n_systems, passes, express_cus=False):
    """Request server on independent electrolyte systems (density 0.8, r_c = 4.5,
    alpha r_c^2 = 14.4, K matched to the real-space exponent): saturation throughput
    with every request submitted at once, then Poisson arrivals at fractions of it.
    Latency = completion observed by the server minus the scheduled arrival."""
    import numpy as np
    import torch

    from paper_1708_01135_amd import ewald, workloads
    t_gen = time.perf_counter()
    mix = workloads.serving_mix(n_systems, seed=0, workers=min(16, os.cpu_count() or 1))
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    pos = [torch.tensor(it["pos"], device=dev) for it in mix]
    q = [torch.tensor(it["q"], device=dev) for it in mix]
    outs = [(torch.empty(5, dtype=torch.float64, device=dev), torch.empty((it["n"], 3), dtype=torch.float64, device=dev),
             None) for it in mix]
    torch.cuda.synchronize()
    ns = np.array([it["n"] for it in mix])
    units = float(sum(it["n"] * ewald.kset_size(it["k_max"]) for it in mix))
    res = {"systems": n_systems, "n_total": int(ns.sum()), "n_range": [int(ns.min()), int(ns.max())],
           "k_range": [min(it["k_max"] for it in mix), max(it["k_max"] for it in mix)], "precision": "mixed",
           "generate_s": round(t_gen, 1)}

    def saturate(srv, ids, sel):
        t0 = time.perf_counter()
        tick = [srv.submit(ids[s], pos[s], q[s], out=outs[s]) for s in sel]
        for t in tick:
            srv.wait(t)
        return time.perf_counter() - t0

    def run(srv, ids, sel=range(n_systems)):
        saturate(srv, ids, sel)  # warm-up
        return min(saturate(srv, ids, sel) for _ in range(3))

    small = [s for s in range(n_systems) if mix[s]["n"] < 5000]
    with ewald.Server(n_streams=1, precision="mixed") as srv:
        ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
        t1 = run(srv, ids)
    # express requests one by one instead of batched: the whole mix, and its
    # systems below 5,000 ions alone
    with ewald.Server(n_streams=4, precision="mixed", express_cus=express_cus, batching=False) as srv:
        ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
        t4_nb = run(srv, ids)
        t_small_nb = run(srv, ids, small)
    with ewald.Server(n_streams=4, precision="mixed", express_cus=express_cus) as srv:
        t_add = time.perf_counter()
        ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
        t_add = time.perf_counter() - t_add
        res["register_s"] = round(t_add, 2)
        t4 = run(srv, ids)
        t_small = run(srv, ids, small)
        st = srv.stats()
        res["arena_gb"] = round(st["budget"] / 1e9, 2)
        res["arena_peak_gb"] = round(st["peak_used"] / 1e9, 2)
        res["requests_held_for_memory"] = st["held_total"]
        sat = n_systems / t4
        res["masked_streams"] = st["masked_streams"]
        res["express_cus"] = bool(express_cus)
        res["saturation"] = {"streams_4": {"systems_per_s": sat, "particle_evals_per_s": ns.sum() / t4,
                                           "tflops_alg": 30.0 * units / t4 / 1e12},
                             "streams_4_unbatched": {"systems_per_s": n_systems / t4_nb,
                                                     "particle_evals_per_s": ns.sum() / t4_nb},
                             "streams_1": {"systems_per_s": n_systems / t1, "particle_evals_per_s": ns.sum() / t1},
                             "below_5000": {"systems": len(small), "systems_per_s": len(small) / t_small,
                                            "unbatched_systems_per_s": len(small) / t_small_nb}}
        res["batched_launches"] = st["batches"]
        res["batched_requests"] = st["batched"]
        res["requests_served"] = st["completed"]
        # stand-alone latency of every system: one request at a time
        alone = np.zeros(n_systems)
        for s in range(n_systems):
            ts = []
            for _ in range(3):
                t = time.perf_counter()
                srv.wait(srv.submit(ids[s], pos[s], q[s], out=outs[s]))
                ts.append(time.perf_counter() - t)
            alone[s] = sorted(ts)[1] * 1e3
        buckets = [(500, 2000), (2000, 5000), (5000, 20000), (20000, 50001)]
        res["buckets"] = [f"{lo}-{hi - 1 if hi == 50001 else hi}" for lo, hi in buckets]
        res["alone_p50_ms"] = {}
        for (lo, hi), name in zip(buckets, res["buckets"]):
            sel = np.sort(alone[(ns >= lo) & (ns < hi)])
            if sel.size:
                res["alone_p50_ms"][name] = float(sel[sel.size // 2])
        rng = np.random.default_rng(1000)
        res["poisson"] = []
        for frac in (0.25, 0.5, 0.7, 0.9):
            rate = frac * sat
            seq = np.concatenate([rng.permutation(n_systems) for _ in range(passes)])
            arrive = np.cumsum(rng.exponential(1.0 / rate, size=seq.size))
            t0 = ewald.Server.clock()
            tick = []
            for s, ta in zip(seq, arrive):
                while ewald.Server.clock() - t0 < ta:
                    pass
                tick.append((t0 + ta, srv.submit(ids[s], pos[s], q[s], out=outs[s])))
            lat = []
            t_end = t0
            for ta, t in tick:
                _, _, td = srv.wait(t)
                lat.append((td - ta) * 1e3)
                t_end = max(t_end, td)
            lat_arr = np.array(lat)
            ratio = lat_arr / alone[seq]
            per_bucket = {}
            for (lo, hi), name in zip(buckets, res["buckets"]):
                m = (ns[seq] >= lo) & (ns[seq] < hi)
                if m.any():
                    lb, rb = sorted(lat_arr[m]), sorted(ratio[m])
                    per_bucket[name] = {"requests": int(m.sum()), "p50_ms": pct(lb, 0.5), "p99_ms": pct(lb, 0.99),
                                        "p99_over_alone": pct(rb, 0.99)}
            lat.sort()
            res["poisson"].append({"load": frac, "rate_per_s": rate, "requests": int(seq.size),
                                   "p50_ms": pct(lat, 0.5), "p99_ms": pct(lat, 0.99), "max_ms": lat[-1],
                                   "achieved_per_s": seq.size / (t_end - t0), "by_size": per_bucket})
            print(f"serving load {frac}: p50 {pct(lat, 0.5):.3f} ms p99 {pct(lat, 0.99):.3f} ms", file=sys.stderr,
                  flush=True)
        for i in ids:
            assert srv.system_status(i) == ewald.OK
    return res


def describe(sysm, nk):
    shape = f"rock-salt {round(sysm.n ** (1 / 3))}^3" if sysm.name.startswith("rocksalt") else "random electrolyte"
    return (f"{sysm.name}: {shape} N={sysm.n} L={sysm.box_L:g} alpha={sysm.alpha} r_c={sysm.r_c} "
            f"k_max={sysm.k_max} |K+|={nk}")


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.calib_copy_mib:
        calib_copy(args.calib_copy_mib)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library evaluates on exactly one GPU (--gpus 1); it has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np

    from paper_1708_01135_amd import ewald, workloads

    t_start = time.perf_counter()
    sysm = workloads.make_config(args.workload, 0)
    n = sysm.n
    nk = ewald.kset_size(sysm.k_max)
    precisions = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    results = {}
    for prec in precisions:
        log(f"{args.workload} {prec}")
        results[prec] = measure(sysm, prec, args.steps, args.warmup, args.latency_calls, args.no_graph,
                                want_forces=True)

    # errors against the FP64 CPU oracle, and the oracle's own rate on this host
    cpu, cpus, errs = None, {}, {}
    if not args.no_cpu_baseline:
        log("oracle on the headline workload")
        sec, used, ref = time_oracle(sysm, 3)
        cpu = cpu_line(sysm, sec, used, 3)
        cpus[sysm.name] = cpu
        for prec, r in results.items():
            errs[prec] = errors_vs(ref[0], ref[1], r["energy"], r["forces"])

    head_prec = "mixed" if "mixed" in results else "fp64"
    head = results[head_prec]
    per_kernel_roofline = {p: rooflines(n, nk, p, r["kernels"], r["stats"], args.workload)
                           for p, r in results.items()}
    roofs = per_kernel_roofline[head_prec]
    dom = max(roofs, key=lambda k: roofs[k]["avg_ms"]) if roofs else None
    roof = roofs.get(dom)

    configs = {}
    if not args.no_configs:
        for name, steps, calls in (("rocksalt8", 200, 300), ("rocksalt64", 20, 200), ("electrolyte1m", 8, 50)):
            if name == args.workload:
                continue
            t = time.perf_counter()
            s = workloads.make_config(name, 0)
            log(f"{name}: generated in {time.perf_counter() - t:.1f} s")
            snk = ewald.kset_size(s.k_max)
            g = golden(name)
            ref = None
            if name == "rocksalt8":
                import oracle
                ref = oracle.energy_forces(s.pos, s.q, s.box_L, s.alpha, s.r_c, s.k_max, oracle.FAST)
            line = {"workload": describe(s, snk), "n": s.n}
            for prec in (["fp64", "mixed"] if args.precision == "both" else [args.precision]):
                log(f"{name} {prec}")
                r = measure(s, prec, steps, 3, calls, args.no_graph, want_forces=True)
                entry = {"value": r["pe_s"], "unit": "particle-evals/s", "ms_per_step": r["ms"], "steps": steps,
                         "latency": r["latency"],
                         "kernels_ms": {k: round(v["avg_ms"], 5) for k, v in r["kernels"].items()},
                         "rooflines": rooflines(s.n, snk, prec, r["kernels"], r["stats"], name),
                         "pairs": r["stats"]["listed_pairs"], "direct_particles": r["stats"]["direct_particles"]}
                if ref is not None:
                    entry["errors_vs_oracle"] = errors_vs(ref[0], ref[1], r["energy"], r["forces"])
                elif g is not None:
                    idx = np.asarray(g["targets"])
                    entry["errors_vs_oracle"] = dict(errors_vs(g["energy"], np.asarray(g["forces"]), r["energy"],
                                                               r["forces"], idx),
                                                     sample=f"{idx.size} particles stratified over the box")
                line[prec] = entry
            if "mixed" in line and "fp64" in line:
                line["mixed_over_fp64"] = line["mixed"]["value"] / line["fp64"]["value"]
            if not args.no_cpu_baseline and (name == "rocksalt8" or not args.no_cpu_large):
                runs = 1 if name == "electrolyte1m" else 3
                log(f"oracle on {name} ({runs} run(s))")
                sec, used, _ = time_oracle(s, runs)
                cpus[name] = cpu_line(s, sec, used, runs)
            configs[name] = line
            del s
        if not args.no_cpu_baseline:
            # single-threaded oracle at the two smallest configs
            for name in ("rocksalt8", args.workload):
                s = workloads.make_config(name, 0)
                runs = 3 if s.n <= 4096 else 1
                log(f"single-thread oracle on {name}")
                sec, used, _ = time_oracle(s, runs, threads=1)
                cpus[f"{name}_1thread"] = cpu_line(s, sec, used, runs)

    serve = batch = None
    if not args.no_serving:
        log("batched small systems")
        batch = batched()
        log("serving mix")
        serve = serving(args.serving_systems, args.serving_passes, args.serving_express_cus)
    line = {
        "metric": METRIC,
        "value": head["pe_s"],
        "unit": "particle-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": describe(sysm, nk), "n": n, "precision": head_prec},
        "latency": head["latency"],
        "fp64": None if "fp64" not in results else {
            "value": results["fp64"]["pe_s"], "ms_per_step": results["fp64"]["ms"],
            "latency": results["fp64"]["latency"]},
        "mixed_over_fp64": (results["mixed"]["pe_s"] / results["fp64"]["pe_s"]) if len(results) == 2 else None,
        "errors_vs_oracle": errs or None,
        "kernels_ms": {p: {k: round(v["avg_ms"], 5) for k, v in r["kernels"].items()} for p, r in results.items()},
        "roofline": roof,
        "rooflines_all": per_kernel_roofline,
        "cpu_baseline": cpu,
        "cpu_baselines": cpus or None,
        "host": host_info(),
        "configs": configs or None,
        "batch": batch,
        "serving": serve,
        "bench_seconds": round(time.perf_counter() - t_start, 1),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
