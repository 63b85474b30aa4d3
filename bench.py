"""Benchmark: Ewald energy + forces throughput on one MI355X.

Workload: rock-salt lattice of 32^3 sites (N = 32768, L = 32, spacing 1,
charges +-1, jitter U(-0.1, 0.1)), alpha = 0.7, r_c = 4.5, k_max = 20 -- the
32^3 NaCl crystal of the paper's strong-scaling study (section 4.2) in reduced
units.  One step = one complete ewald_energy_forces call (binning, cell list,
real-space pairs, phase tables, structure factor, reduction, force gather,
totals) with inputs resident in HBM.

Prints one JSON line: the mixed-precision throughput as ``value`` (particle
evaluations per second), the plain-FP64 throughput beside it, p50/p99 latency,
errors of both paths against the FP64 CPU oracle, the roofline of the dominant
kernel (per-kernel HIP-event timing on the plan's stream), the oracle's own
throughput on this host and, under ``serving``, the request server on a mix of
256 independent electrolyte systems (N = 500 ... 50000, K = 9 ... 41): its
saturation throughput and p50/p99 latency under Poisson arrivals.
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

# Algorithmic flops per unit (one particle x one k vector of the half space),
# counted for a direct evaluation: structure factor 10 (complex phase product 6,
# charge-weighted complex accumulate 4); force gather 20 (phase 6, Re/Im of
# exp(i k.r) conj(G) 6, force accumulate 6, potential 2).  Real space: 30 per
# ordered pair inside the cutoff (plus three special functions).
FLOPS_PER_UNIT = {"sk": 10.0, "gather": 20.0}
# Peaks (MI355X, dense): the structure factor runs FP64 matrix-core products
# (78.6 TFLOP/s) in both precisions; the force gather runs FP32 (157.3) or FP64
# (78.6) matrix-core products.  VALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA)
# x 2.4 GHz = 78.6 TFLOP/s for FP64 and for unpacked FP32 (packed dual-FP32 issue
# is compiled out; the published 157.3 FP32 vector figure counts it).
PEAK_TFLOPS = 78.6
PEAK_FP32_PUBLISHED = 157.3
PEAK_MFMA = {"fp64": 78.6, "fp32": 157.3}


def kernel_bound(kernel, precision):
    """(bound, peak TFLOP/s) of a hot kernel in the default (matrix-core) plan."""
    if kernel == "sk":
        return "mfma", PEAK_MFMA["fp64"]
    if kernel == "gather":
        return "mfma", PEAK_MFMA["fp32" if precision == "mixed" else "fp64"]
    return "alu", PEAK_TFLOPS


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-calls", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-server measurement")
    ap.add_argument("--no-graph", action="store_true",
                    help="plans launch kernel by kernel (no graph replay of repeated evaluations)")
    ap.add_argument("--serving-systems", type=int, default=256)
    ap.add_argument("--serving-passes", type=int, default=3)
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
    on a different kernel source."""
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
    import torch
    plan.profile_reset()
    plan.profile(True)
    for _ in range(steps):
        plan.energy_forces(pos, q, True, False, out=out)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    return {k: {"avg_ms": (v[0] / v[1]) if v[1] else 0.0, "launches": v[1]} for k, v in prof.items()}


def latencies(plan, pos, q, out, calls):
    import torch
    lat = []
    for _ in range(calls):
        t = time.perf_counter()
        plan.energy_forces(pos, q, True, False, out=out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    lat.sort()
    return {"p50_ms": lat[len(lat) // 2], "p99_ms": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)],
            "calls": calls}


def pct(sorted_ms, p):
    return sorted_ms[min(len(sorted_ms) - 1, max(0, int(math.ceil(p * len(sorted_ms))) - 1))]


def serving(n_systems, passes):
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

    def saturate(srv, ids):
        t0 = time.perf_counter()
        tick = [srv.submit(ids[s], pos[s], q[s], out=outs[s]) for s in range(n_systems)]
        for t in tick:
            srv.wait(t)
        return time.perf_counter() - t0

    def run(srv, ids):
        saturate(srv, ids)  # warm-up
        return min(saturate(srv, ids) for _ in range(3))

    with ewald.Server(n_streams=1, precision="mixed") as srv:
        ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
        t1 = run(srv, ids)
    with ewald.Server(n_streams=4, precision="mixed") as srv:
        t_add = time.perf_counter()
        ids = [srv.add_system(it["n"], it["box_L"], it["alpha"], it["r_c"], it["k_max"]) for it in mix]
        t_add = time.perf_counter() - t_add
        res["workspace_gb"] = round(srv.stats()["used"] / 1e9, 2)
        res["register_s"] = round(t_add, 2)
        t4 = run(srv, ids)
        sat = n_systems / t4
        res["saturation"] = {"streams_4": {"systems_per_s": sat, "particle_evals_per_s": ns.sum() / t4,
                                           "tflops_alg": 30.0 * units / t4 / 1e12},
                             "streams_1": {"systems_per_s": n_systems / t1, "particle_evals_per_s": ns.sum() / t1}}
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
            lat.sort()
            res["poisson"].append({"load": frac, "rate_per_s": rate, "requests": int(seq.size),
                                   "p50_ms": pct(lat, 0.5), "p99_ms": pct(lat, 0.99), "max_ms": lat[-1],
                                   "achieved_per_s": seq.size / (t_end - t0)})
            print(f"serving load {frac}: p50 {pct(lat, 0.5):.3f} ms p99 {pct(lat, 0.99):.3f} ms", file=sys.stderr,
                  flush=True)
        for i in ids:
            assert srv.system_status(i) == ewald.OK
    return res


def main():
    args = parse()
    if args.calib_copy_mib:
        calib_copy(args.calib_copy_mib)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on exactly one GPU (--gpus 1); multi-GPU sharding is "
              "described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1708_01135_amd import ewald, workloads

    sysm = workloads.make_config(args.workload, 0)
    n = sysm.n
    dev = torch.device("cuda:0")
    pos = torch.tensor(sysm.pos, dtype=torch.float64, device=dev)
    q = torch.tensor(sysm.q, dtype=torch.float64, device=dev)
    nk = ewald.kset_size(sysm.k_max)
    results = {}
    precisions = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    for prec in precisions:
        plan = ewald.Plan(n, sysm.box_L, sysm.alpha, sysm.r_c, sysm.k_max, prec,
                          flags=ewald.FLAG_NO_GRAPH if args.no_graph else 0)
        out = (torch.empty(5, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64, device=dev),
               torch.empty(n, dtype=torch.float64, device=dev))
        ms = time_steps(plan, pos, q, out, args.steps, args.warmup)
        e, f, _ = plan.energy_forces(pos, q, True, True)
        torch.cuda.synchronize()
        assert plan.status() == ewald.OK
        kp = kernel_profile(plan, pos, q, out, args.steps)
        lat = latencies(plan, pos, q, out, args.latency_calls)
        results[prec] = dict(ms=ms, pe_s=n / (ms * 1e-3), energy=e.cpu().numpy(), forces=f.cpu().numpy(),
                             kernels=kp, latency=lat)
        plan.release()

    # errors against the FP64 CPU oracle, and the oracle's own rate on this host
    cpu = None
    errs = {}
    if not args.no_cpu_baseline:
        import oracle
        reps, t_tot, ref = 0, 0.0, None
        while reps < 3 or (t_tot < 10.0 and reps < 20):
            t = time.perf_counter()
            ref = oracle.energy_forces(sysm.pos, sysm.q, sysm.box_L, sysm.alpha, sysm.r_c, sysm.k_max, oracle.FAST)
            t_tot += time.perf_counter() - t
            reps += 1
        t_one = t_tot / reps
        cpu = {"value": n / t_one, "unit": "particle-evals/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{reps} full FP64 oracle evaluations (energy, forces, dE/dq) of the same "
                         f"{n}-ion workload, mean {t_one:.3f} s each"}
        for prec, r in results.items():
            ef, ff = r["energy"], r["forces"]
            errs[prec] = {"rel_E": abs(ef[0] - ref[0][0]) / abs(ref[0][0]),
                          "rel_F": float(np.linalg.norm(ff - ref[1]) / np.linalg.norm(ref[1]))}

    head = results.get("mixed") or results.get("fp64")
    head_prec = "mixed" if "mixed" in results else "fp64"
    kern = head["kernels"]
    dom = max(("sk", "gather", "pair"), key=lambda k: kern.get(k, {}).get("avg_ms", 0.0))

    def roofline(k, prec, kp):
        if k not in FLOPS_PER_UNIT or k not in kp:
            return None
        flops = FLOPS_PER_UNIT[k] * n * nk
        ach = flops / (kp[k]["avg_ms"] * 1e-3) / 1e12
        bound, peak = kernel_bound(k, prec)
        return {"bound": bound, "kernel": k, "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": traffic_bytes(k, args.workload, prec), "avg_ms": kp[k]["avg_ms"],
                "algorithmic_flops_per_launch": flops}

    roof = roofline(dom, head_prec, kern)
    per_kernel_roofline = {p: {k: roofline(k, p, r["kernels"]) for k in FLOPS_PER_UNIT} for p, r in results.items()}
    serve = None
    if not args.no_serving:
        serve = serving(args.serving_systems, args.serving_passes)
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
        "config": {"workload": f"{args.workload}: rock-salt {round(n ** (1 / 3))}^3 N={n} L={sysm.box_L:g} "
                               f"alpha={sysm.alpha} r_c={sysm.r_c} k_max={sysm.k_max} |K+|={nk}",
                   "n": n, "precision": head_prec},
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
        "serving": serve,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
