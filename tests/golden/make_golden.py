"""Write oracle reference values for the full-size workloads.

Every stored number is computed by the FP64 oracle (``oracle/``) from the
seeded input generators; this script only chooses what to sample and writes
JSON.  For each workload it stores: a checksum of the generated input, every
energy part, S(k) at sampled half-space k vectors, and forces / dE/dq on
sampled particles.

The particle sample is stratified over space: the box is cut into
``N_STRATA``^3 equal blocks and one particle is drawn from every non-empty
block, so that every region of the box (every cell, every work item of the
GPU path, whatever its placement) is represented.

Usage:  python tests/golden/make_golden.py rocksalt64 electrolyte1m
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1708_01135_amd import workloads as wl  # noqa: E402

N_K_SAMPLES = 4096
N_STRATA = 16  # 16^3 = 4096 spatial blocks, one sampled particle each


def input_checksum(s):
    return {"sum_pos": float(np.sum(s.pos)), "sum_pos2": float(np.sum(s.pos * s.pos)),
            "sum_q": float(np.sum(s.q)), "sum_qx": float(np.sum(s.q * s.pos[:, 0]))}


def stratified_targets(pos, L, rng, strata=N_STRATA):
    """One particle index drawn uniformly from each non-empty block of a
    strata^3 grid over the (wrapped) box, in block order."""
    w = np.mod(pos, L)
    b = np.minimum((w / (L / strata)).astype(np.int64), strata - 1)
    key = (b[:, 0] * strata + b[:, 1]) * strata + b[:, 2]
    order = np.argsort(key, kind="stable")
    skey = key[order]
    starts = np.flatnonzero(np.r_[True, skey[1:] != skey[:-1]])
    ends = np.r_[starts[1:], len(skey)]
    pick = starts + (rng.random(len(starts)) * (ends - starts)).astype(np.int64)
    return np.sort(order[pick])


def make(name, seed=0):
    t0 = time.time()
    s = wl.make_config(name, seed)
    print(f"{name}: N={s.n} generated in {time.time() - t0:.1f}s", flush=True)
    rng = np.random.default_rng(12345 + seed)
    targets = stratified_targets(s.pos, s.box_L, rng)
    kv = oracle.kset(s.k_max, half=True)
    kidx = np.sort(rng.choice(len(kv), min(N_K_SAMPLES, len(kv)), replace=False))
    t0 = time.time()
    energy, forces, dEdq, sk = oracle.energy_forces_targets(s.pos, s.q, s.box_L, s.alpha, s.r_c, s.k_max,
                                                            targets=targets, method=oracle.FAST, want_sk=True)
    print(f"  oracle {time.time() - t0:.1f}s, {len(targets)} targets", flush=True)
    out = {
        "workload": name, "seed": seed, "n": s.n, "box_L": s.box_L, "alpha": s.alpha, "r_c": s.r_c,
        "k_max": s.k_max, "input_checksum": input_checksum(s),
        "energy": energy.tolist(),
        "targets": targets.tolist(), "forces": forces.tolist(), "dEdq": dEdq.tolist(),
        "k_samples": kv[kidx].tolist(), "sk_re": sk.real[kidx].tolist(), "sk_im": sk.imag[kidx].tolist(),
        "oracle_threads": oracle.num_threads(),
    }
    path = os.path.join(HERE, f"oracle_{name}_s{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"  wrote {path}", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["rocksalt64", "electrolyte1m"]:
        make(name)
