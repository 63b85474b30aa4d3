"""Write oracle reference values for the full-size workloads.

Calls only the FP64 oracle (``oracle/``) and the seeded input generators.
For each workload it stores: a checksum of the generated input, every energy
part, S(k) at sampled half-space k vectors, and forces / dE/dq on sampled
particles.  Usage:  python tests/golden/make_golden.py rocksalt64 electrolyte1m
"""
import json
import math
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
N_P_SAMPLES = 256


def input_checksum(s):
    return {"sum_pos": float(np.sum(s.pos)), "sum_pos2": float(np.sum(s.pos * s.pos)),
            "sum_q": float(np.sum(s.q)), "sum_qx": float(np.sum(s.q * s.pos[:, 0]))}


def make(name, seed=0):
    t0 = time.time()
    s = wl.make_config(name, seed)
    print(f"{name}: N={s.n} generated in {time.time() - t0:.1f}s", flush=True)
    rng = np.random.default_rng(12345 + seed)
    targets = np.sort(rng.choice(s.n, N_P_SAMPLES, replace=False))
    kv = oracle.kset(s.k_max, half=True)
    kidx = np.sort(rng.choice(len(kv), min(N_K_SAMPLES, len(kv)), replace=False))
    t0 = time.time()
    e_real, f_real, p_real = oracle.real_space(s.pos, s.q, s.box_L, s.alpha, s.r_c, oracle.FAST)
    print(f"  real space {time.time() - t0:.1f}s", flush=True)
    t0 = time.time()
    e_rec, f_rec, p_rec, sk = oracle.recip_space(s.pos, s.q, s.box_L, s.alpha, s.k_max, oracle.FAST,
                                                 targets=targets, want_sk=True)
    print(f"  reciprocal {time.time() - t0:.1f}s", flush=True)
    q2, Q, V = float(np.sum(s.q * s.q)), float(np.sum(s.q)), s.box_L ** 3
    e_self = -math.sqrt(s.alpha / math.pi) * q2
    e_bg = -math.pi * Q * Q / (2 * V * s.alpha)
    forces = f_real[targets] + f_rec
    dEdq = p_real[targets] + p_rec - 2 * math.sqrt(s.alpha / math.pi) * s.q[targets] - math.pi * Q / (V * s.alpha)
    out = {
        "workload": name, "seed": seed, "n": s.n, "box_L": s.box_L, "alpha": s.alpha, "r_c": s.r_c,
        "k_max": s.k_max, "input_checksum": input_checksum(s),
        "energy": [e_real + e_rec + e_self + e_bg, e_real, e_rec, e_self, e_bg],
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
