"""Seeded synthetic inputs for the Ewald hot path.

This module only *draws* particle systems; it holds none of the Ewald
arithmetic, so both the HIP path and the CPU oracle can take their inputs from
it without sharing any of the method.  Every generator is a pure function of
its arguments and a numpy ``default_rng(seed)`` (PCG64) stream.

The systems mimic the paper's benchmark material (section 4: rock-salt NaCl at
fixed number density; the strong-scaling run is a 32^3-site rock-salt crystal)
and a random electrolyte used for the larger and the serving workloads:

* :func:`rock_salt` -- simple cubic lattice of n^3 sites, charges alternating
  +1/-1 by the parity of (i+j+k), every site jittered by U(-j, j)^3.
* :func:`electrolyte` -- N ions placed by random sequential addition (RSA)
  with a minimum (minimum-image) separation, charges +1/-1 balanced to zero.
* :func:`serving_mix` -- a list of independent electrolyte systems with
  log-uniform sizes and Poisson arrival times.

Named configurations (``CONFIGS``) fix shapes and Ewald parameters for the
workloads used by the tests and the benchmark.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = [
    "System",
    "rock_salt",
    "perfect_rock_salt",
    "electrolyte",
    "random_neutral",
    "clustered",
    "serving_mix",
    "CONFIGS",
    "make_config",
]


@dataclasses.dataclass
class System:
    """One periodic system: positions (N,3) float64, charges (N,) float64,
    cubic box side ``box_L`` and the Ewald parameters it is meant for."""

    pos: np.ndarray
    q: np.ndarray
    box_L: float
    alpha: float
    r_c: float
    k_max: int
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.q.shape[0])


def _wrap_into_box(pos: np.ndarray, L: float) -> np.ndarray:
    # Input preparation only: fold jittered lattice sites back into [0, L).
    w = np.mod(pos, L)
    w[w >= L] = 0.0
    return w


def perfect_rock_salt(n_side: int, spacing: float = 1.0) -> Tuple[np.ndarray, np.ndarray, float]:
    """Unjittered rock-salt lattice: sites (i,j,k) in C order (i slowest),
    q = +1 when i+j+k is even, else -1.  Returns (pos, q, L)."""
    idx = np.arange(n_side, dtype=np.int64)
    i, j, k = np.meshgrid(idx, idx, idx, indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    pos = np.stack([i, j, k], axis=1).astype(np.float64) * spacing
    q = np.where((i + j + k) % 2 == 0, 1.0, -1.0)
    return pos, q, n_side * spacing


def rock_salt(n_side: int, jitter: float, seed: int, spacing: float = 1.0,
              wrap: bool = True) -> Tuple[np.ndarray, np.ndarray, float]:
    """Jittered rock-salt lattice: perfect sites plus U(-jitter, jitter)^3
    drawn as one (N,3) array from ``default_rng(seed)``."""
    pos, q, L = perfect_rock_salt(n_side, spacing)
    rng = np.random.default_rng(seed)
    pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    if wrap:
        pos = _wrap_into_box(pos, L)
    return pos, q, L


_RSA_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librsa_accept.so")
_rsa_fn = None


def _rsa_helper():
    """rsa_accept() from csrc_host/rsa_accept.c when it has been built (it
    accepts the same candidates as the NumPy loop below, only faster)."""
    global _rsa_fn
    if _rsa_fn is None and os.path.exists(_RSA_LIB):
        lib = ctypes.CDLL(_RSA_LIB)
        f = lib.rsa_accept
        f.restype = ctypes.c_int64
        f.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                      ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                      ctypes.c_void_p]
        _rsa_fn = f
    return _rsa_fn


def electrolyte(n: int, density: float, seed: int, d_min: float = 0.8,
                batch: int = 65536, use_helper: bool = True) -> Tuple[np.ndarray, np.ndarray, float]:
    """Random electrolyte by random sequential addition (RSA).

    Candidates are drawn uniformly in the cube of side L = (n/density)^(1/3)
    from ``default_rng(seed)``, ``batch`` at a time; a candidate is accepted
    when no previously accepted ion lies closer than ``d_min`` (minimum
    image).  Batching only vectorises the distance tests: acceptance is still
    decided in draw order, so the result is that of one-at-a-time addition.
    Charges: +1 for the first n//2 accepted ions and -1 for the rest (n even),
    then shuffled with the same generator.  With ``use_helper`` the acceptance
    loop runs in the C helper when it is built (same result, faster).
    """
    if n % 2:
        raise ValueError("electrolyte needs an even number of ions")
    L = (n / density) ** (1.0 / 3.0)
    if L < 3.0 * d_min:
        raise ValueError("box too small for RSA with this d_min")
    rng = np.random.default_rng(seed)
    # hash cells with diagonal < d_min hold at most one accepted ion
    g = int(math.floor(L * math.sqrt(3.0) / d_min)) + 1
    h = L / g
    R = int(math.ceil(d_min / h))
    rng_off = np.arange(-R, R + 1, dtype=np.int64)
    offs = np.stack(np.meshgrid(rng_off, rng_off, rng_off, indexing="ij"), -1).reshape(-1, 3)
    occ = np.full(g * g * g, -1, dtype=np.int64)
    out = np.empty((n, 3), dtype=np.float64)
    count = 0
    d2 = d_min * d_min
    helper = _rsa_helper() if use_helper else None
    if helper is not None:
        # the same candidate stream, accepted one at a time in C
        cnt = ctypes.c_int64(0)
        while cnt.value < n:
            cand = np.ascontiguousarray(rng.uniform(0.0, L, size=(batch, 3)))
            helper(L, d_min, g, R, cand.ctypes.data, batch, out.ctypes.data, ctypes.byref(cnt), n,
                   occ.ctypes.data)
        q = np.concatenate([np.ones(n // 2), -np.ones(n - n // 2)])
        rng.shuffle(q)
        return out, q, L

    def min_image(d):
        return d - L * np.round(d / L)

    def key_of(c):
        return (c[..., 0] * g + c[..., 1]) * g + c[..., 2]

    while count < n:
        cand = rng.uniform(0.0, L, size=(batch, 3))
        cell = np.minimum((cand / h).astype(np.int64), g - 1)
        # 1) test against every ion accepted in earlier batches
        ok = np.ones(batch, dtype=bool)
        for o in offs:
            ids = occ[key_of((cell + o) % g)]
            hit = np.nonzero(ok & (ids >= 0))[0]
            if hit.size == 0:
                continue
            d = min_image(cand[hit] - out[ids[hit]])
            ok[hit[np.einsum("pk,pk->p", d, d) < d2]] = False
        surv = np.nonzero(ok)[0]  # increasing draw order
        if surv.size == 0:
            continue
        # 2) conflicts among this batch's survivors (pairs a < b in draw order)
        sc = cell[surv]
        skey_all = key_of(sc)
        order = np.argsort(skey_all, kind="stable")
        skey = skey_all[order]
        pairs = []
        for o in offs:
            nk = key_of((sc + o) % g)
            lo = np.searchsorted(skey, nk, side="left")
            hi = np.searchsorted(skey, nk, side="right")
            cnt = hi - lo
            tot = int(cnt.sum())
            if tot == 0:
                continue
            src = np.repeat(np.arange(surv.size), cnt)
            within = np.arange(tot) - np.repeat(np.cumsum(cnt) - cnt, cnt)
            dst = order[np.repeat(lo, cnt) + within]
            keep = dst < src
            src, dst = src[keep], dst[keep]
            if src.size == 0:
                continue
            d = min_image(cand[surv[src]] - cand[surv[dst]])
            close = np.einsum("pk,pk->p", d, d) < d2
            if close.any():
                pairs.append(np.stack([src[close], dst[close]], axis=1))
        accepted = np.ones(surv.size, dtype=bool)
        if pairs:
            # sorted by the later index b: a's fate is final before b is decided
            for b_, a_ in np.unique(np.concatenate(pairs), axis=0):
                if accepted[a_]:
                    accepted[b_] = False
        take = surv[accepted][: n - count]
        if take.size:
            tkey = key_of(cell[take])
            if np.any(occ[tkey] >= 0) or np.unique(tkey).size != tkey.size:
                raise RuntimeError("RSA hash invariant violated")
            occ[tkey] = count + np.arange(take.size)
            out[count:count + take.size] = cand[take]
            count += take.size
    q = np.concatenate([np.ones(n // 2), -np.ones(n - n // 2)])
    rng.shuffle(q)
    return out, q, L


def random_neutral(n: int, box_L: float, seed: int, charge_scale: float = 1.0,
                   neutral: bool = True) -> Tuple[np.ndarray, np.ndarray]:
    """Uniform random positions in [0, L)^3 and random charges.

    Charges are U(-1, 1) * charge_scale; with ``neutral`` the mean is removed
    so the total charge is zero (up to rounding).  Used for small edge-case
    systems (ragged sizes, tiny boxes, non-integer charges)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box_L, size=(n, 3))
    q = rng.uniform(-1.0, 1.0, size=n) * charge_scale
    if neutral and n > 1:
        q = q - q.mean()
    return pos, q


def clustered(n_cluster: int, n_rest: int, box_L: float, corner, side: float, seed: int,
              jitter: float = 0.3) -> Tuple[np.ndarray, np.ndarray]:
    """A dense cluster inside a dilute background (edge case: crowded cells).

    ``n_cluster`` ions sit on a jittered simple cubic grid filling the cube
    [corner, corner + side)^3 (grid spacing s = side / ceil(n_cluster^(1/3)),
    each site moved by U(-jitter s / 2, jitter s / 2)^3, so no two ions are
    closer than (1 - jitter) s); charges alternate +-1 by the parity of the
    grid site.  ``n_rest`` ions are uniform in the box outside that cube
    (expanded by one grid spacing), with charges +-1 alternating in draw order.
    Everything is drawn from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    m = int(math.ceil(n_cluster ** (1.0 / 3.0) - 1e-9))
    sp = side / m
    idx = np.arange(m ** 3)[:n_cluster]
    i, j, k = idx // (m * m), (idx // m) % m, idx % m
    base = np.asarray(corner, dtype=np.float64) + (np.stack([i, j, k], axis=1) + 0.5) * sp
    pos_c = base + rng.uniform(-0.5 * jitter * sp, 0.5 * jitter * sp, size=base.shape)
    q_c = np.where((i + j + k) % 2 == 0, 1.0, -1.0)
    lo = np.asarray(corner, dtype=np.float64) - sp
    hi = lo + side + 2 * sp
    rest = np.empty((0, 3))
    while rest.shape[0] < n_rest:
        cand = rng.uniform(0.0, box_L, size=(2 * n_rest + 16, 3))
        inside = np.all((cand >= lo) & (cand < hi), axis=1)
        rest = np.concatenate([rest, cand[~inside]])
    rest = rest[:n_rest]
    q_r = np.where(np.arange(n_rest) % 2 == 0, 1.0, -1.0)
    return np.concatenate([pos_c, rest]), np.concatenate([q_c, q_r])


def _serving_system(args):
    n, density, seed = args
    # candidate batches sized to the system (the draw order, hence the ions, do
    # not depend on the batch; only the charge shuffle that follows the draws does)
    pos, q, _ = electrolyte(n, density, seed, batch=min(65536, max(4096, 2 * n)))
    return pos, q


def serving_mix(n_systems: int = 256, seed: int = 0, n_lo: int = 500, n_hi: int = 50000,
                density: float = 0.8, r_c: float = 4.5, real_exponent: float = 14.4,
                rate_hz: float = 1000.0, build_systems: bool = True, workers: int = 1) -> List[Dict]:
    """Independent electrolyte systems for the serving workload.

    Sizes: N_s = 2*round(exp(U(ln n_lo, ln n_hi))/2).  Each system is an RSA
    electrolyte at ``density`` with seed ``seed + 1 + s``; alpha is set so that
    alpha * r_c^2 = ``real_exponent`` and K_s = ceil(sqrt(alpha*real_exponent)*L_s/pi)
    matches the reciprocal exponent to the real one.  Arrival times are a
    Poisson process of ``rate_hz`` drawn from ``default_rng(1000 + seed)``.
    The systems are independent, so ``workers`` > 1 builds them in a process
    pool (same result).
    """
    rng = np.random.default_rng(seed)
    sizes = 2 * np.round(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_systems)) / 2)
    sizes = sizes.astype(np.int64)
    arr = np.random.default_rng(1000 + seed)
    gaps = arr.exponential(1.0 / rate_hz, size=n_systems)
    t_arrive = np.cumsum(gaps) - gaps[0]
    alpha = real_exponent / (r_c * r_c)
    out = []
    for s in range(n_systems):
        n = int(sizes[s])
        L = (n / density) ** (1.0 / 3.0)
        k_max = int(math.ceil(math.sqrt(alpha * real_exponent) * L / math.pi))
        out.append({"n": n, "box_L": L, "alpha": alpha, "r_c": r_c, "k_max": k_max,
                    "t_arrive": float(t_arrive[s]), "seed": seed + 1 + s})
    if build_systems:
        jobs = [(it["n"], density, it["seed"]) for it in out]
        if workers > 1:
            import concurrent.futures as cf
            import multiprocessing as mp
            with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
                built = list(ex.map(_serving_system, jobs, chunksize=1))
        else:
            built = [_serving_system(j) for j in jobs]
        for it, (pos, q) in zip(out, built):
            it["pos"], it["q"] = pos, q
    return out


# Named workloads.  Sizes and parameters follow the rock-salt lattices and the
# random electrolyte described in the module docstring; alpha is the Gaussian
# exponent of the paper's splitting (real-space kernel erfc(sqrt(alpha) r)).
CONFIGS: Dict[str, Dict] = {
    "rocksalt8": dict(kind="rock_salt", n_side=8, jitter=0.1, alpha=0.9, r_c=4.0, k_max=8),
    "rocksalt32": dict(kind="rock_salt", n_side=32, jitter=0.1, alpha=0.7, r_c=4.5, k_max=20),
    "rocksalt64": dict(kind="rock_salt", n_side=64, jitter=0.15, alpha=0.6, r_c=5.0, k_max=32),
    "electrolyte1m": dict(kind="electrolyte", n=1_000_000, density=0.8, alpha=0.5, r_c=5.5,
                          k_max=40),
}


def make_config(name: str, seed: int = 0) -> System:
    """Build one named workload with the given seed."""
    c = CONFIGS[name]
    if c["kind"] == "rock_salt":
        pos, q, L = rock_salt(c["n_side"], c["jitter"], seed)
    elif c["kind"] == "electrolyte":
        pos, q, L = electrolyte(c["n"], c["density"], seed)
    else:  # pragma: no cover
        raise KeyError(name)
    return System(pos=pos, q=q, box_L=L, alpha=c["alpha"], r_c=c["r_c"], k_max=c["k_max"],
                  name=name)
