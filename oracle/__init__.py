"""Plain FP64 CPU oracle for classical Ewald summation -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It wraps ``libewald_oracle.so`` (plain C, see
``ewald_oracle.c`` for the formulas and the paper passages they follow) with
numpy marshalling and shares no code with the HIP path.

Routes (see ``ewald_oracle.c``): ``"brute"`` sums every pair/image and the full
k set with direct sin/cos; ``"fast"`` uses a plain cell list for real space and
the half-space k set with per-axis cos/sin tables for reciprocal space.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libewald_oracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)

BRUTE = 0
FAST = 1


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # compile on first use (CPU only, gcc)
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_kset.restype = ctypes.c_int64
    lib.oracle_kset.argtypes = [ctypes.c_int, ctypes.c_int, _i32]
    lib.oracle_structure_factor.restype = ctypes.c_int
    lib.oracle_structure_factor.argtypes = [ctypes.c_int64, _d, _d, ctypes.c_double, ctypes.c_int64,
                                            _i32, _d, _d]
    lib.oracle_real_space.restype = ctypes.c_int
    lib.oracle_real_space.argtypes = [ctypes.c_int64, _d, _d, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_int64, _i64, _d, _d, _d]
    lib.oracle_recip_space.restype = ctypes.c_int
    lib.oracle_recip_space.argtypes = [ctypes.c_int64, _d, _d, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i64, _d, _d, _d,
                                       _d, _d]
    lib.oracle_energy_forces.restype = ctypes.c_int
    lib.oracle_energy_forces.argtypes = [ctypes.c_int64, _d, _d, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int, _d, _d, _d]
    lib.oracle_energy_forces_targets.restype = ctypes.c_int
    lib.oracle_energy_forces_targets.argtypes = [ctypes.c_int64, _d, _d, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                                 _i64, _d, _d, _d, _d, _d]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray], t=_d):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check(st: int, what: str):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(t: int) -> None:
    _load().oracle_set_num_threads(int(t))


def kset(k_max: int, half: bool = True) -> np.ndarray:
    """Integer vectors n != 0 with |n|^2 <= k_max^2 (half space if ``half``), (nk, 3) int32."""
    lib = _load()
    nk = lib.oracle_kset(int(k_max), int(bool(half)), None)
    out = np.zeros((nk, 3), dtype=np.int32)
    lib.oracle_kset(int(k_max), int(bool(half)), _p(out, _i32))
    return out


def structure_factor(pos, q, box_L: float, kvecs) -> np.ndarray:
    """S_k = sum_j q_j exp(i k.r_j) for integer vectors ``kvecs`` (direct sin/cos)."""
    pos, q = _f64(pos), _f64(q)
    kv = np.ascontiguousarray(np.asarray(kvecs, dtype=np.int32).reshape(-1, 3))
    re = np.zeros(len(kv))
    im = np.zeros(len(kv))
    _check(_load().oracle_structure_factor(len(q), _p(pos), _p(q), box_L, len(kv), _p(kv, _i32),
                                           _p(re), _p(im)), "structure_factor")
    return re + 1j * im


def real_space(pos, q, box_L, alpha, r_c, method=FAST, targets: Optional[Sequence[int]] = None):
    """(E_real or None, F_real (nt,3), phi_real (nt,)) for all particles or the targets."""
    pos, q = _f64(pos), _f64(q)
    tg = None if targets is None else np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    nt = len(q) if tg is None else len(tg)
    e = np.zeros(1)
    f = np.zeros((nt, 3))
    ph = np.zeros(nt)
    _check(_load().oracle_real_space(len(q), _p(pos), _p(q), box_L, alpha, r_c, int(method),
                                     0 if tg is None else len(tg), _p(tg, _i64), _p(e), _p(f), _p(ph)),
           "real_space")
    return (float(e[0]) if tg is None else None), f, ph


def recip_space(pos, q, box_L, alpha, k_max, method=FAST, targets: Optional[Sequence[int]] = None,
                want_sk: bool = False):
    """(E_recip, F_recip (nt,3), phi_recip (nt,)[, S_k over the half space in kset() order])."""
    pos, q = _f64(pos), _f64(q)
    tg = None if targets is None else np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    nt = len(q) if tg is None else len(tg)
    e = np.zeros(1)
    f = np.zeros((nt, 3))
    ph = np.zeros(nt)
    skr = ski = None
    if want_sk:
        if method != FAST:
            raise ValueError("S_k output needs the table route")
        nk = len(kset(k_max, True))
        skr, ski = np.zeros(nk), np.zeros(nk)
    _check(_load().oracle_recip_space(len(q), _p(pos), _p(q), box_L, alpha, int(k_max), int(method),
                                      0 if tg is None else len(tg), _p(tg, _i64), _p(e), _p(f), _p(ph),
                                      _p(skr), _p(ski)), "recip_space")
    if want_sk:
        return float(e[0]), f, ph, skr + 1j * ski
    return float(e[0]), f, ph


def energy_forces(pos, q, box_L, alpha, r_c, k_max, method=FAST) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(energy[5] = total, real, recip, self, background; forces (n,3); dE/dq (n,))."""
    pos, q = _f64(pos), _f64(q)
    n = len(q)
    en = np.zeros(5)
    f = np.zeros((n, 3))
    dq = np.zeros(n)
    _check(_load().oracle_energy_forces(n, _p(pos), _p(q), box_L, alpha, r_c, int(k_max), int(method),
                                        _p(en), _p(f), _p(dq)), "energy_forces")
    return en, f, dq


def energy_forces_targets(pos, q, box_L, alpha, r_c, k_max, targets=None, method=FAST, want_sk=False):
    """(energy[5], forces (nt,3), dE/dq (nt,)[, S_k over the half space in kset() order]) with the
    per-particle results of the listed targets only (all particles when ``targets`` is None).

    Every value is assembled inside the C oracle: the real-space sums run over all
    particles (E_real needs every phi_i), the reciprocal forces and potentials over the
    targets."""
    pos, q = _f64(pos), _f64(q)
    tg = None if targets is None else np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    nt = len(q) if tg is None else len(tg)
    en = np.zeros(5)
    f = np.zeros((nt, 3))
    dq = np.zeros(nt)
    skr = ski = None
    if want_sk:
        nk = len(kset(k_max, True))
        skr, ski = np.zeros(nk), np.zeros(nk)
    _check(_load().oracle_energy_forces_targets(len(q), _p(pos), _p(q), box_L, alpha, r_c, int(k_max),
                                                int(method), 0 if tg is None else len(tg), _p(tg, _i64),
                                                _p(en), _p(f), _p(dq), _p(skr), _p(ski)),
           "energy_forces_targets")
    if want_sk:
        return en, f, dq, skr + 1j * ski
    return en, f, dq
