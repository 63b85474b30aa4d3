"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare with the oracle."""
import json
import os

import numpy as np

TOL = {
    # plain FP64 against the FP64 oracle
    "fp64": dict(energy=1e-10, force=1e-10, dEdq=1e-10),
    # FP32 pair functions and gather phases with FP64 accumulation
    "mixed": dict(energy=1e-6, force=1e-6, dEdq=1e-6),
}
# Per-element bars: max_i |x_i - x_ref,i| over every component, relative to the
# RMS of the reference components.  A norm can hide a fault confined to a few
# particles (one cell, one work item); these cannot.
TOL_ELEM = {"fp64": 1e-9, "mixed": 1e-5}


def run_gpu(pos, q, L, alpha, rc, K, precision, n_max=None, dEdq=True, plan=None, flags=0):
    import torch
    from paper_1708_01135_amd import ewald as ew
    dev = torch.device("cuda:0")
    tp = torch.as_tensor(np.ascontiguousarray(pos), dtype=torch.float64, device=dev)
    tq = torch.as_tensor(np.ascontiguousarray(q), dtype=torch.float64, device=dev)
    own = plan is None
    if own:
        plan = ew.Plan(n_max or len(q), L, alpha, rc, K, precision, flags=flags)
    try:
        e, f, g = plan.energy_forces(tp, tq, True, dEdq)
        torch.cuda.synchronize()
        st = plan.status()
        out = (e.cpu().numpy(), f.cpu().numpy(), None if g is None else g.cpu().numpy(), st)
    finally:
        if own:
            plan.release()
    return out


def rel_err(a, b, floor=0.0):
    """||a - b|| / max(||b||, floor): relative error, with an absolute floor for
    results that vanish exactly (e.g. the force on a lone charge)."""
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    den = max(np.linalg.norm(b), floor)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def _log(record):
    path = os.environ.get("EWALD_ERRLOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(record) + "\n")


def elem_err(a, b, floor=0.0):
    """max_i |a_i - b_i| / max(rms(b), floor) over all components."""
    a, b = np.asarray(a, dtype=float).ravel(), np.asarray(b, dtype=float).ravel()
    rms = max(float(np.sqrt(np.mean(b * b))) if b.size else 0.0, floor)
    return float(np.abs(a - b).max()) / (rms if rms > 0 else 1.0) if b.size else 0.0


def compare(gpu, ref, precision, label=""):
    """Assert the GPU result matches the oracle within the precision's bar;
    returns the measured errors."""
    (eg, fg, dg, st), (er, fr, dr) = gpu, ref
    tol = TOL[precision]
    assert st == 0, f"{label}: device status {st}"
    n = len(fr)
    scale = max(np.abs(er[1:]).max(), 1e-300)
    errs = {
        "energy": abs(eg[0] - er[0]) / max(abs(er[0]), 1e-12 * scale),
        "force": rel_err(fg, fr, 1e-6 * np.sqrt(n)),
        "force_elem": elem_err(fg, fr, 1e-6),
    }
    for p, name in ((1, "real"), (2, "recip"), (3, "self"), (4, "bg")):
        errs[name] = abs(eg[p] - er[p]) / max(abs(er[p]), 1e-12 * scale)
    if dg is not None:
        errs["dEdq"] = rel_err(dg, dr, 1e-6 * np.sqrt(n))
        errs["dEdq_elem"] = elem_err(dg, dr, 1e-6)
    _log({"label": label, "precision": precision, "n": n, **{k: float(v) for k, v in errs.items()}})
    msg = f"{label} {precision}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items())
    print(msg, flush=True)
    assert errs["energy"] <= tol["energy"], msg
    assert errs["force"] <= tol["force"], msg
    assert errs["force_elem"] <= TOL_ELEM[precision], msg
    if dg is not None:
        assert errs["dEdq"] <= tol["dEdq"], msg
        assert errs["dEdq_elem"] <= TOL_ELEM[precision], msg
    return errs
