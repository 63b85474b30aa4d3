"""Thin ctypes binding of ``libewald_mi355x.so`` (C ABI in ``include/ewald.h``).

Argument marshalling only: every step of the evaluation runs in the library's
HIP kernels.  PyTorch supplies device memory and the current stream.  If the
library has not been built, importing the binding raises immediately -- there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libewald_mi355x.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_CAPACITY = -2
ERR_OUT_OF_MEMORY = -3
ERR_DEVICE = -4
ERR_NONFINITE = -5
ERR_ADMISSION = -6
ERR_SCRATCH = -7

FP64 = 0
MIXED = 1
K_MAX_LIMIT = 100
FLAG_VALU_GATHER = 1
FLAG_VALU_SK = 2
FLAG_NO_GRAPH = 4
FLAG_NO_WORKSPACE = 8
FLAG_ONE_STREAM = 16
SERVER_FLAG_EXPRESS_CUS = 1
SERVER_FLAG_NO_BATCH = 2
SCRATCH_BYTES = 64 << 20  # EWALD_SCRATCH_BYTES

ENERGY_PARTS = ("total", "real", "recip", "self", "background")


class EwaldError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _lib.ewald_status_string(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


class Params(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int64), ("box_L", ctypes.c_double), ("alpha", ctypes.c_double),
                ("r_c", ctypes.c_double), ("k_max", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32), ("flags", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class ServerParams(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("n_streams", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("hbm_budget", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("systems", ctypes.c_int64), ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("in_flight", ctypes.c_int64), ("budget", ctypes.c_uint64), ("used", ctypes.c_uint64),
                ("peak_used", ctypes.c_uint64), ("held", ctypes.c_int64), ("held_total", ctypes.c_int64),
                ("masked_streams", ctypes.c_int64), ("batches", ctypes.c_int64), ("batched", ctypes.c_int64)]


class DebugStats(ctypes.Structure):
    _fields_ = [("max_cell_count", ctypes.c_int64), ("direct_particles", ctypes.c_int64),
                ("listed_pairs", ctypes.c_int64), ("cells_per_axis", ctypes.c_int32), ("list_capacity", ctypes.c_int32),
                ("sk_matrix_cores", ctypes.c_int32), ("gather_matrix_cores", ctypes.c_int32),
                ("phase_rows", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sk_mfma_flops", ctypes.c_int64), ("gather_mfma_flops", ctypes.c_int64)]


_lib = None


def _precision_code(precision) -> int:
    if isinstance(precision, str):
        return {"fp64": FP64, "mixed": MIXED}[precision.lower()]
    return int(precision)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python __graft_entry__.py` "
                          "or `python paper_1708_01135_amd/build.py` (hipcc, gfx950)")
    # The library links the HIP runtime by its soname (libamdhip64.so.7); the
    # PyTorch wheel ships its own copy under the same soname.  Loading torch
    # first makes the library bind to that one runtime, so the device pointers
    # and streams torch hands over are valid in it (loaded the other way round,
    # plan creation fails with a device error).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Params)
    vp = ctypes.c_void_p
    lib.ewald_status_string.restype = ctypes.c_char_p
    lib.ewald_status_string.argtypes = [ctypes.c_int]
    lib.ewald_params_validate.restype = ctypes.c_int
    lib.ewald_params_validate.argtypes = [P]
    lib.ewald_plan_workspace_bytes.restype = ctypes.c_size_t
    lib.ewald_plan_workspace_bytes.argtypes = [P]
    lib.ewald_kset_size.restype = ctypes.c_int64
    lib.ewald_kset_size.argtypes = [ctypes.c_int32]
    lib.ewald_plan.restype = ctypes.c_int
    lib.ewald_plan.argtypes = [P, ctypes.POINTER(vp)]
    lib.ewald_plan_set_stream.restype = ctypes.c_int
    lib.ewald_plan_set_stream.argtypes = [vp, vp]
    lib.ewald_energy_forces.restype = ctypes.c_int
    lib.ewald_energy_forces.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp]
    lib.ewald_eval_workspace_bytes.restype = ctypes.c_size_t
    lib.ewald_eval_workspace_bytes.argtypes = [vp, ctypes.c_int64]
    lib.ewald_energy_forces_ws.restype = ctypes.c_int
    lib.ewald_energy_forces_ws.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp, ctypes.c_size_t]
    lib.ewald_energy_forces_noalloc.restype = ctypes.c_int
    lib.ewald_energy_forces_noalloc.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp]
    lib.ewald_energy_forces_batch.restype = ctypes.c_int
    lib.ewald_energy_forces_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(vp),
                                              ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                              ctypes.POINTER(vp), ctypes.POINTER(vp),
                                              ctypes.POINTER(ctypes.c_size_t), vp]
    lib.ewald_energy.restype = ctypes.c_int
    lib.ewald_energy.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
    lib.ewald_energy_backward.restype = ctypes.c_int
    lib.ewald_energy_backward.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    lib.ewald_plan_status.restype = ctypes.c_int
    lib.ewald_plan_status.argtypes = [vp]
    lib.ewald_release.restype = None
    lib.ewald_release.argtypes = [vp]
    lib.ewald_plan_kcount.restype = ctypes.c_int64
    lib.ewald_plan_kcount.argtypes = [vp]
    lib.ewald_debug_kset.restype = ctypes.c_int
    lib.ewald_debug_kset.argtypes = [vp, vp]
    lib.ewald_debug_copy_sk.restype = ctypes.c_int
    lib.ewald_debug_copy_sk.argtypes = [vp, vp, vp]
    lib.ewald_debug_stats_read.restype = ctypes.c_int
    lib.ewald_debug_stats_read.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(DebugStats)]
    lib.ewald_profile_enable.restype = ctypes.c_int
    lib.ewald_profile_enable.argtypes = [vp, ctypes.c_int32]
    lib.ewald_profile_read.restype = ctypes.c_int32
    lib.ewald_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
    lib.ewald_profile_reset.restype = ctypes.c_int
    lib.ewald_profile_reset.argtypes = [vp]
    # request server (include/ewald_server.h)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.ewald_server_clock.restype = ctypes.c_double
    lib.ewald_server_clock.argtypes = []
    lib.ewald_server_create.restype = ctypes.c_int
    lib.ewald_server_create.argtypes = [ctypes.POINTER(ServerParams), ctypes.POINTER(vp)]
    lib.ewald_server_add_system.restype = ctypes.c_int
    lib.ewald_server_add_system.argtypes = [vp, P, ctypes.POINTER(ctypes.c_int32)]
    lib.ewald_server_remove_system.restype = ctypes.c_int
    lib.ewald_server_remove_system.argtypes = [vp, ctypes.c_int32]
    lib.ewald_server_submit.restype = ctypes.c_int
    lib.ewald_server_submit.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, vp, vp, vp, vp, vp, i64p]
    lib.ewald_server_wait.restype = ctypes.c_int
    lib.ewald_server_wait.argtypes = [vp, ctypes.c_int64, dp, dp]
    lib.ewald_server_poll.restype = ctypes.c_int
    lib.ewald_server_poll.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]
    lib.ewald_server_drain.restype = ctypes.c_int
    lib.ewald_server_drain.argtypes = [vp]
    lib.ewald_server_system_status.restype = ctypes.c_int
    lib.ewald_server_system_status.argtypes = [vp, ctypes.c_int32]
    lib.ewald_server_get_stats.restype = ctypes.c_int
    lib.ewald_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.ewald_server_destroy.restype = None
    lib.ewald_server_destroy.argtypes = [vp]
    _lib = lib
    return lib


def library():
    """The loaded ctypes library (raises ImportError if it was not built)."""
    return _load()


def make_params(n_max, box_L, alpha, r_c, k_max, precision=FP64, device=0, stream=None, flags=0) -> Params:
    precision = _precision_code(precision)
    return Params(int(n_max), float(box_L), float(alpha), float(r_c), int(k_max), int(precision),
                  int(device), int(flags), stream)


def validate(params: Params) -> int:
    return int(_load().ewald_params_validate(ctypes.byref(params)))


def workspace_bytes(params: Params) -> int:
    return int(_load().ewald_plan_workspace_bytes(ctypes.byref(params)))


def kset_size(k_max: int) -> int:
    return int(_load().ewald_kset_size(int(k_max)))


def status_string(status: int) -> str:
    return _load().ewald_status_string(int(status)).decode()


def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_outputs(out, n):
    """Caller-given outputs (energy[5], forces (n,3) or None, dEdq (n,) or
    None): contiguous float64 device tensors of exactly those shapes, since the
    kernels write through their pointers."""
    import torch
    e, f, g = out
    for name, t, shape in (("energy", e, (5,)), ("forces", f, (n, 3)), ("dEdq", g, (n,))):
        if t is None and name != "energy":
            continue
        if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {shape}")
    return e, f, g


class Plan:
    """One Ewald plan: box, splitting, cutoffs, capacity and precision fixed.

    ``energy_forces(pos, q)`` takes float64 device tensors (n,3) and (n,) and
    returns ``(energy[5], forces or None, dEdq or None)`` as device tensors,
    enqueued on the current torch stream.
    """

    def __init__(self, n_max: int, box_L: float, alpha: float, r_c: float, k_max: int,
                 precision="fp64", device: int = 0, flags: int = 0):
        lib = _load()
        import torch
        self.device = torch.device("cuda", device)
        self.params = make_params(n_max, box_L, alpha, r_c, k_max, precision, device,
                                  _stream_handle(torch.cuda.current_stream(self.device)), flags)
        h = ctypes.c_void_p()
        st = lib.ewald_plan(ctypes.byref(self.params), ctypes.byref(h))
        if st != OK:
            raise EwaldError(st, "ewald_plan")
        self._h = h

    @property
    def handle(self) -> int:
        if self._h is None:
            raise RuntimeError("plan was released")
        return self._h.value

    @property
    def kcount(self) -> int:
        return int(_load().ewald_plan_kcount(self.handle))

    def energy_forces(self, pos, q, forces: bool = True, dEdq: bool = False, out=None):
        import torch
        lib = _load()
        n = int(q.shape[0])
        for name, t, shape in (("pos", pos, (n, 3)), ("q", q, (n,))):
            if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {shape}")
        if out is None:
            e = torch.empty(5, dtype=torch.float64, device=pos.device)
            f = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if forces else None
            g = torch.empty(n, dtype=torch.float64, device=pos.device) if dEdq else None
        else:
            e, f, g = _check_outputs(out, n)
        st = lib.ewald_plan_set_stream(self.handle, _stream_handle())
        if st != OK:
            raise EwaldError(st, "ewald_plan_set_stream")
        st = lib.ewald_energy_forces(self.handle, n, pos.data_ptr(), q.data_ptr(), e.data_ptr(),
                                     f.data_ptr() if f is not None else None,
                                     g.data_ptr() if g is not None else None)
        if st != OK:
            raise EwaldError(st, "ewald_energy_forces")
        return e, f, g

    def eval_workspace_bytes(self, n: int) -> int:
        """Bytes of the per-evaluation buffers of an evaluation of ``n`` particles."""
        return int(_load().ewald_eval_workspace_bytes(self.handle, int(n)))

    def energy_forces_ws(self, pos, q, workspace, out):
        """Evaluation with the per-evaluation buffers in ``workspace`` (a device
        tensor of at least ``eval_workspace_bytes(n)`` bytes, 256-byte aligned);
        ``out`` = (energy[5], forces (n,3) or None, dEdq (n,) or None)."""
        n = self._check_inputs(pos, q)
        e, f, g = _check_outputs(out, n)
        nbytes = workspace.numel() * workspace.element_size()
        st = _load().ewald_energy_forces_ws(self.handle, n, pos.data_ptr(), q.data_ptr(), e.data_ptr(),
                                            f.data_ptr() if f is not None else None,
                                            g.data_ptr() if g is not None else None, workspace.data_ptr(), nbytes)
        if st != OK:
            raise EwaldError(st, "ewald_energy_forces_ws")
        return e, f, g

    def energy_forces_noalloc(self, pos, q, out):
        """The allocation-free evaluation: ``out`` = (energy[5], forces (n,3) or
        None, dEdq (n,) or None), preallocated float64 device tensors, is
        overwritten; the library's static scratch holds every other buffer."""
        n = self._check_inputs(pos, q)
        e, f, g = _check_outputs(out, n)
        st = _load().ewald_energy_forces_noalloc(self.handle, n, pos.data_ptr(), q.data_ptr(), e.data_ptr(),
                                                 f.data_ptr() if f is not None else None,
                                                 g.data_ptr() if g is not None else None)
        if st != OK:
            raise EwaldError(st, "ewald_energy_forces_noalloc")
        return e, f, g

    def _check_inputs(self, pos, q):
        import torch
        n = int(q.shape[0])
        for name, t, shape in (("pos", pos, (n, 3)), ("q", q, (n,))):
            if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {shape}")
        st = _load().ewald_plan_set_stream(self.handle, _stream_handle())
        if st != OK:
            raise EwaldError(st, "ewald_plan_set_stream")
        return n

    def energy(self, pos, q):
        """Energy parts (5,) only; the force gather is skipped."""
        import torch
        n = self._check_inputs(pos, q)
        e = torch.empty(5, dtype=torch.float64, device=pos.device)
        st = _load().ewald_energy(self.handle, n, pos.data_ptr(), q.data_ptr(), e.data_ptr())
        if st != OK:
            raise EwaldError(st, "ewald_energy")
        return e

    def energy_backward(self, pos, q, grad_energy, need_pos=True, need_q=True):
        """(dL/dpos, dL/dq) for the upstream gradient ``grad_energy`` (device scalar)."""
        import torch
        n = self._check_inputs(pos, q)
        g = grad_energy.detach().to(dtype=torch.float64).reshape(1).contiguous()
        e = torch.empty(5, dtype=torch.float64, device=pos.device)
        gp = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if need_pos else None
        gq = torch.empty(n, dtype=torch.float64, device=pos.device) if need_q else None
        st = _load().ewald_energy_backward(self.handle, n, pos.data_ptr(), q.data_ptr(), g.data_ptr(), e.data_ptr(),
                                           gp.data_ptr() if gp is not None else None,
                                           gq.data_ptr() if gq is not None else None)
        if st != OK:
            raise EwaldError(st, "ewald_energy_backward")
        return gp, gq

    def status(self) -> int:
        return int(_load().ewald_plan_status(self.handle))

    def kset(self):
        import numpy as np
        out = np.zeros((self.kcount, 3), dtype=np.int32)
        st = _load().ewald_debug_kset(self.handle, out.ctypes.data)
        if st != OK:
            raise EwaldError(st, "ewald_debug_kset")
        return out

    def structure_factor(self):
        import numpy as np
        re = np.zeros(self.kcount)
        im = np.zeros(self.kcount)
        st = _load().ewald_debug_copy_sk(self.handle, re.ctypes.data, im.ctypes.data)
        if st != OK:
            raise EwaldError(st, "ewald_debug_copy_sk")
        return re + 1j * im

    def debug_stats(self, n: int) -> Dict[str, int]:
        """Branches the plan takes, and those its last evaluation of ``n`` particles took."""
        out = DebugStats()
        st = _load().ewald_debug_stats_read(self.handle, int(n), ctypes.byref(out))
        if st != OK:
            raise EwaldError(st, "ewald_debug_stats_read")
        return {k: int(getattr(out, k)) for k, _ in DebugStats._fields_ if not k.startswith("reserved")}

    def profile(self, enable: bool = True):
        _load().ewald_profile_enable(self.handle, int(bool(enable)))

    def profile_read(self) -> Dict[str, Tuple[float, int]]:
        lib = _load()
        m = 32
        names = (ctypes.c_char_p * m)()
        ms = (ctypes.c_double * m)()
        cnt = (ctypes.c_int64 * m)()
        k = lib.ewald_profile_read(self.handle, names, ms, cnt, m)
        return {names[i].decode(): (float(ms[i]), int(cnt[i])) for i in range(min(k, m))}

    def profile_reset(self):
        _load().ewald_profile_reset(self.handle)

    def release(self):
        if getattr(self, "_h", None) is not None:
            _load().ewald_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.release()


BATCH_MAX = 1024


def energy_forces_batch(items, workspaces=None):
    """ewald_energy_forces_batch(): many systems in one launch sequence.

    ``items``: sequence of (plan, pos, q, out) with ``out`` = (energy[5],
    forces (n,3) or None, dEdq (n,) or None) preallocated float64 device
    tensors.  ``workspaces``: None (each plan's own buffers) or one device
    tensor per item (or None entries) of at least
    ``plan.eval_workspace_bytes(n)`` bytes.  Enqueued on torch's current
    stream; returns the list of ``out``."""
    import torch
    count = len(items)
    if not 1 <= count <= BATCH_MAX:
        raise ValueError(f"a batch holds 1 .. {BATCH_MAX} systems")
    vp = ctypes.c_void_p
    plans, ns = (vp * count)(), (ctypes.c_int64 * count)()
    pos_a, q_a, e_a, f_a, g_a, w_a = ((vp * count)() for _ in range(6))
    wb = (ctypes.c_size_t * count)()
    for i, (plan, pos, q, out) in enumerate(items):
        n = int(q.shape[0])
        for name, t, shape in (("pos", pos, (n, 3)), ("q", q, (n,))):
            if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {shape}")
        e, f, g = _check_outputs(out, n)
        plans[i], ns[i] = plan.handle, n
        pos_a[i], q_a[i], e_a[i] = pos.data_ptr(), q.data_ptr(), e.data_ptr()
        f_a[i] = f.data_ptr() if f is not None else None
        g_a[i] = g.data_ptr() if g is not None else None
        w = workspaces[i] if workspaces is not None else None
        w_a[i] = w.data_ptr() if w is not None else None
        wb[i] = w.numel() * w.element_size() if w is not None else 0
    st = _load().ewald_energy_forces_batch(count, plans, ns, pos_a, q_a, e_a, f_a, g_a, w_a, wb,
                                           _stream_handle())
    if st != OK:
        raise EwaldError(st, "ewald_energy_forces_batch")
    return [it[3] for it in items]


def energy_forces(pos, q, box_L, alpha, r_c, k_max, precision="fp64", dEdq=False):
    """One-shot evaluation (builds and releases a plan)."""
    with Plan(int(q.shape[0]), box_L, alpha, r_c, k_max, precision, pos.device.index or 0) as p:
        return p.energy_forces(pos, q, True, dEdq)


def _autograd_function():
    import torch

    class EwaldEnergy(torch.autograd.Function):
        """E(pos, q) as a differentiable scalar: the forward runs the energy-only
        path; the backward runs the library's adjoint (recomputing phases and
        S(k)) and returns dL/dpos = -g F and dL/dq = g dE/dq."""

        @staticmethod
        def forward(ctx, pos, q, plan):
            ctx.plan = plan
            ctx.save_for_backward(pos, q)
            return plan.energy(pos.detach().contiguous(), q.detach().contiguous())[0]

        @staticmethod
        def backward(ctx, g):
            pos, q = ctx.saved_tensors
            gp, gq = ctx.plan.energy_backward(pos.detach().contiguous(), q.detach().contiguous(), g,
                                              ctx.needs_input_grad[0], ctx.needs_input_grad[1])
            return gp, gq, None

    return EwaldEnergy


_EwaldEnergy = None


def ewald_energy(pos, q, plan: "Plan"):
    """Differentiable Ewald energy (scalar tensor) for ``plan``."""
    global _EwaldEnergy
    if _EwaldEnergy is None:
        _EwaldEnergy = _autograd_function()
    return _EwaldEnergy.apply(pos, q, plan)


class Server:
    """Request server for many independent systems (``include/ewald_server.h``).

    ``add_system`` registers a system (its plan stays resident); ``submit``
    enqueues one evaluation and returns a ticket at once; ``wait`` returns the
    outputs with the submission and completion times on the server clock
    (``Server.clock()``, the clock of ``time.perf_counter``).  Inputs must be
    complete on the device when submitted (synchronise their producer first);
    the binding keeps the tensors of a request alive until it is waited for.
    """

    def __init__(self, n_streams: int = 4, precision="mixed", device: int = 0, hbm_budget: int = 0,
                 express_cus: bool = False, batching: bool = True):
        lib = _load()
        import torch
        self.device = torch.device("cuda", device)
        prm = ServerParams(int(device), int(n_streams), _precision_code(precision),
                           (SERVER_FLAG_EXPRESS_CUS if express_cus else 0) | (0 if batching else SERVER_FLAG_NO_BATCH),
                           int(hbm_budget))
        h = ctypes.c_void_p()
        st = lib.ewald_server_create(ctypes.byref(prm), ctypes.byref(h))
        if st != OK:
            raise EwaldError(st, "ewald_server_create")
        self._h = h
        self._live = {}
        self._n_max = {}

    @staticmethod
    def clock() -> float:
        return float(_load().ewald_server_clock())

    @property
    def handle(self) -> int:
        if self._h is None:
            raise RuntimeError("server was destroyed")
        return self._h.value

    def add_system(self, n_max: int, box_L: float, alpha: float, r_c: float, k_max: int) -> int:
        prm = make_params(n_max, box_L, alpha, r_c, k_max)
        sid = ctypes.c_int32(-1)
        st = _load().ewald_server_add_system(self.handle, ctypes.byref(prm), ctypes.byref(sid))
        if st != OK:
            raise EwaldError(st, "ewald_server_add_system")
        self._n_max[sid.value] = int(n_max)
        return sid.value

    def remove_system(self, sid: int):
        st = _load().ewald_server_remove_system(self.handle, int(sid))
        if st != OK:
            raise EwaldError(st, "ewald_server_remove_system")
        self._n_max.pop(sid, None)

    def submit(self, sid: int, pos, q, forces: bool = True, dEdq: bool = False, out=None) -> int:
        import torch
        n = int(q.shape[0])
        for name, t, shape in (("pos", pos, (n, 3)), ("q", q, (n,))):
            if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {shape}")
        if out is None:
            e = torch.empty(5, dtype=torch.float64, device=pos.device)
            f = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if forces else None
            g = torch.empty(n, dtype=torch.float64, device=pos.device) if dEdq else None
        else:
            e, f, g = _check_outputs(out, n)
        t = ctypes.c_int64(-1)
        st = _load().ewald_server_submit(self.handle, int(sid), n, pos.data_ptr(), q.data_ptr(), e.data_ptr(),
                                         f.data_ptr() if f is not None else None,
                                         g.data_ptr() if g is not None else None, ctypes.byref(t))
        if st != OK:
            raise EwaldError(st, "ewald_server_submit")
        self._live[t.value] = (pos, q, e, f, g)
        return t.value

    def wait(self, ticket: int):
        """((energy, forces, dEdq), t_submit, t_done) of a request."""
        ts, td = ctypes.c_double(), ctypes.c_double()
        st = _load().ewald_server_wait(self.handle, int(ticket), ctypes.byref(ts), ctypes.byref(td))
        live = self._live.pop(ticket, None)
        if st != OK:
            raise EwaldError(st, "ewald_server_wait")
        return live[2:], ts.value, td.value

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int32(0)
        st = _load().ewald_server_poll(self.handle, int(ticket), ctypes.byref(done))
        if st != OK:
            raise EwaldError(st, "ewald_server_poll")
        return bool(done.value)

    def drain(self):
        st = _load().ewald_server_drain(self.handle)
        if st != OK:
            raise EwaldError(st, "ewald_server_drain")

    def system_status(self, sid: int) -> int:
        return int(_load().ewald_server_system_status(self.handle, int(sid)))

    def stats(self) -> Dict[str, int]:
        out = ServerStats()
        st = _load().ewald_server_get_stats(self.handle, ctypes.byref(out))
        if st != OK:
            raise EwaldError(st, "ewald_server_get_stats")
        return {k: int(getattr(out, k)) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None:
            _load().ewald_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
