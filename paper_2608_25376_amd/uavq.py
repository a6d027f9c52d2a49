"""Thin Python binding over ``libuavq.so`` (the C ABI in ``include/uavq.h``).

Argument marshalling only: every step of the annealing path runs in the
library's HIP kernels.  Device buffers are torch tensors (PyTorch provides
device memory and streams, nothing else).  The library must have been built
(``paper_2608_25376_amd/build.py``); a missing library is an error.
"""
import ctypes as C
import os
import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libuavq.so")

OPEN_PATH = 0x1
DENSE = 0x2
KERNEL_DENSE = 0x1
VARIANT_ROWMASK = 0x10
PERSISTENT = 0x20
GRAPH = 0x40
VARIANT_NOPRODUCER = 0x80
VARIANT_GENERIC = 0x400
STOP_FROZEN = 0x100
REDUCE_AT_END = 0x200
CONCURRENT_CLASSES = 0x800
CHUNK_CLASSES = 9          # sweep kernel classes by ceil(m / 64), 16-bit costs from class 7; m <= 576

OK, EINVAL, ENOMEM, EHIP, ETOOBIG, EINFEASIBLE, EINVARIANT = 0, -1, -2, -3, -4, -5, -6


class UavqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"uavq error {code}: {msg}")
        self.code = code


class _Grid(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("depot", C.c_int32),
                ("nofly", C.POINTER(C.c_uint8)), ("cost_scale", C.c_int32), ("penalty", C.c_int32),
                ("flags", C.c_uint32)]


class _QuboInfo(C.Structure):
    _fields_ = [("m", C.c_int32), ("n_vars", C.c_int32), ("P", C.c_int32), ("w_max", C.c_int32),
                ("c0", C.c_int64), ("closed", C.c_int32), ("has_dense", C.c_int32), ("row_words", C.c_int32),
                ("state_words", C.c_int32)]


class Tune(C.Structure):
    """Launch shape chosen by autotune (per chunk class c = ceil(m/64))."""
    _fields_ = [("waves_per_block", C.c_int32 * 10), ("variant_flags", C.c_uint32), ("trial_ms", C.c_float)]

    def __repr__(self):
        return (f"Tune(waves_per_block={list(self.waves_per_block)[1:]}, variant={self.variant_flags:#x}, "
                f"trial_ms={self.trial_ms:.3f})")


class _Params(C.Structure):
    _fields_ = [("replicas", C.c_int32), ("sweeps", C.c_int32), ("T0", C.c_double), ("T1", C.c_double),
                ("seed", C.c_uint32), ("flags", C.c_uint32), ("waves_per_block", C.c_int32),
                ("tune", C.POINTER(Tune)), ("inst_T", C.POINTER(C.c_double))]


class _PlanInfo(C.Structure):
    _fields_ = [("ws_bytes", C.c_size_t), ("total_replicas", C.c_int64), ("total_state_words", C.c_int64),
                ("n_inst", C.c_int32), ("Dmax", C.c_int32)]


class _Init(C.Structure):
    _fields_ = [("states", C.c_void_p), ("seeded", C.c_void_p), ("start_sweep", C.c_void_p)]


class _Out(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in (
        "final_states", "final_E", "best_E", "best_sweep", "best_states", "accepts", "draws", "inst_best_E",
        "inst_best_replica", "inst_best_sweep", "inst_best_state", "check_E", "attempts")]


EXPORTS = [
    "uavq_last_error", "uavq_version", "uavq_qubo_build", "uavq_qubo_free", "uavq_qubo_info",
    "uavq_qubo_free_cells", "uavq_qubo_costs", "uavq_qubo_export", "uavq_energy_eval",
    "uavq_energy_workspace_bytes", "uavq_energy_eval_dev", "uavq_energy_eval_dev_noalloc", "uavq_decode_path",
    "uavq_schedule",
    "uavq_plan_create", "uavq_plan_free", "uavq_plan_info", "uavq_plan_kernel_name", "uavq_plan_layout",
    "uavq_plan_upload",
    "uavq_anneal_batch", "uavq_anneal_segment", "uavq_anneal_checked", "uavq_plan_set_timing", "uavq_plan_sweep_ms",
    "uavq_autotune",
    "uavq_mlp_param_count", "uavq_mlp_features", "uavq_mlp_workspace_bytes", "uavq_mlp_forward",
    "uavq_mlp_loss_grad", "uavq_mlp_adam", "uavq_quantize_marginals", "uavq_sample_seeds",
    "uavq_pt_ladder", "uavq_pt_exchange", "uavq_pt_exchange_batch",
]

_lib = None


def lib():
    """Load libuavq.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2608_25376_amd/build.py (or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        L.uavq_last_error.restype = C.c_char_p
        L.uavq_version.restype = C.c_int32
        L.uavq_qubo_build.argtypes = [P(_Grid), P(vp)]
        L.uavq_qubo_free.argtypes = [vp]
        L.uavq_qubo_free.restype = None
        L.uavq_qubo_info.argtypes = [vp, P(_QuboInfo)]
        L.uavq_qubo_free_cells.argtypes = [vp, P(C.c_int32)]
        L.uavq_qubo_costs.argtypes = [vp, P(C.c_int32)]
        L.uavq_qubo_export.argtypes = [vp, P(C.c_int32), P(C.c_int32)]
        L.uavq_energy_eval.argtypes = [vp, P(C.c_uint32), C.c_int64, P(C.c_int64)]
        L.uavq_energy_workspace_bytes.argtypes = [vp, P(C.c_size_t)]
        L.uavq_energy_eval_dev.argtypes = [vp, vp, C.c_int64, vp, vp, C.c_size_t, vp]
        L.uavq_energy_eval_dev_noalloc.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.uavq_decode_path.argtypes = [vp, P(C.c_uint32), P(C.c_int32), P(C.c_int64)]
        L.uavq_schedule.argtypes = [C.c_double, C.c_double, C.c_int32, P(C.c_int32), P(C.c_uint32)]
        L.uavq_plan_create.argtypes = [P(vp), C.c_int32, P(C.c_uint32), P(_Params), P(vp)]
        L.uavq_plan_free.argtypes = [vp]
        L.uavq_plan_free.restype = None
        L.uavq_plan_info.argtypes = [vp, P(_PlanInfo)]
        L.uavq_plan_kernel_name.argtypes = [vp, C.c_int32]
        L.uavq_plan_kernel_name.restype = C.c_char_p
        L.uavq_plan_layout.argtypes = [vp, P(C.c_int64), P(C.c_int64)]
        L.uavq_plan_upload.argtypes = [vp, vp, C.c_size_t, vp]
        L.uavq_anneal_batch.argtypes = [vp, vp, C.c_size_t, P(_Init), P(_Out), vp]
        L.uavq_anneal_segment.argtypes = [vp, vp, C.c_size_t, P(_Init), P(_Out), C.c_int32, C.c_int32, C.c_int32, vp]
        L.uavq_anneal_checked.argtypes = [vp, vp, C.c_size_t, P(_Init), P(_Out), C.c_int32, vp, P(C.c_uint64), vp]
        L.uavq_plan_set_timing.argtypes = [vp, C.c_int32]
        L.uavq_plan_sweep_ms.argtypes = [vp, P(C.c_float)]
        L.uavq_autotune.argtypes = [P(vp), C.c_int32, P(C.c_uint32), P(_Params), C.c_int32, C.c_char_p, P(Tune)]
        L.uavq_mlp_param_count.restype = C.c_int
        L.uavq_mlp_features.argtypes = [vp, P(C.c_float)]
        L.uavq_mlp_workspace_bytes.argtypes = [C.c_int32, P(C.c_size_t)]
        L.uavq_mlp_forward.argtypes = [vp, vp, vp, C.c_int32, vp, vp, C.c_size_t, vp]
        L.uavq_mlp_loss_grad.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, C.c_size_t, vp]
        L.uavq_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, vp]
        L.uavq_quantize_marginals.argtypes = [vp, vp, C.c_int32, vp, vp]
        L.uavq_sample_seeds.argtypes = [vp, vp, P(C.c_int64), P(C.c_int32), vp, vp, C.c_size_t, vp]
        L.uavq_pt_ladder.argtypes = [C.c_double, C.c_double, C.c_int32, P(C.c_double), P(C.c_int32), P(C.c_int32),
                                     P(C.c_uint32), C.c_int32]
        L.uavq_pt_exchange.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_uint32, C.c_uint32, C.c_uint32, vp, vp,
                                       C.c_int32, vp, vp, vp, vp]
        L.uavq_pt_exchange_batch.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_uint32, C.c_uint32, vp, vp, vp, vp,
                                             vp, C.c_int32, vp, vp, vp, vp]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise UavqError(rc, lib().uavq_last_error().decode())


def _np_ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _dptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ QUBO ----
class Qubo:
    """Handle returned by qubo_build (library-owned, immutable)."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle)
        info = _QuboInfo()
        _check(lib().uavq_qubo_info(self._h, C.byref(info)))
        self.m, self.n_vars, self.P, self.w_max = info.m, info.n_vars, info.P, info.w_max
        self.c0, self.closed, self.has_dense = info.c0, bool(info.closed), bool(info.has_dense)
        self.row_words, self.state_words = info.row_words, info.state_words

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.uavq_qubo_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def free_cells(self):
        F = np.zeros(self.m, np.int32)
        _check(lib().uavq_qubo_free_cells(self._h, _np_ptr(F, C.c_int32)))
        return F

    def costs(self):
        W = np.zeros((self.m + 1, self.m + 1), np.int32)
        _check(lib().uavq_qubo_costs(self._h, _np_ptr(W, C.c_int32)))
        return W

    def export(self, dense=False):
        b = np.zeros(self.n_vars, np.int32)
        J = np.zeros((self.n_vars, self.n_vars), np.int32) if dense else None
        _check(lib().uavq_qubo_export(self._h, _np_ptr(b, C.c_int32), None if J is None else _np_ptr(J, C.c_int32)))
        return b, J


def qubo_build(rows, cols, nofly=None, depot=0, cost_scale=10, penalty=0, closed=True, dense=False) -> Qubo:
    g = _Grid()
    g.rows, g.cols, g.depot, g.cost_scale, g.penalty = rows, cols, depot, cost_scale, penalty
    g.flags = (0 if closed else OPEN_PATH) | (DENSE if dense else 0)
    nf = None
    if nofly is not None:
        nf = np.ascontiguousarray(nofly, dtype=np.uint8).reshape(-1)
        if nf.size != rows * cols:
            raise ValueError("nofly must have rows*cols entries")
        g.nofly = _np_ptr(nf, C.c_uint8)
    h = C.c_void_p()
    _check(lib().uavq_qubo_build(C.byref(g), C.byref(h)))
    return Qubo(h.value)


# ------------------------------------------------------ state packing ------
def pack_states(x, m):
    """uint8 states [..., m*m] (t-major) -> packed uint32 [..., m*ceil(m/32)]."""
    x = np.asarray(x, np.uint8)
    lead = x.shape[:-1]
    W = (m + 31) // 32
    X = x.reshape(-1, m, m)
    pad = np.zeros((X.shape[0], m, W * 32), np.uint8)
    pad[:, :, :m] = X
    words = np.packbits(pad.reshape(X.shape[0], m, W, 32)[..., ::-1], axis=-1).view(">u4").astype(np.uint32)
    return words.reshape(lead + (m * W,))


def unpack_states(p, m):
    """packed uint32 [..., m*ceil(m/32)] -> uint8 [..., m*m]."""
    p = np.asarray(p, np.uint32)
    lead = p.shape[:-1]
    W = (m + 31) // 32
    P = p.reshape(-1, m, W).astype(">u4").view(np.uint8).reshape(-1, m, W, 4)
    bits = np.unpackbits(P, axis=-1).reshape(-1, m, W, 32)[..., ::-1].reshape(-1, m, W * 32)[:, :, :m]
    return np.ascontiguousarray(bits).reshape(lead + (m * m,))


# --------------------------------------------------------------- energy -----
def energy_eval(q: Qubo, x_packed) -> np.ndarray:
    x = np.ascontiguousarray(x_packed, dtype=np.uint32).reshape(-1, q.state_words)
    E = np.zeros(x.shape[0], np.int64)
    _check(lib().uavq_energy_eval(q.handle, _np_ptr(x, C.c_uint32), x.shape[0], _np_ptr(E, C.c_int64)))
    return E


def energy_eval_dev(q: Qubo, d_states, d_E=None, stream=None):
    import torch
    n = d_states.numel() // q.state_words
    if d_E is None:
        d_E = torch.empty(n, dtype=torch.int64, device=d_states.device)
    nb = C.c_size_t()
    _check(lib().uavq_energy_workspace_bytes(q.handle, C.byref(nb)))
    ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=d_states.device)
    _check(lib().uavq_energy_eval_dev(q.handle, _dptr(d_states), n, _dptr(d_E), _dptr(ws), nb.value,
                                      _stream_handle(stream)))
    return d_E


def energy_eval_dev_noalloc(q: Qubo, d_states, d_E, stream=None):
    """energy_eval on the device with the library's static staging buffer: nothing is
    allocated (``d_E`` is the caller's int64 output of one entry per state)."""
    n = d_states.numel() // q.state_words
    _check(lib().uavq_energy_eval_dev_noalloc(q.handle, _dptr(d_states), n, _dptr(d_E), _stream_handle(stream)))
    return d_E


def decode_path(q: Qubo, x_packed):
    x = np.ascontiguousarray(x_packed, dtype=np.uint32).reshape(-1)
    path = np.zeros(q.m + 2, np.int32)
    cost = C.c_int64()
    rc = lib().uavq_decode_path(q.handle, _np_ptr(x, C.c_uint32), _np_ptr(path, C.c_int32), C.byref(cost))
    if rc == EINFEASIBLE:
        return None, None
    _check(rc)
    return path, int(cost.value)


def schedule(T0, T1, S, table=True):
    dmax = C.c_int32()
    _check(lib().uavq_schedule(T0, T1, S, C.byref(dmax), None))
    if not table:
        return dmax.value, None
    thr = np.zeros((S, dmax.value + 1), np.uint32)
    _check(lib().uavq_schedule(T0, T1, S, C.byref(dmax), _np_ptr(thr, C.c_uint32)))
    return dmax.value, thr


# ------------------------------------------------------------ annealing -----
@dataclass
class AnnealResult:
    final_states: object
    final_E: object
    best_E: object
    best_sweep: object
    best_states: object
    accepts: object
    draws: object
    inst_best_E: object
    inst_best_replica: object
    inst_best_sweep: object
    inst_best_state: object
    attempts: object = None


# outputs that carry a replica across a segment boundary (what a checkpoint holds)
CHECKPOINT_FIELDS = ("final_states", "best_E", "best_sweep", "best_states", "accepts", "draws", "attempts")


def _sync(stream):
    import torch
    if stream is None:
        torch.cuda.synchronize()
    else:
        stream.synchronize()


class Plan:
    """uavq_plan_create + workspace; call ``upload`` once, then ``anneal``."""

    def __init__(self, qubos: Sequence[Qubo], inst_ids: Sequence[int], replicas: int, sweeps: int, T0: float,
                 T1: float, seed: int = 1, dense: bool = False, waves_per_block: int = 0,
                 rowmask: bool = False, persistent: bool = False, graph: bool = False, tune: "Tune" = None,
                 no_producer: bool = False, stop_frozen: bool = False, inst_T=None, reduce_at_end: bool = False,
                 generic_chunk: bool = False, concurrent: bool = False):
        """``inst_T``: optional per-instance schedules, a sequence of (T0_i, T1_i).  ``concurrent``:
        the sweep kernels of different chunk classes run at the same time (UAVQ_CONCURRENT_CLASSES)."""
        self.qubos = list(qubos)
        n = len(self.qubos)
        arr = (C.c_void_p * max(n, 1))(*[q.handle.value for q in self.qubos])
        ids = np.ascontiguousarray(inst_ids, dtype=np.uint32)
        assert ids.size == n
        flags = (KERNEL_DENSE if dense else 0) | (VARIANT_ROWMASK if rowmask else 0)
        flags |= (PERSISTENT if persistent else 0) | (GRAPH if graph else 0)
        flags |= VARIANT_NOPRODUCER if no_producer else 0
        flags |= VARIANT_GENERIC if generic_chunk else 0
        flags |= STOP_FROZEN if stop_frozen else 0
        flags |= REDUCE_AT_END if reduce_at_end else 0
        flags |= CONCURRENT_CLASSES if concurrent else 0
        self._tune = tune
        iT = None
        if inst_T is not None:
            iT = np.ascontiguousarray(inst_T, dtype=np.float64).reshape(-1)
            if iT.size != 2 * n:
                raise ValueError("inst_T needs (T0, T1) for every instance")
        p = _Params(replicas, sweeps, T0, T1, seed, flags, waves_per_block,
                    C.pointer(tune) if tune is not None else None,
                    _np_ptr(iT, C.c_double) if iT is not None else None)
        h = C.c_void_p()
        _check(lib().uavq_plan_create(arr, n, _np_ptr(ids, C.c_uint32), C.byref(p), C.byref(h)))
        self._h = h
        info = _PlanInfo()
        _check(lib().uavq_plan_info(self._h, C.byref(info)))
        self.ws_bytes, self.total_replicas = info.ws_bytes, info.total_replicas
        self.total_state_words, self.n_inst, self.Dmax = info.total_state_words, info.n_inst, info.Dmax
        self.rep_offset = np.zeros(n + 1, np.int64)
        self.state_offset = np.zeros(n + 1, np.int64)
        _check(lib().uavq_plan_layout(self._h, _np_ptr(self.rep_offset, C.c_int64),
                                      _np_ptr(self.state_offset, C.c_int64)))
        self.replicas, self.sweeps = replicas, sweeps
        self.ws = None

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.uavq_plan_free(self._h)
            self._h = None

    def upload(self, device="cuda", stream=None):
        """A device workspace holding the plan's static data; kept as ``self.ws`` (the default
        workspace of ``anneal``) and returned.  Launches that run at the same time need a
        workspace each (persistent and dense launches write into theirs)."""
        import torch
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        if stream is not None:
            torch.cuda.synchronize()
        _check(lib().uavq_plan_upload(self._h, _dptr(self.ws), self.ws_bytes, _stream_handle(stream)))
        return self.ws

    def set_timing(self, enable=True):
        _check(lib().uavq_plan_set_timing(self._h, 1 if enable else 0))

    def kernel_name(self, cls=1):
        """Sweep kernel launched for chunk class cls (1: m <= 64, 2: <= 128, ..., 9: <= 576; fields whose costs
        exceed 255 run in class 7 or above); '' if the class is empty."""
        v = lib().uavq_plan_kernel_name(self._h, int(cls))
        if v is None:
            raise UavqError(-1, lib().uavq_last_error().decode())
        return v.decode()

    def sweep_ms(self):
        """Elapsed ms of the sweep kernels of the last anneal (HIP events on its stream)."""
        v = C.c_float()
        _check(lib().uavq_plan_sweep_ms(self._h, C.byref(v)))
        return float(v.value)

    def alloc_outputs(self, device="cuda"):
        import torch
        R, W = self.total_replicas, self.total_state_words
        inst_words = int(sum(q.state_words for q in self.qubos))
        z = lambda n, dt: torch.zeros(max(n, 1), dtype=dt, device=device)
        return AnnealResult(
            final_states=z(W, torch.int32), final_E=z(R, torch.int64), best_E=z(R, torch.int64),
            best_sweep=z(R, torch.int32), best_states=z(W, torch.int32), accepts=z(R, torch.int64),
            draws=z(R, torch.int64), inst_best_E=z(self.n_inst, torch.int64),
            inst_best_replica=z(self.n_inst, torch.int32), inst_best_sweep=z(self.n_inst, torch.int32),
            inst_best_state=z(inst_words, torch.int32), attempts=z(R, torch.int64))

    def _out_struct(self, out: AnnealResult, check_E=None) -> "_Out":
        return _Out(*[_dptr(check_E) if f == "check_E" else _dptr(getattr(out, f, None)) for f, _ in _Out._fields_])

    def anneal(self, out: Optional[AnnealResult] = None, init_states=None, seeded=None, start_sweep=None,
               check_E=None, stream=None, s_begin: int = 0, s_end: Optional[int] = None,
               resume: bool = False, ws=None) -> AnnealResult:
        """anneal_batch on this plan's workspace (asynchronous on ``stream``).  With a sweep range
        (anneal_segment) only sweeps s_begin .. s_end-1 of the schedule run; ``resume`` continues
        from what ``out`` holds (the outputs of a segment that ended at s_begin, or a restored
        checkpoint).  ``ws``: another uploaded workspace of this plan (default: ``self.ws``)."""
        ws = self.ws if ws is None else ws
        if ws is None:
            raise RuntimeError("Plan.upload() must precede anneal()")
        if out is None:
            if resume:
                raise ValueError("resume needs the outputs of the previous segment")
            out = self.alloc_outputs(ws.device)
        init = _Init(_dptr(init_states), _dptr(seeded), _dptr(start_sweep))
        o = self._out_struct(out, check_E)
        if s_begin == 0 and s_end is None and not resume:
            _check(lib().uavq_anneal_batch(self._h, _dptr(ws), self.ws_bytes, C.byref(init), C.byref(o),
                                           _stream_handle(stream)))
        else:
            _check(lib().uavq_anneal_segment(self._h, _dptr(ws), self.ws_bytes, C.byref(init), C.byref(o),
                                             int(s_begin), int(self.sweeps if s_end is None else s_end),
                                             1 if resume else 0, _stream_handle(stream)))
        return out

    def anneal_checked(self, refresh_every: int, out: Optional[AnnealResult] = None, init_states=None,
                       seeded=None, start_sweep=None, check_E=None, violations=None, stream=None):
        """uavq_anneal_checked: the whole schedule in pieces of ``refresh_every`` sweeps, the
        incrementally kept energies compared with their MFMA recomputation after each piece.
        Returns (outputs, per-replica counts of mismatching pieces, their total); a mismatch is
        reported through the total (the library's UAVQ_EINVARIANT), other errors raise.
        Synchronous."""
        import torch
        if self.ws is None:
            raise RuntimeError("Plan.upload() must precede anneal_checked()")
        dev = self.ws.device
        out = self.alloc_outputs(dev) if out is None else out
        R = max(self.total_replicas, 1)
        check_E = torch.zeros(R, dtype=torch.int64, device=dev) if check_E is None else check_E
        violations = torch.zeros(R, dtype=torch.int32, device=dev) if violations is None else violations
        init = _Init(_dptr(init_states), _dptr(seeded), _dptr(start_sweep))
        o = self._out_struct(out, check_E)
        n = C.c_uint64()
        rc = lib().uavq_anneal_checked(self._h, _dptr(self.ws), self.ws_bytes, C.byref(init), C.byref(o),
                                       int(refresh_every), _dptr(violations), C.byref(n), _stream_handle(stream))
        if rc != EINVARIANT:
            _check(rc)
        return out, violations, int(n.value)

    def checkpoint(self, out: AnnealResult) -> dict:
        """Copy of everything a resumed segment reads (device tensors, on the stream's device)."""
        return {f: getattr(out, f).clone() for f in CHECKPOINT_FIELDS if getattr(out, f, None) is not None}

    def restore(self, ckpt: dict, out: Optional[AnnealResult] = None) -> AnnealResult:
        """Write a checkpoint into output buffers (fresh ones if ``out`` is None); then resume with
        ``anneal(out=out, s_begin=<sweeps done>, resume=True)``."""
        if out is None:
            out = self.alloc_outputs(self.ws.device)
        for f in CHECKPOINT_FIELDS:
            if f in ckpt and getattr(out, f, None) is not None:
                getattr(out, f).copy_(ckpt[f])
        return out

    def anneal_time_limited(self, budget_ms: float, segment_sweeps: Optional[int] = None,
                            out: Optional[AnnealResult] = None, init_states=None, seeded=None, start_sweep=None,
                            stream=None):
        """Time-limit mode: run the schedule in segments of ``segment_sweeps`` sweeps and stop at
        the first segment boundary after which the next segment would overrun ``budget_ms`` of wall
        time (predicted from the time per sweep so far).  The first segment always runs.  Returns
        (outputs, sweeps completed); the outputs equal those of ``anneal(s_end=<sweeps completed>)``
        bit for bit, so only the stopping point depends on timing."""
        S = self.sweeps
        seg = int(segment_sweeps) if segment_sweeps else max(1, S // 20)
        if seg < 1:
            raise ValueError("segment_sweeps must be positive")
        t0 = time.perf_counter()
        done = min(seg, S)
        out = self.anneal(out=out, init_states=init_states, seeded=seeded, start_sweep=start_sweep,
                          stream=stream, s_begin=0, s_end=done)
        _sync(stream)
        while done < S:
            spent = (time.perf_counter() - t0) * 1e3
            nxt = min(done + seg, S)
            if spent + spent / done * (nxt - done) > budget_ms:
                break
            self.anneal(out=out, start_sweep=start_sweep, stream=stream, s_begin=done, s_end=nxt, resume=True)
            _sync(stream)
            done = nxt
        return out, done


def anneal_batch(plan: Plan, **kw) -> AnnealResult:
    return plan.anneal(**kw)


def autotune(qubos: Sequence[Qubo], inst_ids: Sequence[int], replicas: int, sweeps: int, T0: float, T1: float,
             seed: int = 1, persistent: bool = False, trial_sweeps: int = 64, cache: Optional[str] = None) -> Tune:
    """uavq_autotune: fastest launch shape for these instances (never changes results)."""
    n = len(qubos)
    arr = (C.c_void_p * max(n, 1))(*[q.handle.value for q in qubos])
    ids = np.ascontiguousarray(inst_ids, dtype=np.uint32)
    p = _Params(replicas, sweeps, T0, T1, seed, PERSISTENT if persistent else 0, 0, None)
    t = Tune()
    _check(lib().uavq_autotune(arr, n, _np_ptr(ids, C.c_uint32), C.byref(p), trial_sweeps,
                               cache.encode() if cache else None, C.byref(t)))
    return t


# ------------------------------------------------------------ warm start ----
def mlp_param_count() -> int:
    return int(lib().uavq_mlp_param_count())


def mlp_features(q: Qubo) -> np.ndarray:
    X = np.zeros((q.m, 16), np.float32)
    _check(lib().uavq_mlp_features(q.handle, _np_ptr(X, C.c_float)))
    return X


class Mlp:
    """Parameters (fp32 master, device), Adam moments and the step counter of
    the warm-start network; every computation runs in the library's kernels."""

    def __init__(self, params, device="cuda"):
        import torch
        p = torch.as_tensor(np.asarray(params, np.float32)).to(device)
        assert p.numel() == mlp_param_count()
        self.params = p.contiguous()
        self.m1 = torch.zeros_like(self.params)
        self.m2 = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.step_count = 0
        self._ws = None

    def _workspace(self, rows, device):
        import torch
        nb = C.c_size_t()
        _check(lib().uavq_mlp_workspace_bytes(rows, C.byref(nb)))
        if self._ws is None or self._ws.numel() < nb.value:
            self._ws = torch.empty(nb.value, dtype=torch.uint8, device=device)
        return self._ws, nb.value

    def forward(self, X, msteps, stream=None):
        import torch
        rows = X.shape[0]
        probs = torch.empty((rows, 128), dtype=torch.float32, device=X.device)
        ws, nb = self._workspace(rows, X.device)
        _check(lib().uavq_mlp_forward(_dptr(self.params), _dptr(X), _dptr(msteps), rows, _dptr(probs), _dptr(ws), nb,
                                      _stream_handle(stream)))
        return probs

    def loss_grad(self, X, msteps, labels, stream=None):
        rows = X.shape[0]
        ws, nb = self._workspace(rows, X.device)
        _check(lib().uavq_mlp_loss_grad(_dptr(self.params), _dptr(X), _dptr(msteps), _dptr(labels), rows,
                                        _dptr(self.grad), _dptr(self.loss), _dptr(ws), nb, _stream_handle(stream)))
        return self.loss, self.grad

    def adam(self, lr=1e-3, stream=None):
        self.step_count += 1
        _check(lib().uavq_mlp_adam(_dptr(self.params), _dptr(self.m1), _dptr(self.m2), _dptr(self.grad),
                                   self.step_count, lr, _stream_handle(stream)))

    def train_step(self, X, msteps, labels, lr=1e-3, stream=None):
        loss, _ = self.loss_grad(X, msteps, labels, stream)
        self.adam(lr, stream)
        return loss


def quantize_marginals(probs, msteps, stream=None):
    import torch
    rows = probs.shape[0]
    q = torch.empty((rows, 128), dtype=torch.int16, device=probs.device)
    _check(lib().uavq_quantize_marginals(_dptr(probs), _dptr(msteps), rows, _dptr(q), _stream_handle(stream)))
    return q


def sample_seeds(plan: "Plan", q, q_row_off, n_seeded, states, stream=None):
    """Write sampled permutations for replicas 0..n_seeded[i]-1 of every
    instance into ``states`` (plan layout)."""
    import torch
    qo = np.ascontiguousarray(q_row_off, dtype=np.int64)
    ns = np.ascontiguousarray(n_seeded, dtype=np.int32)
    scratch = torch.empty(32 * max(len(ns), 1) + 64, dtype=torch.uint8, device=q.device)
    torch.cuda.synchronize()
    _check(lib().uavq_sample_seeds(plan._h, _dptr(q), _np_ptr(qo, C.c_int64), _np_ptr(ns, C.c_int32), _dptr(states),
                                   _dptr(scratch), scratch.numel(), _stream_handle(stream)))


# ------------------------------------------------------- replica exchange --
def pt_ladder(T_hot: float, T_cold: float, K: int):
    """(T[K], DX[K-1], xthr[K-1][stride]) of the tempering ladder (uavq_pt_ladder)."""
    T = np.zeros(K, np.float64)
    DX = np.zeros(max(K - 1, 1), np.int32)
    mx = C.c_int32()
    _check(lib().uavq_pt_ladder(T_hot, T_cold, K, _np_ptr(T, C.c_double), _np_ptr(DX, C.c_int32), C.byref(mx),
                                None, 0))
    stride = mx.value + 1
    xthr = np.zeros((max(K - 1, 1), stride), np.uint32)
    _check(lib().uavq_pt_ladder(T_hot, T_cold, K, _np_ptr(T, C.c_double), _np_ptr(DX, C.c_int32), C.byref(mx),
                                _np_ptr(xthr, C.c_uint32), stride))
    return T, DX[:K - 1].copy(), xthr[:K - 1].copy()


def pt_exchange(rnd: int, seed: int, inst_id: int, d_DX, d_xthr, states, E, swaps=None, stream=None):
    """One exchange round (uavq_pt_exchange) on device tensors: states int32
    [K, R, words], E int64 [K, R], d_DX int32 [K-1], d_xthr uint32 [K-1, stride]
    (held as int32), swaps int64 [K-1] or None."""
    K, R, W = states.shape
    assert states.is_contiguous() and E.is_contiguous() and tuple(E.shape) == (K, R)
    assert d_xthr.is_contiguous() and d_DX.numel() >= K - 1 and d_xthr.shape[0] >= K - 1
    assert swaps is None or swaps.numel() >= K - 1
    _check(lib().uavq_pt_exchange(K, R, W, rnd & 0xFFFFFFFF, seed & 0xFFFFFFFF, inst_id & 0xFFFFFFFF,
                                  _dptr(d_DX), _dptr(d_xthr), int(d_xthr.shape[1]), _dptr(states), _dptr(E),
                                  _dptr(swaps), _stream_handle(stream)))


class ParallelTempering:
    """Parallel tempering on one instance: K slots of R chains each, run as one
    plan of K instances (the same QUBO, instance ids inst_id + k, the constant
    schedule T_k each), so every segment is one launch for all slots.  The
    slots sweep ``interval`` sweeps at a time (anneal_segment) and, between
    segments, neighbouring slots exchange states (uavq_pt_exchange, rounds
    0, 1, ...).  Every step runs in the library's kernels.  The slots' draws
    are addressed by the ids inst_id .. inst_id + K - 1: give chain sets that
    must be independent disjoint id ranges."""

    def __init__(self, q: Qubo, inst_id: int, K: int, replicas: int, sweeps: int, T_hot: float, T_cold: float,
                 seed: int = 1, interval: int = 1, **plan_kw):
        import torch
        if interval < 1:
            raise ValueError("interval must be >= 1")
        self.q, self.inst_id, self.K, self.R, self.S = q, int(inst_id), int(K), int(replicas), int(sweeps)
        self.seed, self.interval = int(seed), int(interval)
        self.T, DX, xthr = pt_ladder(T_hot, T_cold, K)
        self.plan = Plan([q] * K, [(inst_id + k) & 0xFFFFFFFF for k in range(K)], replicas, sweeps, T_hot, T_hot,
                         seed, inst_T=[(float(t), float(t)) for t in self.T], reduce_at_end=True, **plan_kw)
        self.plan.upload()
        self.d_DX = torch.from_numpy(np.ascontiguousarray(DX if K > 1 else np.zeros(1, np.int32))).cuda()
        xt = xthr if K > 1 else np.zeros((1, 2), np.uint32)
        self.d_xthr = torch.from_numpy(np.ascontiguousarray(xt).view(np.int32)).cuda()

    def run(self, stream=None) -> dict:
        """The whole schedule.  Returns per-slot views of the plan's outputs
        (states and best_states [K, R, words], the others [K, R]; inst_best_*
        [K]), the swaps per pair [K-1] and the number of exchange rounds."""
        import torch
        K, R, W = self.K, self.R, self.q.state_words
        out = self.plan.alloc_outputs()
        states, E = out.final_states.view(K, R, W), out.final_E.view(K, R)
        swaps = torch.zeros(max(K - 1, 1), dtype=torch.int64, device="cuda")
        b, rnd = 0, 0
        while b < self.S:
            end = min(b + self.interval, self.S)
            self.plan.anneal(out=out, s_begin=b, s_end=end, resume=b > 0, stream=stream)
            if end < self.S and K > 1:
                pt_exchange(rnd, self.seed, self.inst_id, self.d_DX, self.d_xthr, states, E, swaps, stream=stream)
                rnd += 1
            b = end
        return {"out": out, "states": states, "E": E, "best_E": out.best_E.view(K, R),
                "best_sweep": out.best_sweep.view(K, R), "best_states": out.best_states.view(K, R, W),
                "accepts": out.accepts.view(K, R), "draws": out.draws.view(K, R), "inst_best_E": out.inst_best_E,
                "inst_best_state": out.inst_best_state.view(K, W), "swaps": swaps[:K - 1], "rounds": rnd}


class ParallelTemperingBatch:
    """Parallel tempering of a batch of fields in one plan: field i has K slots
    of R chains on the same ladder (instances i*K .. i*K + K - 1 of the plan,
    instance ids inst_ids[i] + k, the constant schedule T_k), and one
    uavq_pt_exchange_batch launch exchanges every field's pairs.  Field i's
    outputs equal those of ParallelTempering(q_i, inst_ids[i], ...).  The id
    ranges inst_ids[i] .. inst_ids[i] + K - 1 must not overlap."""

    def __init__(self, qs: Sequence[Qubo], inst_ids: Sequence[int], K: int, replicas: int, sweeps: int,
                 T_hot: float, T_cold: float, seed: int = 1, interval: int = 1, **plan_kw):
        import torch
        if interval < 1:
            raise ValueError("interval must be >= 1")
        ids = [int(v) for v in inst_ids]
        if len(ids) != len(qs):
            raise ValueError("one instance id per field")
        spans = sorted((v, v + K - 1) for v in ids)
        if any(b[0] <= a[1] for a, b in zip(spans, spans[1:])):
            raise ValueError("the id ranges inst_ids[i] .. inst_ids[i] + K - 1 overlap")
        self.qs, self.ids, self.K, self.R, self.S = list(qs), ids, int(K), int(replicas), int(sweeps)
        self.seed, self.interval = int(seed), int(interval)
        self.T, DX, xthr = pt_ladder(T_hot, T_cold, K)
        n = len(self.qs)
        self.plan = Plan([q for q in self.qs for _ in range(K)], [(v + k) & 0xFFFFFFFF for v in ids for k in range(K)],
                         replicas, sweeps, T_hot, T_hot, seed,
                         inst_T=[(float(t), float(t)) for _ in range(n) for t in self.T], reduce_at_end=True, **plan_kw)
        self.plan.upload()
        self.d_DX = torch.from_numpy(np.ascontiguousarray(DX if K > 1 else np.zeros(1, np.int32))).cuda()
        xt = xthr if K > 1 else np.zeros((1, 2), np.uint32)
        self.d_xthr = torch.from_numpy(np.ascontiguousarray(xt).view(np.int32)).cuda()
        self.state_off = [int(self.plan.state_offset[i * K]) for i in range(n)]
        self.d_state_off = torch.tensor(self.state_off, dtype=torch.int64, device="cuda")
        self.d_words = torch.tensor([q.state_words for q in self.qs], dtype=torch.int32, device="cuda")
        self.d_inst = torch.from_numpy(np.array(ids, dtype=np.uint32).view(np.int32)).cuda()

    def run(self, stream=None) -> list:
        """The whole schedule; returns one dict per field, shaped like
        ParallelTempering.run's (views of the plan's outputs)."""
        import torch
        K, R, n = self.K, self.R, len(self.qs)
        out = self.plan.alloc_outputs()
        swaps = torch.zeros(n * max(K - 1, 1), dtype=torch.int64, device="cuda")
        b, rnd = 0, 0
        while b < self.S:
            end = min(b + self.interval, self.S)
            self.plan.anneal(out=out, s_begin=b, s_end=end, resume=b > 0, stream=stream)
            if end < self.S and K > 1:
                _check(lib().uavq_pt_exchange_batch(n, K, R, rnd & 0xFFFFFFFF, self.seed & 0xFFFFFFFF,
                                                    _dptr(self.d_state_off), _dptr(self.d_words), _dptr(self.d_inst),
                                                    _dptr(self.d_DX), _dptr(self.d_xthr), int(self.d_xthr.shape[1]),
                                                    _dptr(out.final_states), _dptr(out.final_E), _dptr(swaps),
                                                    _stream_handle(stream)))
                rnd += 1
            b = end
        res = []
        for i, q in enumerate(self.qs):
            W, o = q.state_words, self.state_off[i]
            rs = slice(i * K * R, (i + 1) * K * R)
            res.append({"states": out.final_states[o:o + K * R * W].view(K, R, W), "E": out.final_E[rs].view(K, R),
                        "best_E": out.best_E[rs].view(K, R), "best_sweep": out.best_sweep[rs].view(K, R),
                        "best_states": out.best_states[o:o + K * R * W].view(K, R, W),
                        "accepts": out.accepts[rs].view(K, R), "draws": out.draws[rs].view(K, R),
                        "inst_best_E": out.inst_best_E[i * K:(i + 1) * K],
                        "swaps": swaps.view(n, max(K - 1, 1))[i, :K - 1], "rounds": rnd})
        return res
