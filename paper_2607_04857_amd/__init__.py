"""MI355X exhaustive dense-QUBO solver: thin Python binding of ``libqubo_mi355x.so``.

Every step of a solve runs inside the HIP library (see ``include/qubo.h``);
this module only marshals arguments.  There is no CPU fallback: if the
library is missing, every call raises ``QuboLibraryMissing``.

A process that uses torch's GPU support as well should import torch before
the first call here: torch ships its own HIP runtime, and when this library
has already brought up the system one, torch finds no device.

Conventions (paper Sec. I and II-B): E(x) = sum_{i,j} Q_ij x_i x_j; a state
is its row ``index`` in the lexicographic matrix U_N (x_0 is the most
significant bit); the answer is the minimum energy with the lowest index.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqubo_mi355x.so")

QUBO_INT32, QUBO_FP32 = 0, 1
STATUS = {0: "QUBO_OK", -1: "QUBO_EINVAL", -2: "QUBO_EOVERFLOW", -3: "QUBO_ENONFINITE",
          -4: "QUBO_ENOMEM", -5: "QUBO_EDEVICE", -6: "QUBO_EAGAIN", -7: "QUBO_EINTERNAL"}


class QuboLibraryMissing(RuntimeError):
    pass


class QuboError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class _State(ctypes.Structure):
    _fields_ = [("energy_i", ctypes.c_int64), ("energy", ctypes.c_double),
                ("index", ctypes.c_uint64)]


class _Result(ctypes.Structure):
    _fields_ = [("best", _State), ("tol", ctypes.c_double), ("p", ctypes.c_int),
                ("A", ctypes.c_int), ("B", ctypes.c_int), ("L", ctypes.c_int),
                ("tier", ctypes.c_int), ("vgpr_levels", ctypes.c_int), ("states", ctypes.c_uint64),
                ("kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int), ("L", ctypes.c_int), ("tier", ctypes.c_int),
                ("waves_per_cu", ctypes.c_int), ("vgpr_levels", ctypes.c_int),
                ("item_first", ctypes.c_int), ("item_count", ctypes.c_int),
                ("reserved", ctypes.c_int)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("A", ctypes.c_int), ("B", ctypes.c_int),
                ("L", ctypes.c_int), ("tier", ctypes.c_int), ("direct", ctypes.c_int),
                ("vgpr_levels", ctypes.c_int), ("p", ctypes.c_int), ("eps_q", ctypes.c_double), ("sum_abs_t", ctypes.c_int64),
                ("items", ctypes.c_uint64), ("pack_shift", ctypes.c_int), ("reserved", ctypes.c_int)]


class _Checkpoint(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("dtype", ctypes.c_int), ("A", ctypes.c_int),
                ("B", ctypes.c_int), ("L", ctypes.c_int), ("tier", ctypes.c_int),
                ("vgpr_levels", ctypes.c_int), ("q_hash", ctypes.c_uint64),
                ("items", ctypes.c_uint64), ("next_item", ctypes.c_uint64), ("found", ctypes.c_int),
                ("best", _State), ("p", ctypes.c_int), ("tol", ctypes.c_double),
                ("walk_ms", ctypes.c_double)]


class _TuneEntry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("dtype", ctypes.c_int), ("B", ctypes.c_int),
                ("L", ctypes.c_int), ("tier", ctypes.c_int), ("vgpr_levels", ctypes.c_int),
                ("walk_ms", ctypes.c_double), ("scope", ctypes.c_int)]


# name -> (restype, argtypes); mirrors include/qubo.h
_VP, _I, _U64P = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)
_SIGS = {
    "qubo_solve": (_I, [_VP, _I, _I, _I, ctypes.POINTER(_Result), ctypes.POINTER(_State)]),
    "qubo_solve_ex": (_I, [_VP, _I, _I, _I, ctypes.POINTER(_Options), ctypes.POINTER(_Result),
                           ctypes.POINTER(_State)]),
    "qubo_solve_device": (_I, [_VP, _I, _I, _I, _VP, ctypes.POINTER(_Result),
                               ctypes.POINTER(_State)]),
    "qubo_solve_noalloc": (_I, [_VP, _I, _I, _VP, ctypes.POINTER(_Result)]),
    "qubo_reduce_outer": (_I, [_VP, _I, _I, ctypes.c_uint64, _VP, ctypes.POINTER(ctypes.c_int64)]),
    "qubo_solve_outer": (_I, [_VP, _I, _I, _I, ctypes.POINTER(_Result)]),
    "qubo_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "qubo_solve_batch": (_I, [_I, ctypes.POINTER(_VP), ctypes.POINTER(_I), ctypes.POINTER(_I),
                              ctypes.POINTER(_Result)]),
    "qubo_batch_create": (_I, [_I, ctypes.POINTER(_VP), ctypes.POINTER(_I), ctypes.POINTER(_I),
                               ctypes.POINTER(_Options), ctypes.POINTER(_VP)]),
    "qubo_batch_run": (_I, [_VP, _VP]),
    "qubo_batch_results": (_I, [_VP, ctypes.POINTER(_Result)]),
    "qubo_batch_stats": (_I, [_VP, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)]),
    "qubo_batch_destroy": (None, [_VP]),
    "qubo_server_create": (_I, [ctypes.c_size_t, _I, ctypes.POINTER(_VP)]),
    "qubo_server_submit": (_I, [_VP, _VP, _I, _I, _U64P]),
    "qubo_server_poll": (_I, [_VP, ctypes.c_uint64, ctypes.POINTER(_Result)]),
    "qubo_server_wait": (_I, [_VP, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(_Result)]),
    "qubo_server_stats": (_I, [_VP, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "qubo_server_info": (_I, [_VP, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                              ctypes.POINTER(_I), _U64P]),
    "qubo_server_destroy": (None, [_VP]),
    "qubo_plan_info": (_I, [_VP, _I, _I, ctypes.POINTER(_Options), ctypes.POINTER(_PlanInfo),
                            ctypes.POINTER(ctypes.c_int32)]),
    "qubo_solve_checkpointed": (_I, [_VP, _I, _I, ctypes.POINTER(_Options), ctypes.c_uint64, _I,
                                     ctypes.c_char_p, ctypes.POINTER(_Result)]),
    "qubo_checkpoint_info": (_I, [ctypes.c_char_p, ctypes.POINTER(_Checkpoint)]),
    "qubo_probe_valu": (_I, [_I, _I, _I, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double)]),
    "qubo_autotune": (_I, [_I, _I, _I, _I, ctypes.c_char_p, ctypes.POINTER(_TuneEntry), _I,
                           ctypes.POINTER(_I)]),
    "qubo_autotune_batch": (_I, [_I, _I, _I, _I, ctypes.c_char_p, ctypes.POINTER(_TuneEntry), _I,
                                 ctypes.POINTER(_I)]),
    "qubo_tune_load": (_I, [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(_I)]),
    "qubo_tune_save": (_I, [ctypes.c_char_p, ctypes.c_char_p]),
    "qubo_tune_set": (_I, [ctypes.POINTER(_TuneEntry), _I]),
    "qubo_tune_lookup": (_I, [_I, _I, _I, ctypes.POINTER(_TuneEntry)]),
    "qubo_tune_clear": (None, []),
    "qubo_device_key": (_I, [ctypes.c_char_p, _I]),
    "qubo_last_error": (ctypes.c_char_p, []),
    "qubo_version": (ctypes.c_char_p, []),
}
EXPORTS = tuple(_SIGS)

_lib = None


def lib() -> ctypes.CDLL:
    """Load the HIP library (raises QuboLibraryMissing when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise QuboLibraryMissing(
            f"{LIB_PATH} is missing: build it with `python -m paper_2607_04857_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise QuboError(status, lib().qubo_last_error().decode(errors="replace"))


@dataclass
class Result:
    energy: float          # exact for int32; float64 rescore for fp32
    energy_i: int          # exact integer energy (scaled by 2^p for fp32)
    index: int             # U_N row of the argmin (lowest index among ties)
    n: int
    tol: float
    p: int
    A: int
    B: int
    L: int
    tier: int
    vgpr_levels: int
    states: int
    kernel_ms: float
    total_ms: float

    @property
    def x(self) -> np.ndarray:
        return np.array([(self.index >> (self.n - 1 - i)) & 1 for i in range(self.n)],
                        dtype=np.int8)


def _result(r: _Result, n: int) -> Result:
    return Result(energy=r.best.energy, energy_i=r.best.energy_i, index=r.best.index, n=n,
                  tol=r.tol, p=r.p, A=r.A, B=r.B, L=r.L, tier=r.tier, vgpr_levels=r.vgpr_levels,
                  states=r.states,
                  kernel_ms=r.kernel_ms, total_ms=r.total_ms)


def _as_q(Q):
    Q = np.asarray(Q)
    if Q.ndim != 2 or Q.shape[0] != Q.shape[1]:
        raise ValueError("Q must be a square matrix")
    if Q.dtype == np.float32:
        return np.ascontiguousarray(Q), QUBO_FP32
    if Q.dtype.kind in "iu":
        if Q.size and (Q.min() < -2**31 or Q.max() > 2**31 - 1):
            raise ValueError("integer Q must fit int32")
        return np.ascontiguousarray(Q, dtype=np.int32), QUBO_INT32
    raise TypeError("Q must be int32 or float32")


def _options(B=0, L=0, tier=0, waves_per_cu=0, vgpr_levels=0, item_first=0,
             item_count=0) -> _Options:
    o = _Options()
    o.B, o.L, o.tier, o.waves_per_cu = int(B), int(L), int(tier), int(waves_per_cu)
    o.vgpr_levels = int(vgpr_levels)
    o.item_first, o.item_count = int(item_first), int(item_count)
    return o


def solve(Q, k: int = 1, *, B: int = 0, L: int = 0, tier: int = 0, waves_per_cu: int = 0,
          vgpr_levels: int = 0, item_first: int = 0, item_count: int = 0):
    """Minimise E(x) for a host matrix.  k > 1 also returns the k smallest (E, index) pairs.
    item_first/item_count restrict the walk to those work items (see qubo_options_t)."""
    Qc, dt = _as_q(Q)
    n = Qc.shape[0]
    out = _Result()
    top = (_State * k)() if k > 1 else None
    opt = _options(B, L, tier, waves_per_cu, vgpr_levels, item_first, item_count)
    _check(lib().qubo_solve_ex(Qc.ctypes.data, n, dt, int(k), ctypes.byref(opt),
                               ctypes.byref(out), top))
    res = _result(out, n)
    if k > 1:
        pairs = [(t.energy if dt == QUBO_FP32 else t.energy_i, int(t.index)) for t in top]
        return res, pairs
    return res


def solve_device(Qt, k: int = 1, stream=None):
    """Solve a QUBO held in a torch CUDA tensor (int32 or float32), ordered on ``stream``."""
    import torch
    if not Qt.is_cuda or Qt.dim() != 2 or Qt.shape[0] != Qt.shape[1]:
        raise ValueError("Qt must be a square CUDA tensor")
    if Qt.dtype == torch.float32:
        dt = QUBO_FP32
    elif Qt.dtype == torch.int32:
        dt = QUBO_INT32
    else:
        raise TypeError("Qt must be int32 or float32")
    Qt = Qt.contiguous()
    s = stream if stream is not None else torch.cuda.current_stream(Qt.device)
    out = _Result()
    top = (_State * k)() if k > 1 else None
    with torch.cuda.device(Qt.device):
        _check(lib().qubo_solve_device(ctypes.c_void_p(Qt.data_ptr()), Qt.shape[0], dt, int(k),
                                       ctypes.c_void_p(s.cuda_stream), ctypes.byref(out), top))
    res = _result(out, Qt.shape[0])
    if k > 1:
        pairs = [(t.energy if dt == QUBO_FP32 else t.energy_i, int(t.index)) for t in top]
        return res, pairs
    return res


def reduce_outer(Q, k: int, xf: int):
    """Fix the first k variables to the bits of xf (the index's top k bits):
    returns (Qr, c), the int32 QUBO of the other n - k variables and the
    constant, with E(xf, x_r) = c + E_Qr(x_r)."""
    Qc, dt = _as_q(Q)
    if dt != QUBO_INT32:
        raise TypeError("reduce_outer takes an int32 matrix")
    n = Qc.shape[0]
    Qr = np.zeros((max(n - int(k), 0),) * 2, dtype=np.int32)
    c = ctypes.c_int64()
    _check(lib().qubo_reduce_outer(Qc.ctypes.data, n, int(k), ctypes.c_uint64(int(xf)),
                                   Qr.ctypes.data, ctypes.byref(c)))
    return Qr, c.value


def solve_outer(Q, k: int) -> Result:
    """Solve an int32 QUBO of up to 64 variables as the batch of its 2^k
    outer-bit reductions."""
    Qc, dt = _as_q(Q)
    n = Qc.shape[0]
    out = _Result()
    _check(lib().qubo_solve_outer(Qc.ctypes.data, n, dt, int(k), ctypes.byref(out)))
    return _result(out, n)


def solve_noalloc(Q, stream=None) -> Result:
    """Best state of a host matrix through ``qubo_solve_noalloc`` (no device
    allocation: the library's per-device scratch array holds the job)."""
    Qc, dt = _as_q(Q)
    out = _Result()
    s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(lib().qubo_solve_noalloc(Qc.ctypes.data, Qc.shape[0], dt, s, ctypes.byref(out)))
    return _result(out, Qc.shape[0])


def noalloc_scratch_bytes() -> int:
    return int(lib().qubo_noalloc_scratch_bytes())


def _batch_args(Qs: Sequence):
    mats = [_as_q(Q) for Q in Qs]
    cnt = len(mats)
    ptrs = (_VP * cnt)(*[m.ctypes.data for m, _ in mats])
    ns = (_I * cnt)(*[m.shape[0] for m, _ in mats])
    dts = (_I * cnt)(*[dt for _, dt in mats])
    return mats, cnt, ptrs, ns, dts


class Batch:
    """Plan, allocate and graph-capture a batch once; ``run()`` replays it."""

    def __init__(self, Qs: Sequence, *, B: int = 0, L: int = 0, tier: int = 0,
                 waves_per_cu: int = 0, vgpr_levels: int = 0):
        self._mats, self.count, ptrs, ns, dts = _batch_args(Qs)
        self._ns = [m.shape[0] for m, _ in self._mats]
        self._h = _VP()
        opt = _options(B, L, tier, waves_per_cu, vgpr_levels)
        _check(lib().qubo_batch_create(self.count, ptrs, ns, dts, ctypes.byref(opt),
                                       ctypes.byref(self._h)))

    def run(self, stream=None):
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(lib().qubo_batch_run(self._h, s))

    def results(self) -> List[Result]:
        out = (_Result * self.count)()
        _check(lib().qubo_batch_results(self._h, out))
        return [_result(out[i], self._ns[i]) for i in range(self.count)]

    def stats(self):
        st, ms = ctypes.c_double(), ctypes.c_double()
        _check(lib().qubo_batch_stats(self._h, ctypes.byref(st), ctypes.byref(ms)))
        return st.value, ms.value

    def close(self):
        if self._h:
            lib().qubo_batch_destroy(self._h)
            self._h = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(Qs: Sequence) -> List[Result]:
    mats, cnt, ptrs, ns, dts = _batch_args(Qs)
    out = (_Result * cnt)()
    _check(lib().qubo_solve_batch(cnt, ptrs, ns, dts, out))
    return [_result(out[i], mats[i][0].shape[0]) for i in range(cnt)]


class Server:
    """Continuous-batching server (see include/qubo.h)."""

    def __init__(self, mem_budget_bytes: int = 1 << 30, max_slots: int = 256):
        self._h = _VP()
        _check(lib().qubo_server_create(int(mem_budget_bytes), int(max_slots),
                                        ctypes.byref(self._h)))
        self._n = {}

    def submit(self, Q) -> int:
        Qc, dt = _as_q(Q)
        t = ctypes.c_uint64()
        _check(lib().qubo_server_submit(self._h, Qc.ctypes.data, Qc.shape[0], dt, ctypes.byref(t)))
        self._n[t.value] = Qc.shape[0]
        return t.value

    def poll(self, ticket: int) -> Optional[Result]:
        out = _Result()
        st = lib().qubo_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(out))
        if st == -6:
            return None
        _check(st)
        return _result(out, self._n[ticket])

    def wait(self, ticket: int, timeout_ms: float = 60000.0) -> Optional[Result]:
        out = _Result()
        st = lib().qubo_server_wait(self._h, ctypes.c_uint64(ticket), float(timeout_ms),
                                    ctypes.byref(out))
        if st == -6:
            return None
        _check(st)
        return _result(out, self._n[ticket])

    def stats(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().qubo_server_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"p50_ms": a.value, "p99_ms": b.value, "states_per_s": c.value}

    def info(self):
        a, b, c, d = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int(), ctypes.c_uint64()
        _check(lib().qubo_server_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                      ctypes.byref(d)))
        return {"mem_in_use": a.value, "mem_peak": b.value, "active_peak": c.value,
                "ticks": d.value}

    def close(self):
        if self._h:
            lib().qubo_server_destroy(self._h)
            self._h = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_info(Q, *, B: int = 0, L: int = 0, tier: int = 0, vgpr_levels: int = 0,
              item_first: int = 0, item_count: int = 0):
    """Host-only plan of a solve (no GPU): split, items, scale; plus the folded T."""
    Qc, dt = _as_q(Q)
    n = Qc.shape[0]
    info = _PlanInfo()
    T = np.zeros((n, n), dtype=np.int32)
    opt = _options(B, L, tier, vgpr_levels=vgpr_levels, item_first=item_first,
                   item_count=item_count)
    _check(lib().qubo_plan_info(Qc.ctypes.data, n, dt, ctypes.byref(opt), ctypes.byref(info),
                                T.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    d = {f: getattr(info, f) for f, _ in _PlanInfo._fields_}
    d["T"] = T
    return d


def solve_checkpointed(Q, path: str, *, items_per_slice: int = 0, max_slices: int = 0,
                       B: int = 0, L: int = 0, tier: int = 0, waves_per_cu: int = 0,
                       vgpr_levels: int = 0) -> Optional[Result]:
    """Solve in slices of work items with a resumable checkpoint at ``path``
    (see ``qubo_solve_checkpointed``).  Returns the result when every item is
    done, None when ``max_slices`` slices ran and items remain."""
    Qc, dt = _as_q(Q)
    n = Qc.shape[0]
    out = _Result()
    opt = _options(B, L, tier, waves_per_cu, vgpr_levels)
    st = lib().qubo_solve_checkpointed(Qc.ctypes.data, n, dt, ctypes.byref(opt),
                                       int(items_per_slice), int(max_slices), path.encode(),
                                       ctypes.byref(out))
    if st == -6:
        return None
    _check(st)
    return _result(out, n)


def checkpoint_info(path: str) -> dict:
    """Progress recorded in a checkpoint file (host only)."""
    c = _Checkpoint()
    _check(lib().qubo_checkpoint_info(path.encode(), ctypes.byref(c)))
    d = {f: getattr(c, f) for f, _ in _Checkpoint._fields_ if f != "best"}
    d["dtype"] = "fp32" if c.dtype == QUBO_FP32 else "int32"
    d["best"] = (c.best.energy_i, c.best.energy, c.best.index)
    return d


def probe_valu(op: str = "add", waves_per_simd: int = 4, iters: int = 4096):
    """Measured int32 VALU lane-operations per second.

    op: 'add', 'min3', 'add+salu' (a scalar add per two vector adds),
    'add+branch' (a never-taken compare/branch per 16 vector adds), 'pk_add16'
    'pk_min16' (packed 16-bit pairs; one lane-op covers two values) or 'add_3w'
    (adds with a register footprint that admits at most 3 waves per SIMD) or
    'add_f32' (scalar float32 adds)."""
    rate, ms = ctypes.c_double(), ctypes.c_double()
    ops = {"add": 0, "min3": 1, "add+salu": 2, "add+branch": 3, "pk_add16": 4, "pk_min16": 5,
           "add_3w": 6, "add_f32": 7}
    _check(lib().qubo_probe_valu(ops[op], int(waves_per_simd), int(iters),
                                 ctypes.byref(rate), ctypes.byref(ms)))
    return rate.value, ms.value


_DTYPES = {"int32": QUBO_INT32, "fp32": QUBO_FP32}


_SCOPES = {"single": 0, "batch": 1}


def _entry_dict(e: _TuneEntry) -> dict:
    return {"n": e.n, "dtype": "fp32" if e.dtype == QUBO_FP32 else "int32", "B": e.B, "L": e.L,
            "tier": e.tier, "vgpr_levels": e.vgpr_levels, "walk_ms": e.walk_ms,
            "scope": "batch" if e.scope == 1 else "single"}


def autotune(n_min: int, n_max: int, dtype: str = "int32", reps: int = 2,
             cache_path: Optional[str] = None, batch: bool = False) -> List[dict]:
    """Time every runnable walk plan for n in [n_min, n_max] and install the
    fastest per n (see ``qubo_autotune``; batch=True: ``qubo_autotune_batch``,
    the plans of instances inside batches and the server); returns the winners."""
    cap = n_max - n_min + 1
    out = (_TuneEntry * max(cap, 1))()
    cnt = ctypes.c_int()
    fn = lib().qubo_autotune_batch if batch else lib().qubo_autotune
    _check(fn(int(n_min), int(n_max), _DTYPES[dtype], int(reps),
              cache_path.encode() if cache_path else None, out, cap, ctypes.byref(cnt)))
    return [_entry_dict(out[k]) for k in range(min(cnt.value, cap))]


def tune_load(path: str, device_key: Optional[str] = None) -> int:
    """Load a tuning cache (device_key None: must match this device)."""
    cnt = ctypes.c_int()
    _check(lib().qubo_tune_load(path.encode(), device_key.encode() if device_key else None,
                                ctypes.byref(cnt)))
    return cnt.value


def tune_save(path: str, device_key: Optional[str] = None):
    _check(lib().qubo_tune_save(path.encode(), device_key.encode() if device_key else None))


def tune_set(entries: Sequence[dict]):
    arr = (_TuneEntry * max(len(entries), 1))()
    for k, e in enumerate(entries):
        arr[k] = _TuneEntry(int(e["n"]), _DTYPES[e.get("dtype", "int32")], int(e["B"]),
                            int(e.get("L", 0)), int(e["tier"]), int(e["vgpr_levels"]),
                            float(e.get("walk_ms", 0.0)), _SCOPES[e.get("scope", "single")])
    _check(lib().qubo_tune_set(arr, len(entries)))


def tune_lookup(n: int, dtype: str = "int32", scope: str = "single") -> Optional[dict]:
    e = _TuneEntry()
    if lib().qubo_tune_lookup(int(n), _DTYPES[dtype], _SCOPES[scope], ctypes.byref(e)):
        return _entry_dict(e)
    return None


def tune_clear():
    lib().qubo_tune_clear()


def device_key() -> str:
    buf = ctypes.create_string_buffer(128)
    _check(lib().qubo_device_key(buf, 128))
    return buf.value.decode()


def version() -> str:
    return lib().qubo_version().decode()
