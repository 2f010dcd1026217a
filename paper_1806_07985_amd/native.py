"""ctypes binding of the C ABI in include/nncp.h (argument marshalling only).

Every computation runs in the HIP library ``lib/libnncp.so``; this module only
turns torch device tensors into pointers and sizes. If the library is missing,
``lib()`` raises: there is no fallback path.

Layout conventions (see include/nncp.h): a tensor of shape (I_1, ..., I_N) is
passed as a flat device tensor in mode-1-fastest order, and a factor matrix
I_n x R (column-major) as a contiguous torch tensor of shape (R, I_n).
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libnncp.so")

NNCP_OK = 0
HALS, MU = 0, 1
F32, BF16, F16 = 0, 1, 2
_UPDATE = {"hals": HALS, "mu": MU}
_DTYPE = {"f32": F32, "bf16": BF16, "f16": F16}

c_i64p = ctypes.POINTER(ctypes.c_int64)
c_dp = ctypes.POINTER(ctypes.c_double)
c_vp = ctypes.c_void_p


class Options(ctypes.Structure):
    _fields_ = [("split", ctypes.c_int), ("no_record_fit", ctypes.c_int), ("no_graph", ctypes.c_int),
                ("phase_timers", ctypes.c_int), ("tol", ctypes.c_double),
                ("pm_wg_kib", ctypes.c_int),
                ("no_tree", ctypes.c_int),
                ("inner_sweeps", ctypes.c_int),
                ("reserved0", ctypes.c_int),
                ("inner_tol", ctypes.c_double),
                ("tree_peel", ctypes.c_uint64)]


class JobRequest(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("dtype", ctypes.c_int), ("N", ctypes.c_int),
                ("dims", ctypes.POINTER(ctypes.c_int64)), ("R", ctypes.c_int), ("update", ctypes.c_int),
                ("iters", ctypes.c_int), ("split", ctypes.c_int), ("H0", ctypes.POINTER(ctypes.c_void_p))]


class JobResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters_done", ctypes.c_int), ("submit_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("start_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("footprint_bytes", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int), ("active", ctypes.c_int), ("peak_active", ctypes.c_int),
                ("ticks", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t), ("budget_bytes", ctypes.c_size_t),
                ("busy_s", ctypes.c_double), ("now_s", ctypes.c_double), ("graph_captures", ctypes.c_int64),
                ("list_updates", ctypes.c_int64), ("rebuild_s", ctypes.c_double), ("graph_s", ctypes.c_double)]


class NNCPError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = _lib.nncp_strerror(status).decode() if _lib is not None else str(status)
        if status == -3 and _lib is not None:
            code, where = last_device_error()
            msg += f" [last HIP error {code} at {where}]"
        super().__init__(f"{what}: {msg} ({status})")
        self.status = status


def last_device_error():
    """(hipError_t, source location) of the library's most recent failed HIP
    call, or (0, 0) if none since it was loaded."""
    L = lib()
    code, where = ctypes.c_int(0), ctypes.c_int(0)
    L.nncp_last_device_error(ctypes.byref(code), ctypes.byref(where))
    return code.value, where.value


_lib = None


def _declare(L):
    L.nncp_strerror.restype = ctypes.c_char_p
    L.nncp_strerror.argtypes = [ctypes.c_int]
    L.nncp_version.restype = ctypes.c_int
    L.nncp_last_device_error.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.nncp_workspace_bytes.restype = ctypes.c_size_t
    L.nncp_workspace_bytes.argtypes = [ctypes.c_int, c_i64p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Options)]
    L.nncp.restype = ctypes.c_int
    L.nncp.argtypes = [c_vp, ctypes.c_int, ctypes.c_int, c_i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                       ctypes.POINTER(c_vp), c_dp, c_dp, ctypes.POINTER(ctypes.c_int), c_vp, ctypes.c_size_t,
                       ctypes.POINTER(Options), c_vp]
    L.nncp_plan_create.restype = ctypes.c_int
    L.nncp_plan_create.argtypes = [ctypes.POINTER(c_vp), c_vp, ctypes.c_int, ctypes.c_int, c_i64p, ctypes.c_int,
                                   ctypes.c_int, ctypes.POINTER(c_vp), c_dp, c_vp, ctypes.c_size_t,
                                   ctypes.POINTER(Options), c_vp]
    L.nncp_plan_run.restype = ctypes.c_int
    L.nncp_plan_run.argtypes = [c_vp, ctypes.c_int, c_dp, ctypes.POINTER(ctypes.c_int)]
    L.nncp_plan_finish.restype = ctypes.c_int
    L.nncp_plan_finish.argtypes = [c_vp, c_dp]
    L.nncp_plan_phase_ms.restype = ctypes.c_int
    L.nncp_plan_phase_ms.argtypes = [c_vp, c_dp]
    L.nncp_plan_time_node.restype = ctypes.c_int
    L.nncp_plan_time_node.argtypes = [c_vp, ctypes.c_int, ctypes.c_int, c_dp]
    L.nncp_plan_time_mttkrp.restype = ctypes.c_int
    L.nncp_plan_time_mttkrp.argtypes = [c_vp, ctypes.c_int, c_dp]
    L.nncp_plan_set_stream.restype = ctypes.c_int
    L.nncp_plan_set_stream.argtypes = [c_vp, c_vp]
    L.nncp_plan_destroy.restype = ctypes.c_int
    L.nncp_plan_destroy.argtypes = [c_vp]
    L.nncp_autotune_split.restype = ctypes.c_int
    L.nncp_autotune_split.argtypes = [c_vp, ctypes.c_int, ctypes.c_int, c_i64p, ctypes.c_int, ctypes.POINTER(c_vp),
                                      c_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), c_dp, c_vp]
    L.nncp_autotune_tree.restype = ctypes.c_int
    L.nncp_autotune_tree.argtypes = [c_vp, ctypes.c_int, ctypes.c_int, c_i64p, ctypes.c_int, ctypes.POINTER(c_vp),
                                     c_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_uint64), c_dp, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int), c_vp]
    L.nncp_quantize.restype = ctypes.c_int
    L.nncp_quantize.argtypes = [c_vp, c_vp, ctypes.c_int, ctypes.c_int64, c_vp]
    L.nncp_norm_sq.restype = ctypes.c_int
    L.nncp_norm_sq.argtypes = [c_vp, ctypes.c_int, ctypes.c_int64, c_vp, c_vp]
    L.nncp_norm_sq_noalloc.restype = ctypes.c_int
    L.nncp_norm_sq_noalloc.argtypes = [c_vp, ctypes.c_int, ctypes.c_int64, c_vp, c_vp]
    L.nncp_partial_mttkrp.restype = ctypes.c_int
    L.nncp_partial_mttkrp.argtypes = [c_vp, ctypes.c_int, ctypes.c_int, c_i64p, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(c_vp), ctypes.c_int, c_vp, c_vp]
    L.nncp_mttv.restype = ctypes.c_int
    L.nncp_mttv.argtypes = [c_vp, ctypes.c_int, c_i64p, ctypes.c_int, ctypes.POINTER(c_vp), ctypes.c_int, c_vp,
                            c_vp]
    L.nncp_mttkrp.restype = ctypes.c_int
    L.nncp_mttkrp.argtypes = [c_vp, ctypes.c_int, ctypes.c_int, c_i64p, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(c_vp), ctypes.c_int, c_vp, c_vp]
    L.nncp_gram.restype = ctypes.c_int
    L.nncp_gram.argtypes = [c_vp, ctypes.c_int64, ctypes.c_int, c_vp, c_vp]
    L.nncp_nls_update.restype = ctypes.c_int
    L.nncp_nls_update.argtypes = [c_vp, c_vp, ctypes.c_int64, ctypes.c_int, c_vp, c_vp, ctypes.c_int, c_vp, c_vp]
    L.nncp_nls_solve.restype = ctypes.c_int
    L.nncp_nls_solve.argtypes = [c_vp, c_vp, ctypes.c_int64, ctypes.c_int, c_vp, c_vp, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, c_vp, c_vp, c_vp]
    L.nncp_plan_fits.restype = ctypes.c_int
    L.nncp_plan_fits.argtypes = [c_vp, c_dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.nncp_batch_create.restype = ctypes.c_int
    L.nncp_batch_create.argtypes = [ctypes.POINTER(c_vp), c_vp]
    L.nncp_batch_add.restype = ctypes.c_int
    L.nncp_batch_add.argtypes = [c_vp, c_vp]
    L.nncp_batch_remove.restype = ctypes.c_int
    L.nncp_batch_remove.argtypes = [c_vp, c_vp]
    L.nncp_batch_size.restype = ctypes.c_int
    L.nncp_batch_size.argtypes = [c_vp]
    L.nncp_batch_run.restype = ctypes.c_int
    L.nncp_batch_run.argtypes = [c_vp, ctypes.c_int]
    L.nncp_batch_stats.restype = ctypes.c_int
    L.nncp_batch_stats.argtypes = [c_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)]
    L.nncp_batch_captures.restype = ctypes.c_int
    L.nncp_batch_captures.argtypes = [c_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.nncp_batch_build_time.restype = ctypes.c_int
    L.nncp_batch_build_time.argtypes = [c_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.nncp_batch_destroy.restype = ctypes.c_int
    L.nncp_batch_destroy.argtypes = [c_vp]
    L.nncp_server_create.restype = ctypes.c_int
    L.nncp_server_create.argtypes = [ctypes.POINTER(c_vp), ctypes.c_size_t, ctypes.c_int, ctypes.c_int]
    L.nncp_server_submit.restype = ctypes.c_int
    L.nncp_server_submit.argtypes = [c_vp, ctypes.POINTER(JobRequest), ctypes.POINTER(ctypes.c_uint64)]
    L.nncp_server_poll.restype = ctypes.c_int
    L.nncp_server_poll.argtypes = [c_vp, ctypes.c_uint64, ctypes.POINTER(JobResult)]
    L.nncp_server_wait.restype = ctypes.c_int
    L.nncp_server_wait.argtypes = [c_vp, ctypes.c_uint64, ctypes.c_double]
    L.nncp_server_fetch.restype = ctypes.c_int
    L.nncp_server_fetch.argtypes = [c_vp, ctypes.c_uint64, ctypes.POINTER(c_vp), c_dp, c_dp, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int)]
    L.nncp_server_get_stats.restype = ctypes.c_int
    L.nncp_server_get_stats.argtypes = [c_vp, ctypes.POINTER(ServerStats)]
    L.nncp_server_destroy.restype = ctypes.c_int
    L.nncp_server_destroy.argtypes = [c_vp]


def lib():
    """Load the built library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_1806_07985_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != NNCP_OK:
        raise NNCPError(status, what)


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _ptr(t) -> int:
    return int(t.data_ptr())


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dims(dims: Sequence[int]):
    arr = (ctypes.c_int64 * len(dims))(*[int(d) for d in dims])
    return arr


def _ptr_array(tensors) -> "ctypes.Array":
    return (c_vp * len(tensors))(*[_ptr(t) for t in tensors])


def _dtype_code(t) -> int:
    import torch
    m = {torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}
    if t.dtype not in m:
        raise TypeError(f"unsupported tensor dtype {t.dtype}")
    return m[t.dtype]


def _need(t, numel: int, dtype=None, name="tensor"):
    import torch
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")


def tensor_to_device(X: np.ndarray, dtype=None, device="cuda"):
    """Flat device copy of a numpy tensor in mode-1-fastest order."""
    import torch
    flat = np.asarray(X).ravel(order="F")
    t = torch.from_numpy(np.ascontiguousarray(flat))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


def factor_to_device(H: np.ndarray, device="cuda"):
    """I x R numpy factor -> device float32 (R, I) tensor (column-major I x R)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(H, dtype=np.float32).T)).to(device)


def factor_to_host(t) -> np.ndarray:
    """Device (R, I) factor -> I x R numpy float64."""
    return t.detach().cpu().numpy().astype(np.float64).T.copy()


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def version() -> int:
    return lib().nncp_version()


def workspace_bytes(dims, R, dtype="f32", split=0, pm_wg_kib=0, no_tree=False, peel=0) -> int:
    o = Options(split=split, pm_wg_kib=pm_wg_kib, no_tree=1 if no_tree else 0, tree_peel=peel)
    return int(lib().nncp_workspace_bytes(len(dims), _dims(dims), R, _DTYPE[dtype], ctypes.byref(o)))


def _dtype_name(t) -> str:
    return {0: "f32", 1: "bf16", 2: "f16"}[_dtype_code(t)]


def nncp(X, dims, R, iters, H, lam=None, update="hals", split=0, graph=True, record_fit=True,
         tol=0.0, workspace=None, stream=None, pm_wg_kib=0, no_tree=False, inner_sweeps=1, inner_tol=0.0,
         peel=0):
    """Run the full driver. H: list of device (R, I_n) float32 tensors, updated in place.

    Returns dict(fit=np.ndarray, lam=np.ndarray, iters_done=int).
    """
    import torch
    L = lib()
    N = len(dims)
    I = int(np.prod(dims))
    _need(X, I, name="X")
    for n, h in enumerate(H):
        _need(h, dims[n] * R, torch.float32, name=f"H[{n}]")
    lam_arr = (ctypes.c_double * R)(*(np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)))
    fit = (ctypes.c_double * max(1, iters))()
    done = ctypes.c_int(0)
    o = Options(split=split, no_record_fit=0 if record_fit else 1, no_graph=0 if graph else 1, tol=tol,
                pm_wg_kib=pm_wg_kib, no_tree=1 if no_tree else 0, inner_sweeps=inner_sweeps, inner_tol=inner_tol,
                tree_peel=peel)
    ws_ptr, ws_bytes = (None, 0)
    if workspace is not None:
        ws_ptr, ws_bytes = _ptr(workspace), workspace.numel() * workspace.element_size()
    st = L.nncp(_ptr(X), _dtype_code(X), N, _dims(dims), R, iters, _UPDATE[update], _ptr_array(H),
                lam_arr, fit, ctypes.byref(done), ws_ptr, ws_bytes, ctypes.byref(o), _stream(stream))
    _check(st, "nncp")
    n_fit = done.value if record_fit else 1
    return dict(fit=np.array(fit[:n_fit]), lam=np.array(lam_arr[:]), iters_done=done.value)


def autotune_split(X, dims, R, H, reps=3, pm_wg_kib=0, stream=None):
    """Fastest root split of the dimension tree for this problem, timed on the
    device (nncp_autotune_split). H: device factors (read only).

    Returns (best_split, ms) with ms[s - 1] the tree-MTTKRP time of split s
    (-1 where its workspace did not fit)."""
    import torch
    N = len(dims)
    _need(X, int(np.prod(dims)), name="X")
    for n, h in enumerate(H):
        _need(h, dims[n] * R, torch.float32, name=f"H[{n}]")
    o = Options(pm_wg_kib=pm_wg_kib)
    best = ctypes.c_int(0)
    ms = (ctypes.c_double * (N - 1))()
    _check(lib().nncp_autotune_split(_ptr(X), _dtype_code(X), N, _dims(dims), R, _ptr_array(H), ctypes.byref(o),
                                     reps, ctypes.byref(best), ms, _stream(stream)), "nncp_autotune_split")
    return best.value, list(ms)


def autotune_tree(X, dims, R, H, reps=3, cap=64, pm_wg_kib=0, stream=None):
    """Every dimension tree (root split and internal splits) timed on the device
    (nncp_autotune_tree). Returns (best_split, best_peel, [(split, peel, ms), ...])."""
    import torch
    N = len(dims)
    _need(X, int(np.prod(dims)), name="X")
    for n, h in enumerate(H):
        _need(h, dims[n] * R, torch.float32, name=f"H[{n}]")
    o = Options(pm_wg_kib=pm_wg_kib)
    splits = (ctypes.c_int * cap)()
    peels = (ctypes.c_uint64 * cap)()
    ms = (ctypes.c_double * cap)()
    count = ctypes.c_int(0)
    best = ctypes.c_int(-1)
    _check(lib().nncp_autotune_tree(_ptr(X), _dtype_code(X), N, _dims(dims), R, _ptr_array(H), ctypes.byref(o),
                                    reps, cap, splits, peels, ms, ctypes.byref(count), ctypes.byref(best),
                                    _stream(stream)), "nncp_autotune_tree")
    rows = [(splits[k], int(peels[k]), ms[k]) for k in range(count.value)]
    return rows[best.value][0], rows[best.value][1], rows


class Plan:
    """Persistent driver state: create once, run repeatedly, finish to normalise."""

    def __init__(self, X, dims, R, H, lam=None, update="hals", split=0, graph=True, phase_timers=False,
                 workspace=None, stream=None, pm_wg_kib=0, no_tree=False, inner_sweeps=1, inner_tol=0.0, peel=0):
        import torch
        L = lib()
        self.dims, self.R, self.H, self.X = list(dims), R, list(H), X
        I = int(np.prod(dims))
        _need(X, I, name="X")
        for n, h in enumerate(H):
            _need(h, dims[n] * R, torch.float32, name=f"H[{n}]")
        lam_arr = None
        if lam is not None:
            lam_arr = (ctypes.c_double * R)(*np.asarray(lam, dtype=np.float64))
        o = Options(split=split, no_graph=0 if graph else 1, phase_timers=1 if phase_timers else 0,
                    pm_wg_kib=pm_wg_kib, no_tree=1 if no_tree else 0, inner_sweeps=inner_sweeps,
                    inner_tol=inner_tol, tree_peel=peel)
        self._ws = workspace
        if workspace is None:
            nbytes = workspace_bytes(dims, R, _dtype_name(X), split, pm_wg_kib, no_tree, peel)
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
        handle = c_vp()
        st = L.nncp_plan_create(ctypes.byref(handle), _ptr(X), _dtype_code(X), len(dims), _dims(dims), R,
                                _UPDATE[update], _ptr_array(H), lam_arr, _ptr(self._ws),
                                self._ws.numel(), ctypes.byref(o), _stream(stream))
        _check(st, "nncp_plan_create")
        self._h = handle

    def run(self, iters: int) -> np.ndarray:
        fit = (ctypes.c_double * max(1, iters))()
        done = ctypes.c_int(0)
        _check(lib().nncp_plan_run(self._h, iters, fit, ctypes.byref(done)), "nncp_plan_run")
        return np.array(fit[:done.value])

    def finish(self) -> np.ndarray:
        lam = (ctypes.c_double * self.R)()
        _check(lib().nncp_plan_finish(self._h, lam), "nncp_plan_finish")
        return np.array(lam[:])

    def phase_ms(self) -> dict:
        ms = (ctypes.c_double * 6)()
        _check(lib().nncp_plan_phase_ms(self._h, ms), "nncp_plan_phase_ms")
        return dict(zip(["pm", "mttv", "nls", "gram", "err", "total"], list(ms)))

    def time_node(self, mode: int, reps: int = 20) -> float:
        """Average ms per launch of the node kernel computed before `mode`'s update."""
        ms = ctypes.c_double(0.0)
        _check(lib().nncp_plan_time_node(self._h, mode, reps, ctypes.byref(ms)), "nncp_plan_time_node")
        return ms.value

    def time_mttkrp(self, reps: int = 10) -> float:
        """Average ms of one whole tree MTTKRP (all node ops and leaf multi-TTVs)."""
        ms = ctypes.c_double(0.0)
        _check(lib().nncp_plan_time_mttkrp(self._h, reps, ctypes.byref(ms)), "nncp_plan_time_mttkrp")
        return ms.value

    def fits(self) -> np.ndarray:
        """Fits recorded since creation (or the last run()), e.g. by batch ticks."""
        buf = (ctypes.c_double * 1024)()
        n = ctypes.c_int(0)
        _check(lib().nncp_plan_fits(self._h, buf, 1024, ctypes.byref(n)), "nncp_plan_fits")
        return np.array(buf[:min(n.value, 1024)])

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().nncp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Plans advanced together, one persistent work-list launch per step and family."""

    def __init__(self, stream=None):
        h = c_vp()
        _check(lib().nncp_batch_create(ctypes.byref(h), _stream(stream)), "nncp_batch_create")
        self._h = h
        self._members = []

    def add(self, plan: "Plan"):
        _check(lib().nncp_batch_add(self._h, plan.handle), "nncp_batch_add")
        self._members.append(plan)

    def remove(self, plan: "Plan"):
        _check(lib().nncp_batch_remove(self._h, plan.handle), "nncp_batch_remove")
        self._members.remove(plan)

    def __len__(self):
        return lib().nncp_batch_size(self._h)

    def run(self, ticks: int):
        _check(lib().nncp_batch_run(self._h, ticks), "nncp_batch_run")

    def stats(self) -> dict:
        n = ctypes.c_int(0)
        it = ctypes.c_int64(0)
        _check(lib().nncp_batch_stats(self._h, ctypes.byref(n), ctypes.byref(it)), "nncp_batch_stats")
        cap = ctypes.c_int64(0)
        upd = ctypes.c_int64(0)
        _check(lib().nncp_batch_captures(self._h, ctypes.byref(cap), ctypes.byref(upd)), "nncp_batch_captures")
        rb = ctypes.c_double(0.0)
        gs = ctypes.c_double(0.0)
        _check(lib().nncp_batch_build_time(self._h, ctypes.byref(rb), ctypes.byref(gs)), "nncp_batch_build_time")
        return dict(launches_per_tick=n.value, items_per_tick=it.value, graph_captures=cap.value,
                    list_updates=upd.value, rebuild_s=rb.value, graph_s=gs.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().nncp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SERVER_SIMULATE = 1


class Server:
    """Continuous-batching NNCP server (native worker thread; see nncp.h).

    submit() takes a host tensor (numpy array in its storage dtype, or a CPU
    torch tensor, e.g. pinned BF16) that must stay alive until the job is done;
    the server keeps a reference for that long.
    """

    def __init__(self, hbm_budget_bytes: int, max_active: int = 64, simulate: bool = False):
        h = c_vp()
        _check(lib().nncp_server_create(ctypes.byref(h), int(hbm_budget_bytes), int(max_active),
                                        SERVER_SIMULATE if simulate else 0), "nncp_server_create")
        self._h = h
        self._keep = {}

    def submit(self, X, dims, R, H0, iters, update="hals", split=0) -> int:
        import torch
        if isinstance(X, torch.Tensor):
            if X.is_cuda:
                raise ValueError("submit takes a host tensor")
            Xc = X.contiguous()
            code = _dtype_code(Xc)
            ptr = Xc.data_ptr()
        else:
            Xc = np.ascontiguousarray(np.asarray(X).ravel(order="F"))
            if Xc.dtype == np.float32:
                code = 0
            elif Xc.dtype == np.float16:
                code = 2
            else:
                raise TypeError(f"unsupported host tensor dtype {Xc.dtype}")
            ptr = Xc.ctypes.data
        Hs = [np.asfortranarray(np.asarray(h, dtype=np.float32)) for h in H0]
        Hp = (c_vp * len(Hs))(*[h.ctypes.data for h in Hs])
        dims_arr = _dims(dims)
        req = JobRequest(X=ptr, dtype=code, N=len(dims), dims=dims_arr, R=int(R), update=_UPDATE[update],
                         iters=int(iters), split=int(split), H0=Hp)
        jid = ctypes.c_uint64(0)
        _check(lib().nncp_server_submit(self._h, ctypes.byref(req), ctypes.byref(jid)), "nncp_server_submit")
        self._keep[jid.value] = (Xc, list(dims), int(R))
        return jid.value

    def poll(self, jid: int):
        """None while queued or running, else dict(status, iters_done, submit_s, admit_s, done_s, footprint)."""
        r = JobResult()
        st = lib().nncp_server_poll(self._h, jid, ctypes.byref(r))
        if st == -4:  # NNCP_EBUSY
            return None
        _check(st, "nncp_server_poll")
        return dict(status=r.status, iters_done=r.iters_done, submit_s=r.submit_s, admit_s=r.admit_s,
                    start_s=r.start_s, done_s=r.done_s, footprint=r.footprint_bytes)

    def wait(self, jid: int, timeout_s: float = -1.0) -> bool:
        st = lib().nncp_server_wait(self._h, jid, float(timeout_s))
        if st == -4:
            return False
        _check(st, "nncp_server_wait")
        return True

    def fetch(self, jid: int) -> dict:
        _, dims, R = self._keep[jid]
        H = [np.zeros((d, R), dtype=np.float32, order="F") for d in dims]
        Hp = (c_vp * len(H))(*[h.ctypes.data for h in H])
        lam = (ctypes.c_double * R)()
        fit = (ctypes.c_double * 1024)()
        nf = ctypes.c_int(0)
        st = lib().nncp_server_fetch(self._h, jid, Hp, lam, fit, 1024, ctypes.byref(nf))
        self._keep.pop(jid, None)
        _check(st, "nncp_server_fetch")
        return dict(H=[h.astype(np.float64) for h in H], lam=np.array(lam[:]), fit=np.array(fit[:min(nf.value, 1024)]))

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().nncp_server_get_stats(self._h, ctypes.byref(s)), "nncp_server_get_stats")
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().nncp_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def quantize(src, dtype: str, stream=None):
    import torch
    tdt = {"bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    _need(src, src.numel(), torch.float32, name="src")
    dst = torch.empty(src.numel(), dtype=tdt, device=src.device)
    _check(lib().nncp_quantize(_ptr(src), _ptr(dst), _DTYPE[dtype], src.numel(), _stream(stream)), "nncp_quantize")
    return dst


def norm_sq(X, stream=None) -> float:
    import torch
    out = torch.zeros(1, dtype=torch.float64, device=X.device)
    _check(lib().nncp_norm_sq(_ptr(X), _dtype_code(X), X.numel(), _ptr(out), _stream(stream)), "nncp_norm_sq")
    return float(out.item())


def norm_sq_noalloc(X, out, stream=None):
    """||X||^2 into the device float64 tensor `out` (one element) through the entry
    point that allocates nothing; enqueued on the stream, not synchronised."""
    import torch
    _need(out, 1, torch.float64, name="out")
    _check(lib().nncp_norm_sq_noalloc(_ptr(X), _dtype_code(X), X.numel(), _ptr(out), _stream(stream)),
           "nncp_norm_sq_noalloc")
    return out


def partial_mttkrp(X, dims, s, side, H, R, stream=None):
    import torch
    IL = int(np.prod(dims[:s]))
    IR = int(np.prod(dims[s:]))
    rows = IL if side == 0 else IR
    T = torch.empty((R, rows), dtype=torch.float64, device=X.device)
    _check(lib().nncp_partial_mttkrp(_ptr(X), _dtype_code(X), len(dims), _dims(dims), s, side, _ptr_array(H), R,
                                     _ptr(T), _stream(stream)), "nncp_partial_mttkrp")
    return T


def mttv(T, node_dims, kind, Hf, R, stream=None):
    import torch
    _need(T, int(np.prod(node_dims)) * R, torch.float64, name="T")
    if kind == 0:
        out = torch.empty((R, node_dims[0]), dtype=torch.float64, device=T.device)
    else:
        out = torch.empty((R, int(np.prod(node_dims[1:]))), dtype=torch.float64, device=T.device)
    _check(lib().nncp_mttv(_ptr(T), len(node_dims), _dims(node_dims), kind, _ptr_array(Hf), R, _ptr(out),
                           _stream(stream)), "nncp_mttv")
    return out


def mttkrp(X, dims, s, n, H, R, stream=None):
    import torch
    M = torch.empty((R, dims[n]), dtype=torch.float64, device=X.device)
    _check(lib().nncp_mttkrp(_ptr(X), _dtype_code(X), len(dims), _dims(dims), s, n, _ptr_array(H), R, _ptr(M),
                             _stream(stream)), "nncp_mttkrp")
    return M


def gram(H, I, R, stream=None):
    import torch
    G = torch.empty((R, R), dtype=torch.float64, device=H.device)
    _check(lib().nncp_gram(_ptr(H), I, R, _ptr(G), _stream(stream)), "nncp_gram")
    return G


def nls_update(M, H, I, R, S, lam, update="hals", stream=None):
    """In place: H <- normalised update; returns (lam, G) as device tensors. M is float64."""
    import torch
    _need(M, I * R, torch.float64, name="M")
    lam_t = lam.clone()
    G = torch.empty((R, R), dtype=torch.float64, device=H.device)
    _check(lib().nncp_nls_update(_ptr(M), _ptr(H), I, R, _ptr(S), _ptr(lam_t), _UPDATE[update], _ptr(G),
                                 _stream(stream)), "nncp_nls_update")
    return lam_t, G


def nls_solve(M, H, I, R, S, lam, update="hals", max_sweeps=1000, tol=0.0, stream=None):
    """In place: H <- the block subproblem solved by up to max_sweeps sweeps per row
    (stopping at relative change tol), normalised. Returns (lam, G, W) as device
    tensors, W the float64 solution before normalisation, shape (R, I)."""
    import torch
    _need(M, I * R, torch.float64, name="M")
    lam_t = lam.clone()
    G = torch.empty((R, R), dtype=torch.float64, device=H.device)
    W = torch.empty((R, I), dtype=torch.float64, device=H.device)
    _check(lib().nncp_nls_solve(_ptr(M), _ptr(H), I, R, _ptr(S), _ptr(lam_t), _UPDATE[update], int(max_sweeps),
                                float(tol), _ptr(W), _ptr(G), _stream(stream)), "nncp_nls_solve")
    return lam_t, G, W
