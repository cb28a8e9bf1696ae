"""ctypes binding of libdr (include/dr.h): argument marshalling only.

Every step of a solve runs in libdr's HIP kernels; this module converts
numpy arrays / torch tensors to pointers and back.  It raises if libdr.so is
missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import build as _build

DR_OK, DR_E_INVALID, DR_E_NOMEM, DR_E_DEVICE, DR_E_STATE = 0, -1, -2, -3, -4
DR_CONVERGED, DR_MAX_ITER, DR_NONFINITE, DR_RUNNING, DR_IDLE, DR_STALLED, DR_ENERGY = 0, 1, 2, 3, 4, 5, 6
DR_ABORTED = 7
DR_FP64, DR_FP32 = 0, 1
DR_RESUME, DR_START_AFFINE, DR_START_ZERO, DR_START_WARM = -1, 0, 1, 2
DR_PLACE_AUTO, DR_PLACE_LDS, DR_PLACE_GLOBAL = 0, 1, 2

_STATUS_NAMES = {DR_E_INVALID: "DR_E_INVALID", DR_E_NOMEM: "DR_E_NOMEM",
                 DR_E_DEVICE: "DR_E_DEVICE", DR_E_STATE: "DR_E_STATE"}

# Every exported symbol of include/dr.h.
EXPORTS = ("dr_options_default", "dr_batch_create", "dr_batch_workspace_bytes",
           "dr_batch_create_in", "dr_solve", "dr_solve_device",
           "dr_stress", "dr_advance", "dr_advance_each", "dr_results", "dr_energy", "dr_sync", "dr_solve_loop",
           "dr_solve_loop_scatter", "dr_solve_loop_scatter_noalloc", "dr_batch_info",
           "dr_batch_scalars", "dr_batch_pass_costs", "dr_batch_class_info", "dr_set_class_plans", "dr_graph_capture",
           "dr_graph_launch", "dr_batch_destroy", "dr_pool_create", "dr_pool_submit", "dr_pool_poll",
           "dr_pool_status", "dr_pool_destroy", "dr_state_bytes_per_node", "dr_last_error")


class DrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class dr_networks(C.Structure):
    _fields_ = [("n_problems", C.c_int32),
                ("node_offsets", C.POINTER(C.c_int64)),
                ("fiber_offsets", C.POINTER(C.c_int64)),
                ("X", C.POINTER(C.c_double)),
                ("fiber_nodes", C.POINTER(C.c_int32)),
                ("EA", C.POINTER(C.c_double)),
                ("fixed", C.POINTER(C.c_uint8)),
                ("band", C.c_double)]


class dr_options(C.Structure):
    _fields_ = [("precision", C.c_int32),
                ("tol", C.c_double),
                ("max_iter", C.c_int64),
                ("damping", C.c_double),
                ("dt_safety", C.c_double),
                ("block", C.c_int32),
                ("placement", C.c_int32),
                ("chunk", C.c_int32),
                ("stall_window", C.c_int64),
                ("energy_tol", C.c_double),
                ("tail_at", C.c_int32),
                ("tail_group", C.c_int32),
                ("dt_rule", C.c_int32)]


_lib = None


def lib_path() -> str:
    return _build.LIB


def load():
    """Loads libdr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2305_07030_amd.build.build()")
    # PyTorch's HIP runtime (same soname as the one libdr links) is loaded
    # first, so the library and torch's streams and memory share one runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.dr_options_default.argtypes = [C.POINTER(dr_options)]
    lib.dr_options_default.restype = None
    lib.dr_batch_create.argtypes = [C.POINTER(dr_networks), C.POINTER(dr_options), vp, C.POINTER(vp)]
    lib.dr_batch_create.restype = C.c_int
    lib.dr_pool_create.argtypes = [C.POINTER(dr_networks), C.POINTER(dr_options), vp, C.c_int64, C.c_int32,
                                    C.c_int64, C.POINTER(vp)]
    lib.dr_pool_create.restype = C.c_int
    lib.dr_pool_submit.argtypes = [vp, C.c_int32, vp, C.c_int64]
    lib.dr_pool_submit.restype = C.c_int
    lib.dr_pool_poll.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp]
    lib.dr_pool_poll.restype = C.c_int
    lib.dr_pool_status.argtypes = [vp, vp, vp, vp, vp]
    lib.dr_pool_status.restype = C.c_int
    lib.dr_pool_destroy.argtypes = [vp]
    lib.dr_pool_destroy.restype = None
    lib.dr_state_bytes_per_node.argtypes = [C.c_int32, C.POINTER(C.c_int64)]
    lib.dr_state_bytes_per_node.restype = C.c_int
    lib.dr_batch_workspace_bytes.argtypes = [C.POINTER(dr_networks), C.POINTER(dr_options),
                                             C.POINTER(C.c_size_t)]
    lib.dr_batch_workspace_bytes.restype = C.c_int
    lib.dr_batch_create_in.argtypes = [C.POINTER(dr_networks), C.POINTER(dr_options), vp, vp, C.c_size_t,
                                       C.POINTER(vp)]
    lib.dr_batch_create_in.restype = C.c_int
    lib.dr_solve.argtypes = [vp, vp, vp, C.c_int32, C.c_int32]
    lib.dr_solve.restype = C.c_int
    lib.dr_solve_device.argtypes = [vp, vp, vp, C.c_int32, C.c_int32]
    lib.dr_solve_device.restype = C.c_int
    lib.dr_stress.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.dr_stress.restype = C.c_int
    lib.dr_advance.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int64]
    lib.dr_advance.restype = C.c_int
    lib.dr_advance_each.argtypes = [vp, vp, vp, vp, vp, C.c_int32]
    lib.dr_advance_each.restype = C.c_int
    lib.dr_results.argtypes = [vp, vp, C.c_int32, vp, vp, vp, vp, vp, vp]
    lib.dr_results.restype = C.c_int
    lib.dr_energy.argtypes = [vp, vp, C.c_int32, vp, vp]
    lib.dr_energy.restype = C.c_int
    lib.dr_sync.argtypes = [vp]
    lib.dr_sync.restype = C.c_int
    lib.dr_solve_loop.argtypes = [vp, vp, vp, C.c_int32, C.c_int32]
    lib.dr_solve_loop.restype = C.c_int
    lib.dr_solve_loop_scatter.argtypes = [vp, vp, vp, C.c_int32, C.c_int32]
    lib.dr_solve_loop_scatter.restype = C.c_int
    lib.dr_solve_loop_scatter_noalloc.argtypes = [vp, vp, vp, C.c_int32, C.c_int32]
    lib.dr_solve_loop_scatter_noalloc.restype = C.c_int
    lib.dr_batch_info.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.dr_batch_info.restype = C.c_int
    lib.dr_batch_scalars.argtypes = [vp, vp, vp, vp]
    lib.dr_batch_scalars.restype = C.c_int
    lib.dr_batch_pass_costs.argtypes = [vp, vp]
    lib.dr_batch_pass_costs.restype = C.c_int
    lib.dr_batch_class_info.argtypes = [vp, C.c_int32] + [vp] * 8
    lib.dr_batch_class_info.restype = C.c_int
    lib.dr_set_class_plans.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    lib.dr_set_class_plans.restype = C.c_int
    lib.dr_graph_capture.argtypes = [vp, vp, vp, C.c_int32, C.c_int32]
    lib.dr_graph_capture.restype = C.c_int
    lib.dr_graph_launch.argtypes = [vp]
    lib.dr_graph_launch.restype = C.c_int
    lib.dr_batch_destroy.argtypes = [vp]
    lib.dr_batch_destroy.restype = None
    lib.dr_last_error.argtypes = []
    lib.dr_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != DR_OK:
        raise DrError(rc, load().dr_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def dr_options_default() -> dr_options:
    o = dr_options()
    load().dr_options_default(C.byref(o))
    return o


def make_options(**kw) -> dr_options:
    o = dr_options_default()
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, v)
    return o


def pack_networks(packed: dict):
    """dr_networks view of Batch.packed() arrays (the arrays are kept alive).
    With packed["fixed"] None the library's band rule decides the prescribed
    nodes (packed["band"])."""
    arrs = dict(
        node_offsets=np.ascontiguousarray(packed["node_offsets"], np.int64),
        fiber_offsets=np.ascontiguousarray(packed["fiber_offsets"], np.int64),
        X=np.ascontiguousarray(packed["X"], np.float64),
        fiber_nodes=np.ascontiguousarray(packed["fiber_nodes"], np.int32),
        EA=np.ascontiguousarray(packed["EA"], np.float64),
    )
    if packed.get("fixed") is not None:
        arrs["fixed"] = np.ascontiguousarray(packed["fixed"], np.uint8)
    n = dr_networks()
    n.n_problems = len(arrs["node_offsets"]) - 1
    n.node_offsets = arrs["node_offsets"].ctypes.data_as(C.POINTER(C.c_int64))
    n.fiber_offsets = arrs["fiber_offsets"].ctypes.data_as(C.POINTER(C.c_int64))
    n.X = arrs["X"].ctypes.data_as(C.POINTER(C.c_double))
    n.fiber_nodes = arrs["fiber_nodes"].ctypes.data_as(C.POINTER(C.c_int32))
    n.EA = arrs["EA"].ctypes.data_as(C.POINTER(C.c_double))
    if "fixed" in arrs:
        n.fixed = arrs["fixed"].ctypes.data_as(C.POINTER(C.c_uint8))
    n.band = float(packed.get("band", 0.0))
    return n, arrs


def dr_batch_create(packed: dict, opt: dr_options, stream=None) -> int:
    """Returns the opaque handle (an int)."""
    lib = load()
    nets, keep = pack_networks(packed)
    h = C.c_void_p()
    _check(lib.dr_batch_create(C.byref(nets), C.byref(opt), stream, C.byref(h)))
    del keep
    return h.value


def dr_batch_workspace_bytes(packed: dict, opt: dr_options) -> int:
    """Device bytes dr_batch_create_in needs (host only, no device call)."""
    lib = load()
    nets, keep = pack_networks(packed)
    n = C.c_size_t()
    _check(lib.dr_batch_workspace_bytes(C.byref(nets), C.byref(opt), C.byref(n)))
    del keep
    return int(n.value)


def dr_batch_create_in(packed: dict, opt: dr_options, stream, workspace_ptr: int,
                       workspace_bytes: int) -> int:
    """As dr_batch_create, with the device arrays in a caller-owned buffer."""
    lib = load()
    nets, keep = pack_networks(packed)
    h = C.c_void_p()
    _check(lib.dr_batch_create_in(C.byref(nets), C.byref(opt), stream, C.c_void_p(workspace_ptr),
                                  C.c_size_t(workspace_bytes), C.byref(h)))
    del keep
    return h.value


def dr_solve(h: int, F: np.ndarray, ids: Optional[np.ndarray] = None, start: int = DR_START_AFFINE):
    F = np.ascontiguousarray(F, np.float64).reshape(-1, 9)
    idsa = None if ids is None else np.ascontiguousarray(ids, np.int32)
    _check(load().dr_solve(h, _ptr(F), _ptr(idsa), F.shape[0], int(start)))


def dr_solve_device(h: int, F_device_ptr: int, ids: Optional[np.ndarray], n_ids: int,
                    start: int = DR_START_AFFINE):
    idsa = None if ids is None else np.ascontiguousarray(ids, np.int32)
    _check(load().dr_solve_device(h, F_device_ptr, _ptr(idsa), int(n_ids), int(start)))


def dr_advance(h: int, F: np.ndarray, ids: np.ndarray, starts: np.ndarray, budget):
    """budget: one pass budget for every slot (dr_advance) or an array of one
    per slot (dr_advance_each)."""
    ids = np.ascontiguousarray(ids, np.int32)
    F = np.ascontiguousarray(F, np.float64).reshape(len(ids), 9)
    starts = np.ascontiguousarray(starts, np.int32)
    if np.ndim(budget) == 0:
        _check(load().dr_advance(h, _ptr(F), _ptr(ids), _ptr(starts), len(ids), int(budget)))
    else:
        bud = np.ascontiguousarray(budget, np.int64)
        assert bud.shape == (len(ids),)
        _check(load().dr_advance_each(h, _ptr(F), _ptr(ids), _ptr(starts), _ptr(bud), len(ids)))


def dr_results(h: int, ids: np.ndarray) -> dict:
    ids = np.ascontiguousarray(ids, np.int32)
    n = len(ids)
    sig = np.zeros((n, 9)); sigf = np.zeros((n, 9))
    res = np.zeros(n, np.int32); it = np.zeros(n, np.int64)
    rho = np.zeros(n); ke = np.zeros(n)
    _check(load().dr_results(h, _ptr(ids), n, _ptr(sig), _ptr(sigf), _ptr(res), _ptr(it),
                             _ptr(rho), _ptr(ke)))
    return dict(sigma=sig.reshape(n, 3, 3), sigma_fib=sigf.reshape(n, 3, 3), result=res,
                iters=it, rho=rho, ke=ke)


def dr_energy(h: int, ids: np.ndarray) -> dict:
    ids = np.ascontiguousarray(ids, np.int32)
    w = np.zeros(len(ids)); d = np.zeros(len(ids))
    _check(load().dr_energy(h, _ptr(ids), len(ids), _ptr(w), _ptr(d)))
    return dict(work_int=w, work_damp=d)


def dr_solve_loop(h: int, F: np.ndarray, ids: Optional[np.ndarray] = None, start: int = DR_START_AFFINE):
    F = np.ascontiguousarray(F, np.float64).reshape(-1, 9)
    idsa = None if ids is None else np.ascontiguousarray(ids, np.int32)
    _check(load().dr_solve_loop(h, _ptr(F), _ptr(idsa), F.shape[0], int(start)))


def dr_solve_loop_scatter(h: int, F: np.ndarray, ids: Optional[np.ndarray] = None, start: int = DR_START_AFFINE):
    F = np.ascontiguousarray(F, np.float64).reshape(-1, 9)
    idsa = None if ids is None else np.ascontiguousarray(ids, np.int32)
    _check(load().dr_solve_loop_scatter(h, _ptr(F), _ptr(idsa), F.shape[0], int(start)))


def dr_solve_loop_scatter_noalloc(h: int, F: np.ndarray, ids: Optional[np.ndarray] = None,
                                  start: int = DR_START_AFFINE):
    F = np.ascontiguousarray(F, np.float64).reshape(-1, 9)
    idsa = None if ids is None else np.ascontiguousarray(ids, np.int32)
    _check(load().dr_solve_loop_scatter_noalloc(h, _ptr(F), _ptr(idsa), F.shape[0], int(start)))


def dr_stress(h: int, n_ids: int, total_nodes: Optional[int] = None, want_u: bool = False) -> dict:
    sig = np.zeros((n_ids, 9)); sigf = np.zeros((n_ids, 9))
    res = np.zeros(n_ids, np.int32); it = np.zeros(n_ids, np.int64)
    rho = np.zeros(n_ids); ke = np.zeros(n_ids)
    u = np.zeros((total_nodes, 3)) if want_u else None
    _check(load().dr_stress(h, _ptr(sig), _ptr(sigf), _ptr(u), _ptr(res), _ptr(it), _ptr(rho), _ptr(ke)))
    return dict(sigma=sig.reshape(n_ids, 3, 3), sigma_fib=sigf.reshape(n_ids, 3, 3), u=u,
                result=res, iters=it, rho=rho, ke=ke)


def dr_sync(h: int):
    _check(load().dr_sync(h))


def dr_batch_info(h: int) -> dict:
    a = C.c_int32(); b = C.c_int64(); c = C.c_int64(); d = C.c_int32(); e = C.c_int32(); f = C.c_int32()
    _check(load().dr_batch_info(h, C.addressof(a), C.addressof(b), C.addressof(c), C.addressof(d),
                                C.addressof(e), C.addressof(f)))
    return dict(n_problems=a.value, total_nodes=b.value, total_fibers=c.value, block=d.value,
                lds_bytes=e.value, nodes_per_thread=f.value)


def dr_batch_pass_costs(h: int, n_problems: int) -> np.ndarray:
    out = np.zeros(n_problems)
    _check(load().dr_batch_pass_costs(h, _ptr(out)))
    return out


def dr_batch_scalars(h: int, n_problems: int) -> dict:
    dt = np.zeros(n_problems); c = np.zeros(n_problems); fl = np.zeros(n_problems)
    _check(load().dr_batch_scalars(h, _ptr(dt), _ptr(c), _ptr(fl)))
    return dict(dt=dt, c=c, s_floor=fl)


def dr_batch_class_info(h: int) -> list:
    """One dict per size class."""
    out = []
    c = 0
    while True:
        v = [C.c_int32() for _ in range(8)]
        rc = load().dr_batch_class_info(h, c, *[C.addressof(x) for x in v])
        if c >= v[0].value:
            break
        _check(rc)
        out.append(dict(n_lo=v[1].value, n_hi=v[2].value, n_problems=v[3].value, block=v[4].value,
                        nodes_per_thread=v[5].value, chunk=v[6].value, lds_bytes=v[7].value))
        c += 1
    return out


def dr_set_class_plans(h: int, n_hi, block, chunk, placement):
    a = [np.ascontiguousarray(x, np.int32) for x in (n_hi, block, chunk, placement)]
    _check(load().dr_set_class_plans(h, len(a[0]), *[_ptr(x) for x in a]))


def dr_graph_capture(h: int, F_device_ptr: int, ids: Optional[np.ndarray], n_ids: int,
                     start: int = DR_START_AFFINE):
    idsa = None if ids is None else np.ascontiguousarray(ids, np.int32)
    _check(load().dr_graph_capture(h, F_device_ptr, _ptr(idsa), int(n_ids), int(start)))


def dr_graph_launch(h: int):
    _check(load().dr_graph_launch(h))


def dr_batch_destroy(h: int):
    load().dr_batch_destroy(h)


def state_bytes_per_node(precision: int = DR_FP64) -> int:
    """Running-state bytes per node of an in-flight solve (the unit of a
    serving pool's state budget)."""
    v = C.c_int64()
    _check(load().dr_state_bytes_per_node(int(precision), C.byref(v)))
    return int(v.value)


def dr_last_error() -> str:
    return load().dr_last_error().decode()


def current_stream():
    """The current torch HIP stream as a raw pointer (None without a GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class Pool:
    """The library's serving pool (dr_pool_*) over a resident batch: submit
    requests (network, F, tag), poll() runs one scheduling step and returns
    the finished ones."""

    def __init__(self, batch, *, state_budget_bytes=0, max_slots=256, tick_passes=4000, stream=None,
                 **opts):
        lib = load()
        nets, keep = pack_networks(batch.packed())
        h = C.c_void_p()
        _check(lib.dr_pool_create(C.byref(nets), C.byref(make_options(**opts)),
                                  stream if stream is not None else current_stream(),
                                  int(state_budget_bytes), int(max_slots), int(tick_passes), C.byref(h)))
        del keep
        self.h = h.value
        self.cap = max(1, len(batch))

    def submit(self, net: int, F, tag: int):
        F = np.ascontiguousarray(F, np.float64).reshape(9)
        _check(load().dr_pool_submit(self.h, int(net), _ptr(F), int(tag)))

    def poll(self, max_out=None) -> dict:
        m = self.cap if max_out is None else int(max_out)
        tags = np.zeros(max(m, 1), np.int64)
        ids = np.zeros(max(m, 1), np.int32)
        sigma = np.zeros((max(m, 1), 3, 3))
        res = np.zeros(max(m, 1), np.int32)
        it = np.zeros(max(m, 1), np.int64)
        n = C.c_int32()
        _check(load().dr_pool_poll(self.h, m, _ptr(tags), _ptr(ids), _ptr(sigma), _ptr(res), _ptr(it),
                                   C.byref(n)))
        k = n.value
        return dict(tags=tags[:k], ids=ids[:k], sigma=sigma[:k], result=res[:k], iters=it[:k])

    def status(self) -> dict:
        q, f, c = C.c_int32(), C.c_int32(), C.c_int32()
        b = C.c_int64()
        _check(load().dr_pool_status(self.h, C.byref(q), C.byref(f), C.byref(c), C.byref(b)))
        return dict(queued=q.value, in_flight=f.value, completed=c.value, state_bytes=b.value)

    def close(self):
        if self.h:
            load().dr_pool_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(batch, **opts) -> int:
    """Device bytes a DRBatch of `batch` with these options needs as its
    workspace (host only)."""
    return dr_batch_workspace_bytes(batch.packed(), make_options(**opts))


class DRBatch:
    """Owns one dr_batch handle for a paper_2305_07030_amd.inputs.Batch."""

    def __init__(self, batch, *, tol=1e-8, max_iter=2_000_000, damping=1e-3, dt_safety=0.9,
                 block=0, placement=DR_PLACE_AUTO, chunk=0, stall_window=0, precision=DR_FP64,
                 energy_tol=0.0, tail_at=0, tail_group=0, dt_rule=0, stream=None, workspace=None):
        """workspace: None (the library allocates), or a device tensor whose
        storage holds the batch's device arrays (at least
        workspace_bytes(...) bytes, 256-byte aligned); it is kept referenced
        until close()."""
        self.batch = batch
        self.P = len(batch)
        self.total_nodes = batch.total_nodes
        self.opt = make_options(precision=precision, tol=tol, max_iter=max_iter, damping=damping,
                                dt_safety=dt_safety, block=block, placement=placement,
                                chunk=chunk, stall_window=stall_window, energy_tol=energy_tol,
                                tail_at=tail_at, tail_group=tail_group, dt_rule=dt_rule)
        st = stream if stream is not None else current_stream()
        self.workspace = workspace
        if workspace is None:
            self.h = dr_batch_create(batch.packed(), self.opt, st)
        else:
            nbytes = workspace.numel() * workspace.element_size()
            self.h = dr_batch_create_in(batch.packed(), self.opt, st, workspace.data_ptr(), nbytes)
        self._n_last = None

    def solve(self, F=None, ids=None, start=DR_START_AFFINE):
        if F is None:
            F = self.batch.F if ids is None else self.batch.F[np.asarray(ids)]
        F = np.asarray(F).reshape(-1, 9)
        dr_solve(self.h, F, ids, start)
        self._n_last = F.shape[0]

    def solve_loop(self, F=None, ids=None, start=DR_START_AFFINE, scatter=False):
        if F is None:
            F = self.batch.F if ids is None else self.batch.F[np.asarray(ids)]
        F = np.asarray(F).reshape(-1, 9)
        (dr_solve_loop_scatter if scatter else dr_solve_loop)(self.h, F, ids, start)
        self._n_last = F.shape[0]

    def solve_device(self, F_dev, ids=None, start=DR_START_AFFINE):
        n = int(F_dev.shape[0])
        dr_solve_device(self.h, F_dev.data_ptr(), ids, n, start)
        self._n_last = n

    def advance(self, ids, starts, budget, F=None):
        ids = np.asarray(ids, np.int32)
        if F is None:
            F = np.tile(np.eye(3), (len(ids), 1, 1))
        dr_advance(self.h, F, ids, starts, budget)

    def query(self, ids) -> dict:
        return dr_results(self.h, ids)

    def energy(self, ids=None) -> dict:
        ids = np.arange(self.P, dtype=np.int32) if ids is None else ids
        return dr_energy(self.h, ids)

    def results(self, want_u=False) -> dict:
        if self._n_last is None:
            raise DrError(DR_E_STATE, "no solve yet")
        r = dr_stress(self.h, self._n_last, self.total_nodes, want_u)
        if want_u:
            no = self.batch.packed()["node_offsets"]
            r["u_list"] = [r["u"][no[i]:no[i + 1]] for i in range(self.P)]
        return r

    def sync(self):
        dr_sync(self.h)

    def info(self) -> dict:
        return dr_batch_info(self.h)

    def classes(self) -> list:
        return dr_batch_class_info(self.h)

    def set_class_plans(self, plans):
        """plans: list of dicts with n_hi, block, chunk, placement."""
        dr_set_class_plans(self.h, [p["n_hi"] for p in plans], [p["block"] for p in plans],
                           [p["chunk"] for p in plans], [p["placement"] for p in plans])

    def graph_capture(self, F_dev, ids=None, start=DR_START_AFFINE):
        n = int(F_dev.shape[0])
        dr_graph_capture(self.h, F_dev.data_ptr(), ids, n, start)
        self._graph_n = n

    def graph_launch(self):
        dr_graph_launch(self.h)
        self._n_last = self._graph_n

    def scalars(self) -> dict:
        return dr_batch_scalars(self.h, self.P)

    def pass_costs(self) -> np.ndarray:
        """Estimated seconds per pass of each problem (dr_batch_pass_costs)."""
        return dr_batch_pass_costs(self.h, self.P)

    def close(self):
        if self.h:
            dr_batch_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
