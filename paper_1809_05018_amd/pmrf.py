"""Thin ctypes binding of ``libpmrf.so`` (declared in ``include/pmrf.h``).

Only argument marshalling happens here: every step of the EM path runs in the
library's HIP kernels.  Device buffers are torch tensors on a ROCm device; the
HIP stream is torch's current stream unless one is given.  Importing works
without a GPU (host-side calls such as ``pmrf_build_neighborhoods`` run on the
CPU); device calls need the GPU.  If the library is not built this module
raises at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import time
from ctypes import POINTER, Structure, c_char_p, c_double, c_int32, c_int64, c_void_p

import numpy as np

# PMRF_LIB names another build of the library (an instrumented host build, say)
LIB_PATH = os.environ.get("PMRF_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpmrf.so")

PMRF_OK = 0
PMRF_EINVAL = -1
PMRF_ENOMEM = -2
PMRF_EDEVICE = -3
PMRF_EUNSUPPORTED = -4
PMRF_EBADLABEL = -10
PMRF_EBADPARAM = -11
PMRF_ERANGE = -12
PMRF_ETIMEOUT = -13

CTR_STATUS, CTR_ITERS, CTR_MAP_CONV, CTR_EM_CONV, CTR_NEAR_TIES, CTR_EVALS = range(6)
NCOUNTERS = 8

EXPORTED = (
    "pmrf_last_error", "pmrf_abi_version", "pmrf_build_neighborhoods", "pmrf_hoods_get_info",
    "pmrf_hoods_export", "pmrf_hoods_upload", "pmrf_replicate_indices", "pmrf_replicate_hood_array",
    "pmrf_hoods_free", "pmrf_em_params_default", "pmrf_em_workspace_bytes", "pmrf_em_run",
    "pmrf_em_batch_workspace_bytes", "pmrf_em_batch", "pmrf_set_launch", "pmrf_get_launch",
    "pmrf_profile_begin", "pmrf_profile_end", "pmrf_image_graph_workspace_bytes", "pmrf_image_graph",
    "pmrf_labels_to_pixels", "pmrf_confusion", "pmrf_volume_graph_workspace_bytes", "pmrf_volume_graph",
    "pmrf_launch_stats", "pmrf_em_run_noalloc", "pmrf_build_neighborhoods_device", "pmrf_hoods_device_buffer",
)


class PmrfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pmrf error {code}: {msg}")
        self.code = code


class HoodsInfo(Structure):
    _fields_ = [("n", c_int64), ("H", c_int64), ("M", c_int64), ("A", c_int64), ("max_hood", c_int64),
                ("tiles", c_int64), ("device_bytes", c_int64)]


class EmParams(Structure):
    _fields_ = [("L", c_int32), ("beta", c_double), ("max_iters", c_int32), ("conv_window", c_int32),
                ("conv_tol", c_double), ("early_exit", c_int32), ("init_from_labels", c_int32),
                ("sigma_min", c_double), ("tie_eps", c_double), ("scatter_rule", c_int32)]


class EmItem(Structure):
    _fields_ = [("hoods", c_void_p), ("d_hoodbuf", c_void_p), ("d_y", c_void_p), ("d_labels", c_void_p),
                ("d_mu", c_void_p), ("d_sigma", c_void_p), ("d_hood_energy", c_void_p), ("d_trace", c_void_p),
                ("d_iter_stats", c_void_p), ("d_counters", c_void_p), ("params", EmParams)]


class Launch(Structure):
    _fields_ = [("mode", c_int32), ("waves_per_block", c_int32), ("tiles_per_wave", c_int32),
                ("blocks_per_cu", c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1809_05018_amd/build_lib.py (or __graft_entry__.build())")
    # torch first: the library's HIP calls must go to the HIP runtime that torch
    # loads (and allocates device memory with), whatever order callers import in
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    P = POINTER
    lib.pmrf_last_error.restype = c_char_p
    lib.pmrf_abi_version.restype = c_int32
    lib.pmrf_build_neighborhoods.argtypes = [c_int32, P(c_int32), P(c_int32), c_int32, P(c_void_p)]
    lib.pmrf_build_neighborhoods_device.argtypes = [c_int32, c_void_p, c_void_p, c_int32, c_void_p, P(c_void_p)]
    lib.pmrf_hoods_device_buffer.argtypes = [c_void_p, P(c_void_p), P(c_int64)]
    lib.pmrf_hoods_get_info.argtypes = [c_void_p, P(HoodsInfo)]
    lib.pmrf_hoods_export.argtypes = [c_void_p, P(c_int64), P(c_int32), P(c_int64), P(c_int32), P(c_int64)]
    lib.pmrf_hoods_upload.argtypes = [c_void_p, c_void_p, c_int64, c_void_p]
    lib.pmrf_replicate_indices.argtypes = [c_void_p, c_int32, P(c_int32), P(c_int64), P(c_int32)]
    lib.pmrf_replicate_hood_array.argtypes = [c_int64, P(c_int64), c_int32, P(c_int32), P(c_int64), P(c_int32)]
    lib.pmrf_hoods_free.argtypes = [c_void_p]
    lib.pmrf_hoods_free.restype = None
    lib.pmrf_em_params_default.argtypes = [P(EmParams)]
    lib.pmrf_em_params_default.restype = None
    lib.pmrf_em_workspace_bytes.argtypes = [c_void_p, P(EmParams), P(c_int64)]
    lib.pmrf_em_run.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_void_p, c_void_p, c_int64, P(EmParams), c_void_p]
    lib.pmrf_em_run_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p, c_void_p, P(EmParams), c_void_p]
    lib.pmrf_em_batch_workspace_bytes.argtypes = [c_int32, P(EmItem), P(c_int64)]
    lib.pmrf_em_batch.argtypes = [c_int32, P(EmItem), c_void_p, c_int64, c_void_p]
    lib.pmrf_set_launch.argtypes = [P(Launch)]
    lib.pmrf_get_launch.argtypes = [P(Launch)]
    lib.pmrf_launch_stats.argtypes = [P(c_int64), P(c_int64), P(c_int64)]
    lib.pmrf_profile_begin.argtypes = []
    lib.pmrf_profile_end.argtypes = [P(c_double), P(c_int64)]
    lib.pmrf_image_graph_workspace_bytes.argtypes = [c_int32, c_int32, c_int32, P(c_int64)]
    lib.pmrf_image_graph.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_int64,
                                     c_void_p, P(c_int64), c_void_p, c_int64, c_void_p]
    lib.pmrf_volume_graph_workspace_bytes.argtypes = [c_int32, c_int32, c_int32, c_int32, P(c_int64)]
    lib.pmrf_volume_graph.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                      c_int64, c_void_p, P(c_int64), c_void_p, c_int64, c_void_p]
    lib.pmrf_labels_to_pixels.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p]
    lib.pmrf_confusion.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p]
    for name in EXPORTED:
        if name not in ("pmrf_last_error", "pmrf_abi_version", "pmrf_hoods_free", "pmrf_em_params_default"):
            getattr(lib, name).restype = c_int32
    return lib


lib = _load()


def _check(code):
    if code != PMRF_OK:
        raise PmrfError(code, lib.pmrf_last_error().decode())


def _p(a, ct):
    return a.ctypes.data_as(POINTER(ct))


SCATTER_OWNER, SCATTER_LAST, SCATTER_MIN = 0, 1, 2


def pmrf_em_params(L=2, beta=0.5, max_iters=20, conv_window=3, conv_tol=1e-4, early_exit=False,
                   init_from_labels=False, sigma_min=1e-3, tie_eps=1e-9, scatter_rule=SCATTER_OWNER) -> EmParams:
    p = EmParams()
    lib.pmrf_em_params_default(ctypes.byref(p))
    p.L, p.beta, p.max_iters, p.conv_window, p.conv_tol = int(L), float(beta), int(max_iters), int(conv_window), float(conv_tol)
    p.early_exit, p.init_from_labels = int(bool(early_exit)), int(bool(init_from_labels))
    p.sigma_min, p.tie_eps = float(sigma_min), float(tie_eps)
    p.scatter_rule = int(scatter_rule)
    return p


class Hoods:
    """Owner of a ``pmrf_hoods`` host object."""

    def __init__(self, handle):
        self.handle = c_void_p(handle)
        info = HoodsInfo()
        _check(lib.pmrf_hoods_get_info(self.handle, ctypes.byref(info)))
        self.info = info
        self.n, self.H, self.M, self.A = info.n, info.H, info.M, info.A
        self.max_hood, self.tiles, self.device_bytes = info.max_hood, info.tiles, info.device_bytes

    def free(self):
        if self.handle is not None and self.handle.value:
            lib.pmrf_hoods_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def export(self):
        hp = np.zeros(self.H + 1, np.int64)
        hv = np.zeros(max(1, self.M), np.int32)
        cp = np.zeros(self.H + 1, np.int64)
        own = np.zeros(max(1, self.n), np.int64)
        _check(lib.pmrf_hoods_export(self.handle, _p(hp, c_int64), _p(hv, c_int32), _p(cp, c_int64), None,
                                     _p(own, c_int64)))
        cv = np.zeros(max(1, int(cp[-1])), np.int32)
        _check(lib.pmrf_hoods_export(self.handle, None, None, None, _p(cv, c_int32), None))
        return {"hood_ptr": hp, "hood_vid": hv[: self.M], "clique_ptr": cp, "clique_vid": cv[: int(cp[-1])],
                "owner": own[: self.n]}

    def replicate(self, L):
        K = self.M * L
        tl = np.zeros(max(1, K), np.int32)
        oi = np.zeros(max(1, K), np.int64)
        hi = np.zeros(max(1, K), np.int32)
        _check(lib.pmrf_replicate_indices(self.handle, int(L), _p(tl, c_int32), _p(oi, c_int64), _p(hi, c_int32)))
        return tl[:K], oi[:K], hi[:K]

    def device_held(self):
        """(layout pointer, bytes held) of a device-built structure, else (None, 0)."""
        p, b = c_void_p(), c_int64()
        _check(lib.pmrf_hoods_device_buffer(self.handle, ctypes.byref(p), ctypes.byref(b)))
        return p.value, b.value

    def upload(self, device=None, stream=None):
        """Device copy of the layout as a uint8 torch tensor."""
        import torch

        buf = torch.empty(max(256, self.device_bytes), dtype=torch.uint8, device=device or "cuda")
        _check(lib.pmrf_hoods_upload(self.handle, c_void_p(buf.data_ptr()), buf.numel(), _stream(stream, buf.device)))
        return buf


def pmrf_build_neighborhoods(n, row_ptr, col_idx, k=1) -> Hoods:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)
    out = c_void_p()
    _check(lib.pmrf_build_neighborhoods(int(n), _p(rp, c_int32), _p(ci, c_int32), int(k), ctypes.byref(out)))
    return Hoods(out.value)


def pmrf_build_neighborhoods_device(n, row_ptr, col_idx, k=1, stream=None) -> Hoods:
    """Same structure built on the device from a CSR held in device memory
    (int32 tensors row_ptr[n + 1] and col_idx[row_ptr[n]]); numpy arrays are
    copied to the current device first.  Returns after the build has finished."""
    import torch

    dev = torch.device("cuda", torch.cuda.current_device())
    rp = torch.as_tensor(np.asarray(row_ptr, dtype=np.int32) if not torch.is_tensor(row_ptr) else row_ptr,
                         dtype=torch.int32, device=dev).contiguous()
    ci = torch.as_tensor(np.asarray(col_idx, dtype=np.int32) if not torch.is_tensor(col_idx) else col_idx,
                         dtype=torch.int32, device=dev).contiguous()
    if ci.numel() == 0:
        ci = torch.zeros(1, dtype=torch.int32, device=dev)
    out = c_void_p()
    _check(lib.pmrf_build_neighborhoods_device(int(n), rp.data_ptr(), ci.data_ptr(), int(k), _stream(stream, dev),
                                               ctypes.byref(out)))
    return Hoods(out.value)


def pmrf_replicate_hood_array(hood_ptr, L):
    hp = np.ascontiguousarray(hood_ptr, dtype=np.int64)
    K = int(hp[-1]) * L
    tl = np.zeros(max(1, K), np.int32)
    oi = np.zeros(max(1, K), np.int64)
    hi = np.zeros(max(1, K), np.int32)
    _check(lib.pmrf_replicate_hood_array(hp.size - 1, _p(hp, c_int64), int(L), _p(tl, c_int32), _p(oi, c_int64),
                                         _p(hi, c_int32)))
    return tl[:K], oi[:K], hi[:K]


def _stream(stream, device):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream(device)
    return c_void_p(stream.cuda_stream)


def _ptr(t, dtype, numel, name):
    import torch

    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"{name} must be contiguous with at least {numel} elements")
    return c_void_p(t.data_ptr())


def pmrf_em_workspace_bytes(hoods: Hoods, params: EmParams) -> int:
    b = c_int64()
    _check(lib.pmrf_em_workspace_bytes(hoods.handle, ctypes.byref(params), ctypes.byref(b)))
    return b.value


def pmrf_em_run(hoods: Hoods, hoodbuf, y, labels, mu, sigma, hood_energy, trace, iter_stats, counters, ws,
                params: EmParams, stream=None):
    import torch

    L, T = params.L, params.max_iters
    _check(lib.pmrf_em_run(
        hoods.handle, _ptr(hoodbuf, torch.uint8, hoods.device_bytes, "hoodbuf"), _ptr(y, torch.float64, hoods.n, "y"),
        _ptr(labels, torch.int32, hoods.n, "labels"), _ptr(mu, torch.float64, L, "mu"),
        _ptr(sigma, torch.float64, L, "sigma"), _ptr(hood_energy, torch.float64, hoods.H, "hood_energy"),
        _ptr(trace, torch.float64, T, "trace"), _ptr(iter_stats, torch.int64, 2 * T, "iter_stats"),
        _ptr(counters, torch.int64, NCOUNTERS, "counters"), _ptr(ws, torch.uint8, 0, "ws"),
        ws.numel(), ctypes.byref(params), _stream(stream, ws.device)))


NOALLOC_WS_BYTES = 64 << 20  # PMRF_NOALLOC_WS_BYTES


def pmrf_em_run_noalloc(hoods: Hoods, hoodbuf, y, labels, mu, sigma, hood_energy, trace, iter_stats, counters,
                        params: EmParams, stream=None):
    """pmrf_em_run with the library's static per-GPU workspace (allocates nothing)."""
    import torch

    L, T = params.L, params.max_iters
    dev = labels.device if isinstance(labels, torch.Tensor) else None
    _check(lib.pmrf_em_run_noalloc(
        hoods.handle, _ptr(hoodbuf, torch.uint8, hoods.device_bytes, "hoodbuf"), _ptr(y, torch.float64, hoods.n, "y"),
        _ptr(labels, torch.int32, hoods.n, "labels"), _ptr(mu, torch.float64, L, "mu"),
        _ptr(sigma, torch.float64, L, "sigma"), _ptr(hood_energy, torch.float64, hoods.H, "hood_energy"),
        _ptr(trace, torch.float64, T, "trace"), _ptr(iter_stats, torch.int64, 2 * T, "iter_stats"),
        _ptr(counters, torch.int64, NCOUNTERS, "counters"), ctypes.byref(params), _stream(stream, dev)))


def pmrf_em_batch_workspace_bytes(items) -> int:
    arr = (EmItem * len(items))(*items)
    b = c_int64()
    _check(lib.pmrf_em_batch_workspace_bytes(len(items), arr, ctypes.byref(b)))
    return b.value


def pmrf_em_batch(items, ws, stream=None):
    import torch

    arr = (EmItem * len(items))(*items)
    _check(lib.pmrf_em_batch(len(items), arr, _ptr(ws, torch.uint8, 0, "ws"), ws.numel(), _stream(stream, ws.device)))


def pmrf_set_launch(mode=0, waves_per_block=0, tiles_per_wave=0, blocks_per_cu=0):
    _check(lib.pmrf_set_launch(ctypes.byref(Launch(mode, waves_per_block, tiles_per_wave, blocks_per_cu))))


def pmrf_get_launch():
    out = Launch()
    _check(lib.pmrf_get_launch(ctypes.byref(out)))
    return {"mode": out.mode, "waves_per_block": out.waves_per_block, "tiles_per_wave": out.tiles_per_wave,
            "blocks_per_cu": out.blocks_per_cu}


def pmrf_launch_stats():
    """{captures, replays, direct}: runs since load that captured a HIP graph,
    replayed one from the cache, or launched directly."""
    c, r, d = c_int64(), c_int64(), c_int64()
    _check(lib.pmrf_launch_stats(ctypes.byref(c), ctypes.byref(r), ctypes.byref(d)))
    return {"captures": c.value, "replays": r.value, "direct": d.value}


def pmrf_profile_begin():
    _check(lib.pmrf_profile_begin())


def pmrf_profile_end():
    """(summed milliseconds, launches) of the bracketed EM-iteration launches."""
    ms, n = c_double(), c_int64()
    _check(lib.pmrf_profile_end(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# Launch shapes the autotuner tries: (mode, waves_per_block, tiles_per_wave,
# blocks_per_cu).  Graph replay with the automatic block size (one wave per
# chunk of a single graph's superchunks, 4 for a batch) and with 2, 4, 8 or 16
# waves per block, the persistent grid with 4 or 8 resident blocks per compute
# unit, and direct launches with the automatic and the 4-wave block.
AUTOTUNE_SHAPES = ((1, 0, 0, 0), (1, 4, 0, 0), (1, 2, 0, 0), (1, 8, 0, 0), (1, 16, 0, 0), (2, 4, 0, 4),
                   (2, 4, 0, 8), (3, 0, 0, 0), (3, 4, 0, 0))


def autotune_launch(run, shapes=AUTOTUNE_SHAPES, reps=3, sync=None, clock=time.perf_counter):
    """Pick the fastest launch shape for a workload and keep it selected.

    ``run()`` enqueues the work once (one pmrf_em_run or pmrf_em_batch on the
    device); ``sync()`` waits for the device (default: torch.cuda.synchronize).
    Every shape is tried once untimed (graph capture), then timed over ``reps``
    runs; the shape with the lowest mean time is set with pmrf_set_launch.
    Results do not depend on the launch shape (every reduction order is fixed
    by the graph), so this only changes speed.  Returns (best_shape,
    {shape: seconds per run})."""
    if sync is None:
        import torch

        sync = torch.cuda.synchronize
    timings = {}
    for shape in shapes:
        pmrf_set_launch(*shape)
        run()
        sync()
        t0 = clock()
        for _ in range(reps):
            run()
        sync()
        timings[tuple(shape)] = (clock() - t0) / reps
    best = min(timings, key=timings.get)
    pmrf_set_launch(*best)
    return best, timings


# --------------------------------------------------------------------------
# Convenience: one problem with its device buffers (allocation + marshalling)
# --------------------------------------------------------------------------
class Problem:
    """Device-resident state of one graph: neighbourhood layout, intensities,
    labels, parameters, outputs and workspace, all torch tensors."""

    def __init__(self, n, row_ptr, col_idx, y, L, device="cuda", hoods: Hoods | None = None):
        import torch

        self.hoods = hoods or pmrf_build_neighborhoods(n, row_ptr, col_idx)
        self.device = torch.device(device)
        self.n, self.L = int(n), int(L)
        self.hoodbuf = self.hoods.upload(self.device)
        self.y = torch.zeros(max(1, self.n), dtype=torch.float64, device=self.device)
        self.y[: self.n].copy_(torch.as_tensor(np.ascontiguousarray(y, dtype=np.float64)))
        # labels, mu and sigma are views of one buffer (`state`), so a caller
        # can save and restore the whole starting state with one copy
        n1 = max(1, self.n)
        off_mu = (4 * n1 + 255) // 256 * 256
        off_sg = off_mu + (8 * self.L + 255) // 256 * 256
        self.state = torch.zeros(off_sg + 8 * self.L, dtype=torch.uint8, device=self.device)
        self.labels = self.state[: 4 * n1].view(torch.int32)
        self.mu = self.state[off_mu: off_mu + 8 * self.L].view(torch.float64)
        self.sigma = self.state[off_sg: off_sg + 8 * self.L].view(torch.float64)
        self.sigma.fill_(1.0)
        self.hood_energy = torch.zeros(max(1, self.hoods.H), dtype=torch.float64, device=self.device)
        self.counters = torch.zeros(NCOUNTERS, dtype=torch.int64, device=self.device)
        self.trace = None
        self.iter_stats = None
        self.ws = None

    def set_state(self, labels, mu, sigma):
        import torch

        self.labels[: self.n].copy_(torch.as_tensor(np.ascontiguousarray(labels, dtype=np.int32)))
        self.mu.copy_(torch.as_tensor(np.asarray(mu, dtype=np.float64)))
        self.sigma.copy_(torch.as_tensor(np.asarray(sigma, dtype=np.float64)))

    def prepare(self, params: EmParams, workspace: bool = True):
        """Size the trace/statistics outputs (and, unless batched, the workspace)."""
        import torch

        T = max(1, params.max_iters)
        if self.trace is None or self.trace.numel() < T:
            self.trace = torch.zeros(T, dtype=torch.float64, device=self.device)
            self.iter_stats = torch.zeros(2 * T, dtype=torch.int64, device=self.device)
        if not workspace:
            return
        need = pmrf_em_workspace_bytes(self.hoods, params)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)

    def run(self, params: EmParams, stream=None):
        self.prepare(params)
        pmrf_em_run(self.hoods, self.hoodbuf, self.y, self.labels, self.mu, self.sigma, self.hood_energy,
                    self.trace, self.iter_stats, self.counters, self.ws, params, stream)

    def item(self, params: EmParams) -> EmItem:
        """Argument set of this problem for pmrf_em_batch (the batch brings its own workspace)."""
        self.prepare(params, workspace=False)
        return EmItem(self.hoods.handle.value, self.hoodbuf.data_ptr(), self.y.data_ptr(), self.labels.data_ptr(),
                      self.mu.data_ptr(), self.sigma.data_ptr(), self.hood_energy.data_ptr(), self.trace.data_ptr(),
                      self.iter_stats.data_ptr(), self.counters.data_ptr(), params)

    def results(self, params: EmParams):
        """Host copies of the outputs (synchronises)."""
        import torch

        torch.cuda.synchronize(self.device)
        c = self.counters.cpu().numpy()
        it = int(c[CTR_ITERS])
        return {
            "status": int(c[CTR_STATUS]), "iters": it, "map_conv_iter": int(c[CTR_MAP_CONV]),
            "em_conv_iter": int(c[CTR_EM_CONV]), "total_near_ties": int(c[CTR_NEAR_TIES]), "evals": int(c[CTR_EVALS]),
            "x": self.labels[: self.n].cpu().numpy(), "mu": self.mu.cpu().numpy(), "sigma": self.sigma.cpu().numpy(),
            "S": self.hood_energy[: self.hoods.H].cpu().numpy(), "trace": self.trace[:it].cpu().numpy(),
            "near_ties": self.iter_stats[0: 2 * it: 2].cpu().numpy(),
            "nonconv": self.iter_stats[1: 2 * it: 2].cpu().numpy(),
        }


def solve(n, row_ptr, col_idx, y, x0, mu0, sigma0, params: EmParams, device="cuda"):
    """Build, upload and run one problem; returns host results."""
    prob = Problem(n, row_ptr, col_idx, y, params.L, device)
    prob.set_state(x0, mu0, sigma0)
    prob.run(params)
    out = prob.results(params)
    if out["status"] != 0:
        raise PmrfError(out["status"], "device-reported error")
    return out


# ---------------------------------------------------------------- image in/out
def pmrf_image_graph_workspace_bytes(width, height, n) -> int:
    b = c_int64()
    _check(lib.pmrf_image_graph_workspace_bytes(int(width), int(height), int(n), ctypes.byref(b)))
    return b.value


def pmrf_volume_graph_workspace_bytes(width, height, depth, n) -> int:
    b = c_int64()
    _check(lib.pmrf_volume_graph_workspace_bytes(int(width), int(height), int(depth), int(n), ctypes.byref(b)))
    return b.value


_nnz_seen: dict = {}  # (width, height, depth, n) -> adjacency entries of the last call


def image_graph(regions, pixels, n, ws=None, stream=None):
    """Region adjacency graph and region means of an oversegmented image
    (``regions`` int32 and ``pixels`` uint8 device tensors of shape
    (height, width)) or volume (shape (depth, height, width), 6-connected);
    returns device tensors (row_ptr int32[n+1], col_idx int32[nnz], means
    float64[n])."""
    import torch

    shape = tuple(int(d) for d in regions.shape)
    if len(shape) not in (2, 3):
        raise ValueError("regions must be (height, width) or (depth, height, width)")
    depth, height, width = (1,) + shape if len(shape) == 2 else shape
    dev = regions.device
    _ptr(regions, torch.int32, depth * height * width, "regions")
    _ptr(pixels, torch.uint8, depth * height * width, "pixels")
    if ws is None:
        ws = torch.empty(pmrf_volume_graph_workspace_bytes(width, height, depth, n), dtype=torch.uint8, device=dev)
    s = _stream(stream, dev)
    row_ptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
    means = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    # First capacity: a 4-connected region graph is planar (at most 3n - 6
    # edges, 6n entries); regions of a volume meet about 14 others on average
    # (3-D cells), so 16n there.  The entry count of the last call with the
    # same shape is kept, so a repeated call never needs a second pass.
    key = (width, height, depth, int(n))
    cap = max(12, 6 * n if depth == 1 else 16 * n, _nnz_seen.get(key, 0))
    nnz = c_int64()
    while True:
        col = torch.empty(cap, dtype=torch.int32, device=dev)
        if len(shape) == 2:
            code = lib.pmrf_image_graph(regions.data_ptr(), pixels.data_ptr(), width, height, int(n),
                                        row_ptr.data_ptr(), col.data_ptr(), cap, means.data_ptr(), ctypes.byref(nnz),
                                        ws.data_ptr(), ws.numel(), s)
        else:
            code = lib.pmrf_volume_graph(regions.data_ptr(), pixels.data_ptr(), width, height, depth, int(n),
                                         row_ptr.data_ptr(), col.data_ptr(), cap, means.data_ptr(), ctypes.byref(nnz),
                                         ws.data_ptr(), ws.numel(), s)
        if code == PMRF_ENOMEM and nnz.value > cap:
            cap = nnz.value
            _nnz_seen[key] = cap
            continue
        _check(code)
        _nnz_seen[key] = max(_nnz_seen.get(key, 0), nnz.value)
        return row_ptr, col[: nnz.value], means[:n]


def labels_to_pixels(regions, labels, n, stream=None):
    """uint8 image of the labels of each pixel's region (device tensors)."""
    import torch

    _ptr(regions, torch.int32, regions.numel(), "regions")
    _ptr(labels, torch.int32, n, "labels")
    out = torch.empty(regions.shape, dtype=torch.uint8, device=regions.device)
    _check(lib.pmrf_labels_to_pixels(regions.data_ptr(), labels.data_ptr(), regions.numel(), int(n),
                                     out.data_ptr(), _stream(stream, regions.device)))
    return out


def confusion(a, b, k, stream=None):
    """int64 (k, k) device tensor: counts[i, j] = pixels with a = i and b = j."""
    import torch

    _ptr(a, torch.uint8, a.numel(), "a")
    _ptr(b, torch.uint8, a.numel(), "b")
    counts = torch.empty((k, k), dtype=torch.int64, device=a.device)
    _check(lib.pmrf_confusion(a.data_ptr(), b.data_ptr(), a.numel(), int(k), counts.data_ptr(),
                              _stream(stream, a.device)))
    return counts


def segmentation_scores(counts, positive=1, void=0):
    """The verification metrics of the paper (Sec. 4.2.1) from confusion
    counts (rows: segmentation, columns: ground truth): precision, recall and
    accuracy of the ``positive`` label, and the porosity of the segmentation
    (share of pixels labelled ``void``)."""
    c = np.asarray(counts, dtype=np.int64)
    total = int(c.sum())
    tp = int(c[positive, positive])
    fp = int(c[positive].sum()) - tp
    fn = int(c[:, positive].sum()) - tp
    tn = total - tp - fp - fn
    return {"precision": tp / (tp + fp) if tp + fp else float("nan"),
            "recall": tp / (tp + fn) if tp + fn else float("nan"),
            "accuracy": (tp + tn) / total if total else float("nan"),
            "porosity": int(c[void].sum()) / total if total else float("nan")}
