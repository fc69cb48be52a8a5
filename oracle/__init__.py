"""Python access to the serial FP64 oracle (``pmrf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``.  The product path (``paper_1809_05018_amd``)
never imports this package, and this package imports nothing from it.

``build()`` compiles the C source with gcc (``-O2 -ffp-contract=off``, no
fast-math).  ``load()`` builds only when no library is present.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from ctypes import POINTER, c_double, c_int, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pmrf_oracle.c")
# ORACLE_LIB names another build of the oracle (an instrumented one, say)
LIB = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

_lib = None


def build(extra_flags: tuple[str, ...] = (), out: str = LIB) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           *extra_flags, "-o", out + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _bind(lib):
    P = POINTER
    lib.or_build.restype = c_void_p
    lib.or_build.argtypes = [c_int, P(c_int), P(c_int)]
    lib.or_build_k.restype = c_void_p
    lib.or_build_k.argtypes = [c_int, P(c_int), P(c_int), c_int]
    lib.or_free.argtypes = [c_void_p]
    lib.or_info.argtypes = [c_void_p, P(c_int64)]
    lib.or_get_cliques.argtypes = [c_void_p, P(c_int64), P(c_int)]
    lib.or_get_hoods.argtypes = [c_void_p, P(c_int64), P(c_int)]
    lib.or_get_adjacency.argtypes = [c_void_p, P(c_int64), P(c_int)]
    lib.or_get_owner.argtypes = [c_void_p, P(c_int64)]
    lib.or_replicate.argtypes = [c_int, P(c_int64), c_int, P(c_int), P(c_int64), P(c_int)]
    lib.or_gather.argtypes = [c_int64, P(c_int64), P(c_int), P(c_int), P(c_double), P(c_int), P(c_double)]
    lib.or_mstep.restype = c_int
    lib.or_mstep.argtypes = [c_int, P(c_double), c_int, P(c_int), P(c_double), P(c_double), c_double,
                             P(c_double), P(c_double)]
    lib.or_em_step.restype = c_int
    lib.or_em_step.argtypes = [c_void_p, P(c_double), c_int, c_double, c_int, P(c_int), P(c_double), P(c_double),
                               c_double, c_double, P(c_int), P(c_double), P(c_double), P(c_double),
                               P(c_double), P(c_int64), P(c_double), P(c_int), P(c_double)]
    lib.or_hood_converged.restype = c_int
    lib.or_hood_converged.argtypes = [c_int, c_double, P(c_double)]
    lib.or_em_run.restype = c_int
    lib.or_em_run.argtypes = [c_void_p, P(c_double), c_int, c_double, c_int, c_int, c_int, c_double, c_int,
                              c_double, c_double, c_int, P(c_int), P(c_double), P(c_double), P(c_double),
                              P(c_double), P(c_int64), P(c_int64), P(c_int64)]
    return lib


def load(path: str | None = None):
    """Load the oracle library, compiling it first only if none is built."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _bind(ctypes.CDLL(LIB))
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(POINTER(ct))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# Scatter rules of the label update ("Update Output Labels"): which element's
# write stands for a vertex that several neighbourhoods hold.
RULE_OWNER, RULE_LAST, RULE_MIN = 0, 1, 2


class OracleGraph:
    """Neighbourhood structure built by the oracle from a CSR graph (k-neighbourhoods)."""

    def __init__(self, n, row_ptr, col_idx, lib=None, k=1):
        self.lib = lib or load()
        self.row_ptr = _i32(row_ptr)
        self.col_idx = _i32(col_idx) if len(col_idx) else np.zeros(1, np.int32)
        self.k = int(k)
        self.h = self.lib.or_build_k(int(n), _p(self.row_ptr, c_int), _p(self.col_idx, c_int), self.k)
        if not self.h:
            raise ValueError("oracle: invalid CSR graph")
        info = np.zeros(6, np.int64)
        self.lib.or_info(self.h, _p(info, c_int64))
        self.n, self.H, self.M, self.A, self.max_hood, self.clique_members = (int(v) for v in info)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.or_free(self.h)
            self.h = None

    def cliques(self):
        ptr = np.zeros(self.H + 1, np.int64)
        vid = np.zeros(max(1, self.clique_members), np.int32)
        self.lib.or_get_cliques(self.h, _p(ptr, c_int64), _p(vid, c_int))
        return ptr, vid[: self.clique_members]

    def hoods(self):
        ptr = np.zeros(self.H + 1, np.int64)
        vid = np.zeros(max(1, self.M), np.int32)
        self.lib.or_get_hoods(self.h, _p(ptr, c_int64), _p(vid, c_int))
        return ptr, vid[: self.M]

    def adjacency(self):
        ptr = np.zeros(self.M + 1, np.int64)
        loc = np.zeros(max(1, self.A), np.int32)
        self.lib.or_get_adjacency(self.h, _p(ptr, c_int64), _p(loc, c_int))
        return ptr, loc[: self.A]

    def owner(self):
        own = np.zeros(max(1, self.n), np.int64)
        self.lib.or_get_owner(self.h, _p(own, c_int64))
        return own[: self.n]

    def em_step(self, y, L, beta, x, mu, sigma, sigma_min=1e-3, tie_eps=1e-9, per_element=False, rule=RULE_OWNER):
        y, x, mu, sigma = _f64(y), _i32(x), _f64(mu), _f64(sigma)
        xo = np.zeros(max(1, self.n), np.int32)
        muo, so = np.zeros(L), np.zeros(L)
        S = np.zeros(max(1, self.H))
        T = np.zeros(1)
        nt = np.zeros(1, np.int64)
        M = max(1, self.M)
        m = np.zeros(M) if per_element else None
        a = np.zeros(M, np.int32) if per_element else None
        gap = np.zeros(M) if per_element else None
        nul_d = ctypes.cast(None, POINTER(c_double))
        nul_i = ctypes.cast(None, POINTER(c_int))
        rc = self.lib.or_em_step(self.h, _p(y, c_double), int(L), float(beta), int(rule), _p(x, c_int), _p(mu, c_double),
                                 _p(sigma, c_double), float(sigma_min), float(tie_eps), _p(xo, c_int),
                                 _p(muo, c_double), _p(so, c_double), _p(S, c_double), _p(T, c_double),
                                 _p(nt, c_int64), _p(m, c_double) if per_element else nul_d,
                                 _p(a, c_int) if per_element else nul_i,
                                 _p(gap, c_double) if per_element else nul_d)
        if rc != 0:
            raise ValueError("oracle: em_step rejected its arguments")
        out = {"x": xo[: self.n], "mu": muo, "sigma": so, "S": S[: self.H], "T": float(T[0]),
               "near_ties": int(nt[0])}
        if per_element:
            out.update(m=m[: self.M], a=a[: self.M], gap=gap[: self.M])
        return out

    def em_run(self, y, L, beta, x0, mu0, sigma0, iters, window=3, tol=1e-4, early_exit=False,
               sigma_min=1e-3, tie_eps=1e-9, init_from_labels=False, rule=RULE_OWNER):
        y = _f64(y)
        x = _i32(x0).copy()
        if x.size == 0:
            x = np.zeros(1, np.int32)
        mu, sigma = _f64(mu0).copy(), _f64(sigma0).copy()
        trace = np.zeros(max(1, iters))
        S = np.zeros(max(1, self.H))
        nt = np.zeros(max(1, iters), np.int64)
        nc = np.zeros(max(1, iters), np.int64)
        summ = np.zeros(4, np.int64)
        rc = self.lib.or_em_run(self.h, _p(y, c_double), int(L), float(beta), int(rule), int(iters), int(window), float(tol),
                                int(bool(early_exit)), float(sigma_min), float(tie_eps), int(bool(init_from_labels)),
                                _p(x, c_int), _p(mu, c_double), _p(sigma, c_double), _p(trace, c_double),
                                _p(S, c_double), _p(nt, c_int64), _p(nc, c_int64), _p(summ, c_int64))
        if rc != 0:
            raise ValueError("oracle: em_run rejected its arguments")
        it = int(summ[0])
        return {"x": x[: self.n], "mu": mu, "sigma": sigma, "trace": trace[:it], "S": S[: self.H],
                "near_ties": nt[:it], "nonconv": nc[:it], "iters": it, "map_conv_iter": int(summ[1]),
                "em_conv_iter": int(summ[2]), "total_near_ties": int(summ[3])}


def replicate(hood_ptr, L, lib=None):
    lib = lib or load()
    hood_ptr = np.ascontiguousarray(hood_ptr, dtype=np.int64)
    H = hood_ptr.size - 1
    K = int(hood_ptr[-1]) * L
    tl = np.zeros(max(1, K), np.int32)
    oi = np.zeros(max(1, K), np.int64)
    hi = np.zeros(max(1, K), np.int32)
    lib.or_replicate(H, _p(hood_ptr, c_int64), int(L), _p(tl, c_int), _p(oi, c_int64), _p(hi, c_int))
    return tl[:K], oi[:K], hi[:K]


def gather(old_index, hood_vid, x, y, lib=None):
    lib = lib or load()
    old_index = np.ascontiguousarray(old_index, dtype=np.int64)
    hood_vid, x, y = _i32(hood_vid), _i32(x), _f64(y)
    K = old_index.size
    vl = np.zeros(max(1, K), np.int32)
    vm = np.zeros(max(1, K))
    lib.or_gather(K, _p(old_index, c_int64), _p(hood_vid, c_int), _p(x, c_int), _p(y, c_double),
                  _p(vl, c_int), _p(vm, c_double))
    return vl[:K], vm[:K]


def mstep(y, L, x, mu_in, sigma_in, sigma_min=1e-3, lib=None):
    lib = lib or load()
    y, x, mu_in, sigma_in = _f64(y), _i32(x), _f64(mu_in), _f64(sigma_in)
    mu, sg = np.zeros(L), np.zeros(L)
    lib.or_mstep(int(y.size), _p(y, c_double), int(L), _p(x, c_int), _p(mu_in, c_double), _p(sigma_in, c_double),
                 float(sigma_min), _p(mu, c_double), _p(sg, c_double))
    return mu, sg


def hood_converged(hist, tol, lib=None):
    lib = lib or load()
    hist = _f64(hist)
    return bool(lib.or_hood_converged(int(hist.size - 1), float(tol), _p(hist, c_double)))
