"""Python access to the Moss oracle (plain C reference in moss_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this module.  The GPU library never imports or links it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "moss_oracle.c")
_LIB = os.path.join(_HERE, "libmoss_oracle.so")

OK = 0
E_ARG, E_UNSORTED, E_SELF_LOOP, E_DUPLICATE, E_ASYMMETRIC, E_OVERFLOW, E_NOMEM = -1, -2, -3, -4, -5, -6, -7
MOSS4, MOSS4MIN, T5, PATH5 = 4, 0x41, 0x51, 0x52
MIX_POOLED, MIX_PAPER = 0, 1

TAB_S, TAB_Q, TAB_GAMMA, TAB_GAMMA1, TAB_GAMMA2 = 0, 1, 2, 3, 4
TAB_ACC_GAMMA, TAB_ACC_GAMMA1, TAB_ACC_GAMMA2, TAB_ACC_SIGMA, TAB_ACC_TAU = 5, 6, 7, 8, 9
TAB_GAMMA_MIN, TAB_ACC_GAMMA_MIN, TAB_ACC_CHECK, TAB_RANK, TAB_RANK_MIRROR, TAB_COL_RANK = 10, 11, 12, 13, 14, 15

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _Totals(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_uint64), ("gamma1", ctypes.c_uint64), ("gamma2", ctypes.c_uint64),
                ("lambda3", ctypes.c_uint64), ("lambda4", ctypes.c_uint64), ("gamma_min", ctypes.c_uint64),
                ("min_status", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n_motifs", ctypes.c_int32), ("K", ctypes.c_uint64 * 2),
                ("hits", (ctypes.c_uint64 * 22) * 2), ("estimate", ctypes.c_double * 21),
                ("variance", ctypes.c_double * 21)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            u64, i64, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32
            L.orc_build.argtypes = [i32, i64, P, P, ctypes.c_int, ctypes.POINTER(P)]
            L.orc_free.argtypes = [P]
            L.orc_totals_get.argtypes = [P, ctypes.POINTER(_Totals)]
            L.orc_table.argtypes = [P, ctypes.c_int, P]
            L.orc_philox4x64_10.argtypes = [P, P, P]
            L.orc_bounded.argtypes = [u64, u64]
            L.orc_bounded.restype = u64
            L.orc_pick_u64.argtypes = [P, i64, u64]
            L.orc_pick_u64.restype = i64
            L.orc_classify.argtypes = [ctypes.c_int, P]
            L.orc_sample.argtypes = [P, ctypes.c_int, u64, u64, P]
            L.orc_run.argtypes = [P, ctypes.c_int, u64, u64, u64, ctypes.c_int, P]
            L.orc_finals4.argtypes = [u64, P, u64, u64, P, P]
            L.orc_finals5.argtypes = [u64, u64, P, P, u64, u64, u64, ctypes.c_int, P, P, P]
            L.orc_finals4min.argtypes = [u64, P, u64, u64, u64, P, u64, ctypes.c_int, P, P]
            L.orc_ways_of.argtypes = [P, P]
            L.orc_estimate4min.argtypes = [P, u64, u64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Result)]
            L.orc_normal_two_sided.argtypes = [ctypes.c_double]
            L.orc_normal_two_sided.restype = ctypes.c_double
            L.orc_plan_budget.argtypes = [ctypes.POINTER(_Result), ctypes.c_double, ctypes.c_double, ctypes.c_uint32,
                                          P, ctypes.POINTER(u64)]
            L.orc_concentrations.argtypes = [ctypes.POINTER(_Result), P]
            L.orc_estimate_to_precision.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_uint32, u64, u64, u64, u64, ctypes.c_int, ctypes.c_int,
                                                    ctypes.POINTER(_Result), ctypes.POINTER(u64)]
            L.orc_estimate.argtypes = [P, ctypes.c_int, u64, u64, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(_Result)]
            L.orc_count_cis.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
            L.orc_count4_exact.argtypes = [P, P]
            L.orc_line_count.argtypes = [P, ctypes.c_int, u64, u64, u64, ctypes.POINTER(ctypes.c_double)]
            _lib = L
        return _lib


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox(counter, key) -> np.ndarray:
    c = np.asarray(counter, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def bounded(x: int, n: int) -> int:
    return int(lib().orc_bounded(x, n))


def pick(acc, x: int) -> int:
    a = np.ascontiguousarray(acc, dtype=np.uint64)
    return int(lib().orc_pick_u64(_ptr(a), a.shape[0], x))


def classify(k: int, adj) -> int:
    a = np.ascontiguousarray(np.asarray(adj, dtype=np.uint8).reshape(k, k))
    return int(lib().orc_classify(k, _ptr(a)))


class Result:
    def __init__(self, r: _Result):
        self.raw = r
        self.k = r.k
        self.n_motifs = r.n_motifs
        self.K = [int(r.K[0]), int(r.K[1])]
        self.hits = np.array([[r.hits[s][i] for i in range(22)] for s in range(2)], dtype=np.uint64)
        self.estimate = np.array(r.estimate[: r.n_motifs], dtype=np.float64)
        self.variance = np.array(r.variance[: r.n_motifs], dtype=np.float64)


class Graph:
    """Oracle tables for one CSR graph (copied)."""

    def __init__(self, csr, validate: bool = True):
        L = lib()
        self.n, self.nnz = csr.n, csr.nnz
        self._rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int32)
        self._col = np.ascontiguousarray(csr.col, dtype=np.int32)
        h = ctypes.c_void_p()
        st = L.orc_build(self.n, self.nnz, _ptr(self._rp), _ptr(self._col), int(validate), ctypes.byref(h))
        if st != OK:
            raise OracleError(st, "orc_build")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            try:
                _lib.orc_free(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    def totals(self) -> dict:
        t = _Totals()
        lib().orc_totals_get(self._h, ctypes.byref(t))
        return dict(gamma=t.gamma, gamma1=t.gamma1, gamma2=t.gamma2, lambda3=t.lambda3, lambda4=t.lambda4,
                    gamma_min=t.gamma_min, min_status=t.min_status)

    def table(self, which: int) -> np.ndarray:
        if which in (TAB_ACC_SIGMA, TAB_RANK, TAB_RANK_MIRROR):
            out = np.zeros(self.nnz, np.uint32)
        elif which == TAB_COL_RANK:
            out = np.zeros(self.nnz, np.int32)
        elif which in (TAB_ACC_TAU, TAB_ACC_CHECK):
            out = np.zeros(self.nnz, np.uint64)
        else:
            out = np.zeros(self.n, np.uint64)
        st = lib().orc_table(self._h, which, _ptr(out))
        if st != OK:
            raise OracleError(st, "orc_table")
        return out

    def sample(self, sampler: int, seed: int, k: int):
        nodes = np.zeros(5, np.int32)
        c = lib().orc_sample(self._h, sampler, seed, k, _ptr(nodes))
        if c < 0:
            raise OracleError(c, "orc_sample")
        return c, [int(x) for x in nodes]

    def run(self, sampler: int, seed: int, k0: int, k1: int, threads: int = 1) -> np.ndarray:
        hits = np.zeros(22, np.uint64)
        st = lib().orc_run(self._h, sampler, seed, k0, k1, threads, _ptr(hits))
        if st != OK:
            raise OracleError(st, "orc_run")
        return hits

    def estimate(self, k: int, n_samples: int, seed: int, mix: int = MIX_POOLED, threads: int = 1) -> Result:
        r = _Result()
        st = lib().orc_estimate(self._h, k, n_samples, seed, mix, threads, ctypes.byref(r))
        if st != OK:
            raise OracleError(st, "orc_estimate")
        return Result(r)

    def estimate4min(self, n_samples: int, seed: int, mix: int = MIX_POOLED, threads: int = 1) -> Result:
        r = _Result()
        st = lib().orc_estimate4min(self._h, n_samples, seed, mix, threads, ctypes.byref(r))
        if st != OK:
            raise OracleError(st, "orc_estimate4min")
        return Result(r)

    def estimate_to_precision(self, k: int, eps: float, delta: float, motif_mask: int, pilot_samples: int,
                              pilot_seed: int, max_samples: int, seed: int, with_min: bool = False,
                              mix: int = MIX_POOLED, threads: int = 1):
        r = _Result()
        K = ctypes.c_uint64()
        st = lib().orc_estimate_to_precision(self._h, k, int(with_min), eps, delta, motif_mask, pilot_samples,
                                             pilot_seed, max_samples, seed, mix, threads, ctypes.byref(r),
                                             ctypes.byref(K))
        if st != OK:
            raise OracleError(st, "orc_estimate_to_precision")
        return Result(r), int(K.value)

    def count_cis(self, k: int, threads: int = 1) -> np.ndarray:
        out = np.zeros(22, np.uint64)
        st = lib().orc_count_cis(self._h, k, threads, _ptr(out))
        if st != OK:
            raise OracleError(st, "orc_count_cis")
        return out

    def count4_exact(self) -> np.ndarray:
        out = np.zeros(7, np.uint64)
        st = lib().orc_count4_exact(self._h, _ptr(out))
        if st != OK:
            raise OracleError(st, "orc_count4_exact")
        return out

    def line_count(self, sampler: int, seed: int, k0: int, k1: int) -> float:
        v = ctypes.c_double()
        st = lib().orc_line_count(self._h, sampler, seed, k0, k1, ctypes.byref(v))
        if st != OK:
            raise OracleError(st, "orc_line_count")
        return float(v.value)


def finals4(K: int, hits, gamma: int, lambda3: int):
    h = np.ascontiguousarray(np.asarray(hits, dtype=np.uint64)[:7])
    est = np.zeros(6)
    var = np.zeros(6)
    st = lib().orc_finals4(K, _ptr(h), gamma, lambda3, _ptr(est), _ptr(var))
    if st != OK:
        raise OracleError(st, "orc_finals4")
    return est, var


def finals5(K1: int, K2: int, hits1, hits2, gamma1: int, gamma2: int, lambda4: int, mix: int = MIX_POOLED):
    h1 = np.ascontiguousarray(np.asarray(hits1, dtype=np.uint64)[:22])
    h2 = np.ascontiguousarray(np.asarray(hits2, dtype=np.uint64)[:22])
    est = np.zeros(21)
    var = np.zeros(21)
    cov = np.zeros(21 * 21)
    st = lib().orc_finals5(K1, K2, _ptr(h1), _ptr(h2), gamma1, gamma2, lambda4, mix, _ptr(est), _ptr(var),
                           _ptr(cov))
    if st != OK:
        raise OracleError(st, "orc_finals5")
    return est, var, cov.reshape(21, 21)


def finals4min(K: int, hits, gamma: int, lambda3: int, Kc: int, hits_min, gamma_min: int, mix: int = MIX_POOLED):
    h = np.ascontiguousarray(np.asarray(hits, dtype=np.uint64)[:7])
    hm = np.ascontiguousarray(np.asarray(hits_min, dtype=np.uint64)[:10])
    est = np.zeros(6)
    var = np.zeros(6)
    st = lib().orc_finals4min(K, _ptr(h), gamma, lambda3, Kc, _ptr(hm), gamma_min, mix, _ptr(est), _ptr(var))
    if st != OK:
        raise OracleError(st, "orc_finals4min")
    return est, var


def ways_of(adj, keys) -> int:
    """Ordered MOSS-4Min draws (w, v, u, r) that give a 4-node set (adjacency 4x4, order keys)."""
    a = np.ascontiguousarray(np.asarray(adj, dtype=np.uint8).reshape(16))
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64).reshape(4))
    return int(lib().orc_ways_of(_ptr(a), _ptr(k)))


def normal_two_sided(delta: float) -> float:
    return float(lib().orc_normal_two_sided(delta))


def plan_budget(pilot: Result, eps: float, delta: float, motif_mask: int = 0):
    """(per-motif budgets, largest over the mask) from a pilot result."""
    b = np.zeros(21, np.uint64)
    mx = ctypes.c_uint64()
    st = lib().orc_plan_budget(ctypes.byref(pilot.raw), eps, delta, motif_mask, _ptr(b), ctypes.byref(mx))
    if st != OK:
        raise OracleError(st, "orc_plan_budget")
    return b[: pilot.n_motifs], int(mx.value)


def concentrations(r: Result) -> np.ndarray:
    out = np.zeros(21)
    st = lib().orc_concentrations(ctypes.byref(r.raw), _ptr(out))
    if st != OK:
        raise OracleError(st, "orc_concentrations")
    return out[: r.n_motifs]
