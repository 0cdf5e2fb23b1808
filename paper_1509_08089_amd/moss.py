"""ctypes binding of libmoss.so (include/moss.h).

Functions carry the C ABI's names and only marshal arguments: every step of the
estimate runs in the library's HIP kernels and host code.  PyTorch provides device
memory and streams.  There is no fallback: if the library is missing or no GPU is
usable, calls fail loudly.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmoss.so")

OK = 0
STATUS = {
    0: "MOSS_OK", -1: "MOSS_E_ARG", -2: "MOSS_E_UNSORTED", -3: "MOSS_E_SELF_LOOP", -4: "MOSS_E_DUPLICATE",
    -5: "MOSS_E_ASYMMETRIC", -6: "MOSS_E_OVERFLOW", -7: "MOSS_E_NOMEM", -8: "MOSS_E_DEVICE",
    -9: "MOSS_E_NOT_BUILT", -10: "MOSS_E_BUSY", -11: "MOSS_E_TIMEOUT", -12: "MOSS_E_CANCELLED",
    -13: "MOSS_E_ADMISSION", -14: "MOSS_E_TOO_LARGE",
}
globals().update({v: k for k, v in STATUS.items()})

MOSS_SAMPLER_MOSS4, MOSS_SAMPLER_MOSS4MIN, MOSS_SAMPLER_T5, MOSS_SAMPLER_PATH5 = 0x4, 0x41, 0x51, 0x52
MOSS_SCHEDULE_AUTO, MOSS_SCHEDULE_PLAIN, MOSS_SCHEDULE_XCD = 0, 1, 2
MOSS_TRUST_CSR = 0x1
MOSS_MIX_POOLED, MOSS_MIX_PAPER, MOSS_K4_MIN = 0x0, 0x1, 0x2
MOSS_TABLES_K4, MOSS_TABLES_K5, MOSS_TABLES_K4MIN = 1 << 4, 1 << 5, 1 << 6
MOSS_TAB_ACC_GAMMA, MOSS_TAB_ACC_GAMMA1, MOSS_TAB_ACC_GAMMA2, MOSS_TAB_ACC_SIGMA, MOSS_TAB_ACC_TAU = 5, 6, 7, 8, 9
MOSS_TAB_ACC_GAMMA_MIN, MOSS_TAB_ACC_CHECK, MOSS_TAB_RANK, MOSS_TAB_COL_RANK = 11, 12, 13, 15
MOSS_TAB_SIGMA_GUIDE, MOSS_TAB_TAU_GUIDE, MOSS_TAB_CHECK_GUIDE = 16, 17, 18
MOSS_NOALLOC_MAX_SAMPLES, MOSS_NOALLOC_SCRATCH_BYTES = 1 << 22, 32 << 20

# every symbol include/moss.h declares
EXPORTED = [
    "moss_status_string", "moss_graph_create", "moss_graph_create_device", "moss_graph_destroy",
    "moss_build_tables", "moss_graph_get_info", "moss_table_read", "moss_estimate", "moss_sample_range",
    "moss_sample_nodes", "moss_class_lut", "moss_finals", "moss_estimate_batch", "moss_set_tuning",
    "moss_get_tuning", "moss_autotune", "moss_server_create", "moss_server_add_graph", "moss_server_submit",
    "moss_server_wait", "moss_server_cancel", "moss_server_stats_get", "moss_server_destroy",
    "moss_plan_budget", "moss_estimate_to_precision", "moss_concentrations", "moss_sample_range_noalloc",
]


class MossError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)}")
        self.status = status


class moss_graph_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("max_degree", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("built_mask", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("gamma", ctypes.c_uint64),
                ("gamma1", ctypes.c_uint64), ("gamma2", ctypes.c_uint64), ("lambda3", ctypes.c_uint64),
                ("lambda4", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64), ("gamma_min", ctypes.c_uint64),
                ("sampling_bytes", ctypes.c_uint64)]


class moss_result(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n_motifs", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_int32), ("n_samples", ctypes.c_uint64), ("K", ctypes.c_uint64 * 2),
                ("hits", (ctypes.c_uint64 * 22) * 2), ("gamma", ctypes.c_uint64 * 2), ("lambda_", ctypes.c_uint64),
                ("estimate", ctypes.c_double * 21), ("variance", ctypes.c_double * 21),
                ("device_ms", ctypes.c_double)]

    @property
    def hits_np(self) -> np.ndarray:
        return np.array([[self.hits[s][i] for i in range(22)] for s in range(2)], dtype=np.uint64)

    @property
    def estimate_np(self) -> np.ndarray:
        return np.array(self.estimate[: self.n_motifs], dtype=np.float64)

    @property
    def variance_np(self) -> np.ndarray:
        return np.array(self.variance[: self.n_motifs], dtype=np.float64)


class moss_request(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("k", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("n_samples", ctypes.c_uint64), ("seed", ctypes.c_uint64)]


class moss_tuning(ctypes.Structure):
    _fields_ = [("tile_samples", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("threads_per_block", ctypes.c_uint32), ("schedule", ctypes.c_uint32),
                ("group_min_samples_log2", ctypes.c_uint32), ("group_min_footprint_mb", ctypes.c_uint32),
                ("sort_window", ctypes.c_uint32)]


class moss_server_config(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_uint32),
                ("express_off", ctypes.c_uint32), ("chunk_samples", ctypes.c_uint64),
                ("iteration_samples", ctypes.c_uint64), ("express_samples", ctypes.c_uint64)]


class moss_server_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("samples", ctypes.c_uint64), ("iterations", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("active", ctypes.c_uint64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("samples_per_s", ctypes.c_double), ("table_bytes", ctypes.c_uint64),
                ("evictions", ctypes.c_uint64), ("express_launches", ctypes.c_uint64)]


_lock = threading.Lock()
_lib = None


def lib():
    """Loads libmoss.so (built by paper_1509_08089_amd.build); raises if it is missing."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1509_08089_amd.build` "
                              "(hipcc --offload-arch=gfx950); there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, u32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint64
        PP = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "moss_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "moss_graph_create": ([i32, i64, P, P, u32, P, PP], ctypes.c_int),
            "moss_graph_create_device": ([i32, i64, P, P, u32, P, PP], ctypes.c_int),
            "moss_graph_destroy": ([P], ctypes.c_int),
            "moss_build_tables": ([P, u32], ctypes.c_int),
            "moss_graph_get_info": ([P, ctypes.POINTER(moss_graph_info)], ctypes.c_int),
            "moss_table_read": ([P, i32, P, i64], ctypes.c_int),
            "moss_estimate": ([P, i32, u64, u64, u32, ctypes.POINTER(moss_result)], ctypes.c_int),
            "moss_sample_range": ([P, i32, u64, u64, u64, P, P], ctypes.c_int),
            "moss_sample_range_noalloc": ([P, i32, u64, u64, u64, P, P], ctypes.c_int),
            "moss_sample_nodes": ([P, i32, u64, P, i64, P, P], ctypes.c_int),
            "moss_class_lut": ([i32, P, i32], ctypes.c_int),
            "moss_finals": ([ctypes.POINTER(moss_result)], ctypes.c_int),
            "moss_plan_budget": ([ctypes.POINTER(moss_result), ctypes.c_double, ctypes.c_double, u32, P,
                                  ctypes.POINTER(u64)], ctypes.c_int),
            "moss_estimate_to_precision": ([P, i32, ctypes.c_double, ctypes.c_double, u32, u64, u64, u64, u64, u32,
                                            ctypes.POINTER(moss_result)], ctypes.c_int),
            "moss_concentrations": ([ctypes.POINTER(moss_result), P], ctypes.c_int),
            "moss_estimate_batch": ([P, i32, P, P], ctypes.c_int),
            "moss_set_tuning": ([ctypes.POINTER(moss_tuning)], ctypes.c_int),
            "moss_get_tuning": ([ctypes.POINTER(moss_tuning)], ctypes.c_int),
            "moss_autotune": ([P, i32, ctypes.POINTER(moss_tuning), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "moss_server_create": ([ctypes.POINTER(moss_server_config), P, PP], ctypes.c_int),
            "moss_server_add_graph": ([P, P, ctypes.POINTER(i32)], ctypes.c_int),
            "moss_server_submit": ([P, i32, i32, u64, u64, u32, ctypes.POINTER(u64)], ctypes.c_int),
            "moss_server_wait": ([P, u64, i64, ctypes.POINTER(moss_result)], ctypes.c_int),
            "moss_server_cancel": ([P, u64], ctypes.c_int),
            "moss_server_stats_get": ([P, ctypes.POINTER(moss_server_stats)], ctypes.c_int),
            "moss_server_destroy": ([P], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
        return L


def _check(status: int, what: str):
    if status != OK:
        raise MossError(status, what)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _hptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---- thin wrappers with the C names -------------------------------------------------
def moss_status_string(status: int) -> str:
    return lib().moss_status_string(status).decode()


def moss_graph_create(n: int, nnz: int, row_ptr: np.ndarray, col: np.ndarray, flags: int = 0, stream=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(lib().moss_graph_create(n, nnz, _hptr(rp), _hptr(cl), flags, _stream(stream), ctypes.byref(h)),
           "moss_graph_create")
    return h


def moss_graph_create_device(n: int, nnz: int, d_row_ptr, d_col, flags: int = 0, stream=None):
    h = ctypes.c_void_p()
    _check(lib().moss_graph_create_device(n, nnz, _dptr(d_row_ptr), _dptr(d_col), flags, _stream(stream),
                                          ctypes.byref(h)), "moss_graph_create_device")
    return h


def moss_graph_destroy(g):
    _check(lib().moss_graph_destroy(g), "moss_graph_destroy")


def moss_build_tables(g, k_mask: int):
    _check(lib().moss_build_tables(g, k_mask), "moss_build_tables")


def moss_graph_get_info(g) -> moss_graph_info:
    info = moss_graph_info()
    _check(lib().moss_graph_get_info(g, ctypes.byref(info)), "moss_graph_get_info")
    return info


def moss_table_read(g, which: int, count: int) -> np.ndarray:
    """One table as a numpy array (MOSS_TAB_RANK: count x 2 u32 pairs)."""
    if which == MOSS_TAB_RANK:
        out = np.zeros((count, 2), np.uint32)
    else:
        dtype = {MOSS_TAB_ACC_SIGMA: np.uint32, MOSS_TAB_COL_RANK: np.int32, MOSS_TAB_SIGMA_GUIDE: np.uint32,
                 MOSS_TAB_TAU_GUIDE: np.uint32, MOSS_TAB_CHECK_GUIDE: np.uint32}.get(which, np.uint64)
        out = np.zeros(count, dtype)
    _check(lib().moss_table_read(g, which, _hptr(out), count), "moss_table_read")
    return out


def moss_estimate(g, k: int, n_samples: int, seed: int, flags: int = 0) -> moss_result:
    r = moss_result()
    _check(lib().moss_estimate(g, k, n_samples, seed, flags, ctypes.byref(r)), "moss_estimate")
    return r


def moss_sample_range(g, sampler: int, seed: int, k0: int, k1: int, d_class_out=None) -> np.ndarray:
    hits = np.zeros(22, np.uint64)
    _check(lib().moss_sample_range(g, sampler, seed, k0, k1, _dptr(d_class_out), _hptr(hits)), "moss_sample_range")
    return hits


def moss_sample_range_noalloc(g, sampler: int, seed: int, k0: int, k1: int, d_class_out=None) -> np.ndarray:
    hits = np.zeros(22, np.uint64)
    _check(lib().moss_sample_range_noalloc(g, sampler, seed, k0, k1, _dptr(d_class_out), _hptr(hits)),
           "moss_sample_range_noalloc")
    return hits


def moss_sample_nodes(g, sampler: int, seed: int, d_index, d_nodes_out, d_class_out=None):
    _check(lib().moss_sample_nodes(g, sampler, seed, _dptr(d_index), int(d_index.numel()), _dptr(d_nodes_out),
                                   _dptr(d_class_out)), "moss_sample_nodes")


def moss_class_lut(sampler: int) -> np.ndarray:
    n = 8 if sampler in (MOSS_SAMPLER_MOSS4, MOSS_SAMPLER_MOSS4MIN) else 64
    out = np.zeros(n, np.uint8)
    _check(lib().moss_class_lut(sampler, _hptr(out), n), "moss_class_lut")
    return out


def moss_finals(r: moss_result) -> moss_result:
    _check(lib().moss_finals(ctypes.byref(r)), "moss_finals")
    return r


def moss_plan_budget(pilot: moss_result, eps: float, delta: float, motif_mask: int = 0):
    """(per-motif budgets, largest over the mask)."""
    b = np.zeros(21, np.uint64)
    mx = ctypes.c_uint64()
    _check(lib().moss_plan_budget(ctypes.byref(pilot), eps, delta, motif_mask, _hptr(b), ctypes.byref(mx)),
           "moss_plan_budget")
    return b[: pilot.n_motifs], int(mx.value)


def moss_estimate_to_precision(g, k: int, eps: float, delta: float, motif_mask: int, pilot_samples: int,
                               pilot_seed: int, max_samples: int, seed: int, flags: int = 0) -> moss_result:
    r = moss_result()
    _check(lib().moss_estimate_to_precision(g, k, eps, delta, motif_mask, pilot_samples, pilot_seed, max_samples,
                                            seed, flags, ctypes.byref(r)), "moss_estimate_to_precision")
    return r


def moss_concentrations(r: moss_result) -> np.ndarray:
    out = np.zeros(21)
    _check(lib().moss_concentrations(ctypes.byref(r), _hptr(out)), "moss_concentrations")
    return out[: r.n_motifs]


def moss_estimate_batch(requests, stream=None):
    """requests: sequence of (graph_handle, k, n_samples, seed, flags)."""
    n = len(requests)
    reqs = (moss_request * max(n, 1))()
    for i, (g, k, ns, seed, flags) in enumerate(requests):
        reqs[i].g = g.value if isinstance(g, ctypes.c_void_p) else g
        reqs[i].k, reqs[i].n_samples, reqs[i].seed, reqs[i].flags = k, ns, seed, flags
    out = (moss_result * max(n, 1))()
    _check(lib().moss_estimate_batch(ctypes.cast(reqs, ctypes.c_void_p), n, ctypes.cast(out, ctypes.c_void_p),
                                     _stream(stream)), "moss_estimate_batch")
    return [out[i] for i in range(n)]


def _requests(requests):
    n = len(requests)
    reqs = (moss_request * max(n, 1))()
    for i, (g, k, ns, seed, flags) in enumerate(requests):
        reqs[i].g = g.value if isinstance(g, ctypes.c_void_p) else g
        reqs[i].k, reqs[i].n_samples, reqs[i].seed, reqs[i].flags = k, ns, seed, flags
    return reqs, n


def moss_set_tuning(tile_samples: int = 0, blocks_per_cu: int = 0, threads_per_block: int = 0, schedule: int = 0,
                    group_min_samples_log2: int = 0, group_min_footprint_mb: int = 0, sort_window: int = 0):
    t = moss_tuning(tile_samples, blocks_per_cu, threads_per_block, schedule, group_min_samples_log2,
                    group_min_footprint_mb, sort_window)
    _check(lib().moss_set_tuning(ctypes.byref(t)), "moss_set_tuning")


def moss_get_tuning() -> moss_tuning:
    t = moss_tuning()
    _check(lib().moss_get_tuning(ctypes.byref(t)), "moss_get_tuning")
    return t


def moss_autotune(requests):
    reqs, n = _requests(requests)
    best = moss_tuning()
    ms = ctypes.c_double()
    _check(lib().moss_autotune(ctypes.cast(reqs, ctypes.c_void_p), n, ctypes.byref(best), ctypes.byref(ms)),
           "moss_autotune")
    return best, ms.value


def moss_server_create(mem_budget_bytes: int = 0, max_slots: int = 0, chunk_samples: int = 0, stream=None,
                       iteration_samples: int = 0, express_samples: int = 0, express: bool = True):
    cfg = moss_server_config(mem_budget_bytes, max_slots, 0 if express else 1, chunk_samples, iteration_samples,
                             express_samples)
    h = ctypes.c_void_p()
    _check(lib().moss_server_create(ctypes.byref(cfg), ctypes.c_void_p(0), ctypes.byref(h)), "moss_server_create")
    return h


def moss_server_add_graph(s, g) -> int:
    gid = ctypes.c_int32()
    _check(lib().moss_server_add_graph(s, g, ctypes.byref(gid)), "moss_server_add_graph")
    return gid.value


def moss_server_submit(s, graph_id: int, k: int, n_samples: int, seed: int, flags: int = 0) -> int:
    t = ctypes.c_uint64()
    _check(lib().moss_server_submit(s, graph_id, k, n_samples, seed, flags, ctypes.byref(t)), "moss_server_submit")
    return t.value


def moss_server_wait(s, ticket: int, timeout_ms: int = -1) -> moss_result:
    r = moss_result()
    _check(lib().moss_server_wait(s, ticket, timeout_ms, ctypes.byref(r)), "moss_server_wait")
    return r


def moss_server_cancel(s, ticket: int):
    _check(lib().moss_server_cancel(s, ticket), "moss_server_cancel")


def moss_server_stats_get(s) -> moss_server_stats:
    st = moss_server_stats()
    _check(lib().moss_server_stats_get(s, ctypes.byref(st)), "moss_server_stats_get")
    return st


def moss_server_destroy(s):
    _check(lib().moss_server_destroy(s), "moss_server_destroy")


# ---- convenience object over a graph handle ----------------------------------------
class Graph:
    """A resident graph: CSR on the device (borrowed torch tensors or a library copy)."""

    def __init__(self, csr, device_tensors: bool = True, flags: int = 0, stream=None):
        self.n, self.nnz = csr.n, csr.nnz
        if device_tensors:
            import torch
            self._rp = torch.from_numpy(np.ascontiguousarray(csr.row_ptr, dtype=np.int32)).cuda()
            self._col = torch.from_numpy(np.ascontiguousarray(csr.col, dtype=np.int32)).cuda()
            if self._col.numel() == 0:
                self._col = torch.zeros(1, dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
            self.h = moss_graph_create_device(self.n, self.nnz, self._rp, self._col, flags, stream)
        else:
            self._rp = self._col = None
            self.h = moss_graph_create(self.n, self.nnz, csr.row_ptr, csr.col, flags, stream)

    @classmethod
    def from_device(cls, d_row_ptr, d_col, flags: int = 0, stream=None):
        """Borrows int32 device tensors row_ptr[n+1], col[nnz] (kept alive by the object)."""
        self = cls.__new__(cls)
        self.n, self.nnz = int(d_row_ptr.numel()) - 1, int(d_col.numel())
        self._rp, self._col = d_row_ptr, d_col
        self.h = moss_graph_create_device(self.n, self.nnz, d_row_ptr, d_col, flags, stream)
        return self

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            moss_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_tables(self, k_mask: int = MOSS_TABLES_K4 | MOSS_TABLES_K5):
        moss_build_tables(self.h, k_mask)

    def info(self) -> moss_graph_info:
        return moss_graph_get_info(self.h)

    def table(self, which: int) -> np.ndarray:
        per_entry = (MOSS_TAB_ACC_SIGMA, MOSS_TAB_ACC_TAU, MOSS_TAB_ACC_CHECK, MOSS_TAB_RANK, MOSS_TAB_COL_RANK)
        count = self.nnz if which in per_entry else self.n
        return moss_table_read(self.h, which, count)

    def estimate(self, k: int, n_samples: int, seed: int, flags: int = 0) -> moss_result:
        return moss_estimate(self.h, k, n_samples, seed, flags)

    def estimate_to_precision(self, k: int, eps: float, delta: float, motif_mask: int, pilot_samples: int,
                              pilot_seed: int, max_samples: int, seed: int, flags: int = 0) -> moss_result:
        return moss_estimate_to_precision(self.h, k, eps, delta, motif_mask, pilot_samples, pilot_seed, max_samples,
                                          seed, flags)

    def sample_range(self, sampler: int, seed: int, k0: int, k1: int, class_out=None) -> np.ndarray:
        return moss_sample_range(self.h, sampler, seed, k0, k1, class_out)

    def sample_nodes(self, sampler: int, seed: int, index):
        import torch
        idx = torch.as_tensor(np.asarray(index, dtype=np.uint64).view(np.int64), device="cuda")
        nodes = torch.empty(idx.numel() * 5, dtype=torch.int32, device="cuda")
        cls = torch.empty(idx.numel(), dtype=torch.uint8, device="cuda")
        moss_sample_nodes(self.h, sampler, seed, idx, nodes, cls)
        return nodes.view(-1, 5).cpu().numpy(), cls.cpu().numpy()
