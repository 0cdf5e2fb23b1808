"""ctypes binding of libmoss_probe.so (include/moss_probe.h): the dependent random-gather
probe the benchmark measures the sampling kernels' memory ceiling with.  Same names as
the C calls; tensors are torch CUDA tensors, streams torch streams (None = current)."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmoss_probe.so")
EXPORTED = ("moss_probe_fill", "moss_probe_gather")

_lib = None
_lock = threading.Lock()


def lib():
    """Loads libmoss_probe.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1509_08089_amd.build`")
            L = ctypes.CDLL(LIB_PATH)
            P, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
            L.moss_probe_fill.argtypes = [P, u64, u64, P]
            L.moss_probe_gather.argtypes = [P, u64, u32, u32, u32, P, P]
            for name in EXPORTED:
                getattr(L, name).restype = ctypes.c_int
            _lib = L
        return _lib


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"{name} failed with code {rc}")


def moss_probe_fill(buf, seed: int, stream=None) -> None:
    """Fills the uint64 (int64) tensor buf with SplitMix64 outputs of seed + i."""
    assert buf.is_cuda and buf.dtype.itemsize == 8 and buf.is_contiguous()
    _check(lib().moss_probe_fill(ctypes.c_void_p(buf.data_ptr()), buf.numel(), seed, _stream(stream)),
           "moss_probe_fill")


def moss_probe_gather(buf, blocks: int, steps: int, out, chains: int = 1, stream=None) -> None:
    """blocks x 256 lanes, each following `chains` chains of `steps` dependent loads over
    buf; out holds blocks * 256 words."""
    assert buf.is_cuda and buf.dtype.itemsize == 8 and buf.is_contiguous()
    assert out.is_cuda and out.dtype.itemsize == 8 and out.is_contiguous() and out.numel() >= blocks * 256
    _check(lib().moss_probe_gather(ctypes.c_void_p(buf.data_ptr()), buf.numel(), blocks, steps, chains,
                                   ctypes.c_void_p(out.data_ptr()), _stream(stream)), "moss_probe_gather")
