"""The same erased Chung-Lu recipe as chung_lu.py, generated on a torch device.

Used for the large multi-graph workloads (batched and serving runs), where building
hundreds of millions of edges with numpy would dominate the run.  Streams come from
torch's generator on the device, so the graphs differ from the numpy ones with the
same seed; each is still a fixed function of (n, m, beta, dmax, seed, device type).
Returns int32 row_ptr / col tensors on the device (symmetric, rows ascending).
"""
from __future__ import annotations

import numpy as np

from .chung_lu import chung_lu_weights


def chung_lu_device(n: int, m: int, beta: float, dmax: float, seed: int, device="cuda"):
    import torch

    if m > n * (n - 1) // 2:
        raise ValueError("more edges than a simple graph on n nodes can hold")
    w = chung_lu_weights(n, m, beta, dmax)
    cdf = torch.from_numpy(np.cumsum(w) / w.sum()).to(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    keys = torch.empty(0, dtype=torch.int64, device=device)
    batch = int(m * 1.2) + 16
    while True:
        a = torch.searchsorted(cdf, torch.rand(batch, generator=gen, device=device, dtype=torch.float64), right=True)
        b = torch.searchsorted(cdf, torch.rand(batch, generator=gen, device=device, dtype=torch.float64), right=True)
        a.clamp_(max=n - 1)
        b.clamp_(max=n - 1)
        lo, hi = torch.minimum(a, b), torch.maximum(a, b)
        k = lo * n + hi
        keys = torch.cat([keys, k[lo != hi]])
        uniq, inv = torch.unique(keys, sorted=True, return_inverse=True)
        if uniq.numel() >= m:
            pos = torch.arange(keys.numel(), device=device)
            first = torch.full((uniq.numel(),), keys.numel(), dtype=torch.int64, device=device)
            first.scatter_reduce_(0, inv, pos, reduce="amin")
            first = torch.sort(first).values[:m]
            keys = keys[first]
            break
        batch = int((m - uniq.numel()) * 1.5) + 1024
    perm = torch.randperm(n, generator=gen, device=device)
    src, dst = perm[keys // n], perm[keys % n]
    s2 = torch.cat([src, dst])
    d2 = torch.cat([dst, src])
    order = torch.argsort(s2 * n + d2)
    s2, d2 = s2[order], d2[order]
    counts = torch.bincount(s2, minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return row_ptr.to(torch.int32), d2.to(torch.int32)
