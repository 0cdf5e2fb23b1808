"""The gather probe of the benchmark (libmoss_probe.so) does the loads its header
describes: the fill is SplitMix64 of seed + i, and each lane's sum follows its chains
j <- floor((x ^ salt) * words / 2^64) from their starts, recomputed here in Python."""
import numpy as np
import pytest
import torch

from paper_1509_08089_amd import probe

pytestmark = pytest.mark.gpu

M = (1 << 64) - 1


def splitmix64(z):
    z = (z + 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


@pytest.mark.parametrize("words,blocks,steps", [(1, 1, 3), (1000, 2, 17), (12345, 3, 40)])
@pytest.mark.parametrize("chains", [1, 2, 4, 8])
def test_probe_matches_its_definition(words, blocks, steps, chains):
    buf = torch.empty(words, dtype=torch.int64, device="cuda")
    probe.moss_probe_fill(buf, 7)
    out = torch.zeros(blocks * 256, dtype=torch.int64, device="cuda")
    probe.moss_probe_gather(buf, blocks, steps, out, chains)
    torch.cuda.synchronize()
    b = buf.cpu().numpy().view(np.uint64)
    want_b = [splitmix64(7 + i) for i in range(words)]
    assert [int(x) for x in b] == want_b
    got = out.cpu().numpy().view(np.uint64)
    for t in list(range(0, blocks * 256, 37)) + [blocks * 256 - 1]:
        acc = 0
        for c in range(chains):  # chain c of lane t: id t * chains + c
            i = t * chains + c
            salt = splitmix64(~i & M) | 1
            j = (splitmix64(i) * words) >> 64
            for _ in range(steps):
                x = want_b[j]
                acc = (acc + x) & M
                j = ((x ^ salt) * words) >> 64
        assert int(got[t]) == acc, t
