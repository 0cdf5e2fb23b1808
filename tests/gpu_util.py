"""Shared helpers of the GPU tests (imported by tests marked `gpu` only)."""
import numpy as np

import oracle
from paper_1509_08089_amd import moss

SAMPLERS = (moss.MOSS_SAMPLER_MOSS4, moss.MOSS_SAMPLER_T5, moss.MOSS_SAMPLER_PATH5)
ORACLE_SAMPLER = {moss.MOSS_SAMPLER_MOSS4: oracle.MOSS4, moss.MOSS_SAMPLER_T5: oracle.T5,
                  moss.MOSS_SAMPLER_PATH5: oracle.PATH5, moss.MOSS_SAMPLER_MOSS4MIN: oracle.MOSS4MIN}


def rel_close(a, b, scale=0.0, tol=1e-12):
    return abs(a - b) <= tol * max(abs(a), abs(b), scale, 1e-300)


def assert_result_matches(gpu: moss.moss_result, orc: oracle.Result, lam: float):
    """Hits bit-exact; estimates and variances within 1e-12 relative.  The estimate of
    n_2 / eta_2 is a difference taken from Lambda, which cancels in double, so its bound
    is relative to max(|x|, Lambda); every variance is held to 1e-12 of its own size."""
    assert gpu.k == orc.k and gpu.n_motifs == orc.n_motifs
    assert [int(gpu.K[0]), int(gpu.K[1])] == orc.K
    np.testing.assert_array_equal(gpu.hits_np, orc.hits)
    for i in range(orc.n_motifs):
        scale = lam if i == 1 else 0.0
        assert rel_close(gpu.estimate[i], orc.estimate[i], scale), (i, gpu.estimate[i], orc.estimate[i])
        assert rel_close(gpu.variance[i], orc.variance[i]), (i, gpu.variance[i], orc.variance[i])
