"""The estimators over many seeds on the GPU, against exact counts (the method of the
paper's Section 6: R independent runs, the empirical normalised root mean square error
set beside the standard error the variance formulas give).

C1 graph (Chung-Lu n = 2e3, m = 1e4) with its exact 4- and 5-node counts (the oracle's
enumeration, tests/golden/exact_c1.json); 200 seeds per case.  For every motif the mean
of the estimates must lie within 5 standard errors of the mean of the exact count
(Theorems 2, 6 and 8 make them unbiased), and where the estimator is well concentrated
(standard error at most 5% of the count) the empirical NRMSE must be within 20% of the
root of the mean reported variance (Theorems 3 and 10)."""
import json
import math
import os

import numpy as np
import pytest

import graphgen as gg
from paper_1509_08089_amd import moss

pytestmark = pytest.mark.gpu

RUNS = 200


def _exact(key):
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_c1.json")))
    return np.array(d[key], dtype=np.float64)


@pytest.mark.parametrize("k,samples,flags", [(4, 100_000, 0), (5, 200_000, 0), (5, 200_000, moss.MOSS_MIX_PAPER),
                                             (4, 100_000, moss.MOSS_K4_MIN)])
def test_seeds_against_exact_counts(k, samples, flags):
    G = moss.Graph(gg.config_graph("C1"))
    exact = _exact("n4" if k == 4 else "eta5")
    est, var = [], []
    for seed in range(1, RUNS + 1):
        r = G.estimate(k, samples, 1000 * k + seed, flags)
        est.append(r.estimate_np[: len(exact)])
        var.append(r.variance_np[: len(exact)])
    est, var = np.array(est), np.array(var)
    sd = np.sqrt(var.mean(axis=0))                     # the formulas' standard error
    mean_err = np.abs(est.mean(axis=0) - exact)
    nrmse = np.sqrt(((est - exact) ** 2).mean(axis=0))
    for i in range(len(exact)):
        assert mean_err[i] <= 5 * sd[i] / math.sqrt(RUNS), (i + 1, est[:, i].mean(), exact[i], sd[i])
        if exact[i] > 0 and sd[i] <= 0.05 * exact[i]:
            assert abs(nrmse[i] - sd[i]) <= 0.2 * sd[i], (i + 1, nrmse[i], sd[i])
