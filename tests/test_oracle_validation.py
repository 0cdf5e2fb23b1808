"""The creation tests' plain validator (tests/defects.py) against the oracle's own CSR
validation, on the same single-edit defects the GPU tests place at span edges: both
read the problem statement's rules (Section 2: an undirected simple graph, here as
symmetric CSR with strictly ascending rows) and must name the same defect, so the GPU
status codes are tied to the oracle's."""
import numpy as np
import pytest

import defects
import oracle
from graphgen.csr import CSR


def oracle_status(rp, col):
    try:
        oracle.Graph(CSR(np.asarray(rp, np.int32), np.asarray(col, np.int32), "case"), validate=True)
        return oracle.OK
    except oracle.OracleError as e:
        return e.status


@pytest.fixture(scope="module")
def base():
    g = defects.span_graph()
    return np.asarray(g.row_ptr, np.int32), np.asarray(g.col, np.int32)


def test_codes_are_the_libraries_codes():
    from paper_1509_08089_amd import moss
    assert (defects.ARG, defects.UNSORTED, defects.SELF_LOOP, defects.DUPLICATE, defects.ASYMMETRIC) == \
        (moss.MOSS_E_ARG, moss.MOSS_E_UNSORTED, moss.MOSS_E_SELF_LOOP, moss.MOSS_E_DUPLICATE, moss.MOSS_E_ASYMMETRIC)
    assert (oracle.E_ARG, oracle.E_UNSORTED, oracle.E_SELF_LOOP, oracle.E_DUPLICATE, oracle.E_ASYMMETRIC) == \
        (moss.MOSS_E_ARG, moss.MOSS_E_UNSORTED, moss.MOSS_E_SELF_LOOP, moss.MOSS_E_DUPLICATE, moss.MOSS_E_ASYMMETRIC)


def test_validators_agree_on_every_single_edit_defect(base):
    rp, col = base
    assert defects.expected_status(rp, col) == oracle_status(rp, col) == 0
    n_cases = 0
    for name, r, c in defects.cases(rp, col):
        want = defects.expected_status(r, c)
        assert want != 0, name
        assert oracle_status(r, c) == want, name
        n_cases += 1
    assert n_cases > 150
    rp2 = np.concatenate([rp, np.full(5000, rp[-1], np.int32)])  # trailing rows without entries
    nnz = len(col)
    for name, r, c in defects.cases(rp2, col, [nnz - 1, nnz - 2, (nnz - 1) // 256 * 256]):
        assert oracle_status(r, c) == defects.expected_status(r, c) != 0, name
