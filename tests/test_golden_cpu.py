"""The stored eigenvalue files: that the elasticity golden holds the p leftmost eigenvalues (Alg. 2 asks for
the p smallest; deflation, Sec. 3.2, could skip one and residuals alone would not show it), and that the
inertia count used for it agrees with dense eigenvalues on small cases.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_1312_1553_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import check_inertia as CI  # noqa: E402


@pytest.mark.parametrize("ne", [3, 5])
def test_negative_pivots_count_the_eigenvalues_below_sigma(ne):
    """Sylvester's law of inertia through SuperLU with diagonal pivots, in both elimination orders, against
    numpy's dense eigenvalues of the same Q1 elasticity matrix."""
    M = W.elasticity_q1(ne, seed=2).to_scipy()
    ev = np.linalg.eigvalsh(M.toarray())
    perm = CI.nested_dissection_q1(ne)
    assert np.array_equal(np.sort(perm), np.arange(M.shape[0]))
    for k in (1, 4, 17, M.shape[0] // 2):
        sigma = 0.5 * (ev[k - 1] + ev[k])
        assert CI.negative_pivots(M, sigma, perm)[0] == k
        assert CI.negative_pivots(M, sigma)[0] == k


def test_elasticity_golden_holds_the_leftmost_p():
    """The counts written by check_inertia.py for the 50^3 elasticity golden: p eigenvalues below a shift just
    above the stored lambda_p, p - 1 below one between lambda_{p-1} and lambda_p."""
    g = json.load(open(os.path.join(GOLDEN, "oracle_evals_elasticity_50_p20.json")))
    ev = np.array(g["evals"])
    p = len(ev)
    inert = g["inertia"]
    assert p == 20 and np.all(np.diff(ev) > 0)
    assert ev[-1] < inert["sigma_above_lambda_p"] <= ev[-1] * (1 + 1e-3) * (1 + 1e-12)
    assert ev[-2] < inert["sigma_between_lambda_p-1_and_lambda_p"] < ev[-1]
    assert inert["count_above"] == p
    assert inert["count_between"] == p - 1
