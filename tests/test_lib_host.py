"""Host-side checks of the HIP library (no GPU calls): exported symbols and
the closed-form Toeplitz tensor against the oracle's quadrature."""
import os
import re

import numpy as np
import pytest

import paper_2105_08627_amd as svh
from oracle import green

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "svh.h")).read()
    declared = set(re.findall(r"\b(svh_[a-z0-9_]+)\s*\(", hdr))
    assert declared, "no declarations parsed"
    L = svh.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(svh.EXPORTED)


@pytest.mark.parametrize("K", [(8, 8, 8), (5, 3, 4), (1, 1, 1), (2, 7, 3)])
def test_closed_form_toeplitz_matches_oracle(K):
    T = svh.green_toeplitz(*K)
    ref = green.family_table("M0", *K)
    assert np.max(np.abs(T - ref) / np.abs(ref)) < 2e-14


def test_closed_form_toeplitz_far_offsets():
    """Far offsets (sixth-difference cancellation of about |d|^6) stay accurate."""
    T = svh.green_toeplitz(300, 1, 200)
    offs = [(299, 0, 199), (150, 0, 0), (0, 0, 199), (17, 0, 3)]
    ref = green.family_values("M0", offs)
    got = np.array([T[o[2], o[1], o[0]] for o in offs])
    assert np.max(np.abs(got - ref) / ref) < 1e-14
