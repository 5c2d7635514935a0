"""Tucker decomposition (oracle; test infrastructure only).

Algorithm 1 (Tucker-SVD) and the i-mode product of eqs. 10-11, Sec. II.B.
Modes are numpy axes 0, 1, 2 of the array passed in.
"""
from __future__ import annotations

import numpy as np


def unfold(O, mode):
    """Mode-i unfolding: rows indexed by axis ``mode``, columns by the other two."""
    return np.moveaxis(O, mode, 0).reshape(O.shape[mode], -1)


def mode_product(C, F, mode):
    """i-mode product (eq. 11): V[.., v_i, ..] = sum_{i'} C[.., i', ..] F[v_i, i']."""
    out = np.tensordot(F, C, axes=([1], [mode]))  # new axis first
    return np.moveaxis(out, 0, mode)


def select_rank(s, tol, norm_O):
    """Truncation index of Alg. 1 step 7.

    Reading of the paper's "index of the maximum normalised singular value
    smaller than tol/sqrt(3)": the smallest d such that the discarded tail
    satisfies sqrt(sum_{j>d} s_j^2) <= tol/sqrt(3) * ||O||_F.  With this choice
    the three truncations together keep ||O - O~||_F <= tol ||O||_F."""
    thr = tol / np.sqrt(3.0) * norm_O
    tail = np.sqrt(np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]]))
    # tail[d] = norm of s[d:], d = 0..len(s)
    d = int(np.argmax(tail <= thr))
    return max(d, 1)


def tucker_svd(O, tol):
    """Algorithm 1: for each mode unfold the ORIGINAL tensor O (step 5), take its
    SVD (step 6), truncate (step 7) and project the running core with the
    conjugate-transposed factor (step 8).  Returns (core, [F1, F2, F3])."""
    O = np.asarray(O)
    norm_O = np.linalg.norm(O.ravel())
    C = O
    F = []
    for i in range(3):
        U, s, _ = np.linalg.svd(unfold(O, i), full_matrices=False)
        d = select_rank(s, tol, norm_O)
        Fi = U[:, :d]
        F.append(Fi)
        C = mode_product(C, Fi.conj().T, i)
    return C, F


def tucker_full(C, F):
    """Restore a tensor from its Tucker form (eq. 10)."""
    O = C
    for i in range(3):
        O = mode_product(O, F[i], i)
    return O
