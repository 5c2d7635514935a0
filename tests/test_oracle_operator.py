"""Pins of the oracle's operator, embedding and Tucker code (CPU only)."""
import numpy as np
import pytest

import workloads as wl
from oracle import operator as op
from oracle import tucker


def test_two_fluid_material():
    f, s0, lam = 10e9, 1e7, 90e-9
    c = op.material_c(f, s0, lam)
    w = 2 * np.pi * f
    sigma = s0 - 1j / (w * op.MU0 * lam ** 2)  # eq. 3
    assert abs(c * sigma - 1) < 1e-15
    a, b = op.material_ab(f, s0, lam)         # eqs. 22-23
    assert abs((a + 1j * w * op.MU0 * b) - c) < 1e-15 * abs(c)
    # numeric value for the thin-film material (10 GHz, 1e7 S/m, 90 nm)
    assert abs(c.real - 4.0901e-12) < 1e-15 and abs(c.imag - 6.3952e-10) < 1e-13
    # sigma0 = 0: pure kinetic inductance, c = j w mu lam^2
    c0 = op.material_c(f, 0.0, lam)
    assert abs(c0 - 1j * w * op.MU0 * lam ** 2) < 1e-16 * abs(c0)


def test_mass_coefficients_match_eq9():
    assert op.mass_coefficient("x", "x") == 1.0
    assert abs(op.mass_coefficient("2D", "2D") - 1 / 6) < 1e-16
    assert abs(op.mass_coefficient("3D", "3D") - 1 / 2) < 1e-16
    for b, a in [("x", "2D"), ("x", "3D"), ("2D", "3D"), ("x", "y"), ("z", "3D")]:
        assert op.mass_coefficient(b, a) == 0.0


def test_block_pattern_matches_eq8():
    names = op.BASIS_SETS[5]
    nz = np.array([[bool(op.block_terms(b, a)) for a in names] for b in names])
    expect = np.array([[1, 0, 0, 1, 1],
                       [0, 1, 0, 1, 1],
                       [0, 0, 1, 0, 1],
                       [1, 1, 0, 1, 1],
                       [1, 1, 1, 1, 1]], dtype=bool)
    assert (nz == expect).all()
    assert nz.sum() == 17
    assert op.block_terms("x", "x") == op.block_terms("y", "y") == op.block_terms("z", "z") == [(1.0, "M0")]


def _setup(K, basis, seed, fill):
    m = wl.full_box(*K) if fill >= 1 else wl.random_mask(seed, *K, fill=fill)
    P = op.voxel_coords(m)
    fam = op.FamilyCache(*K)
    dx = 0.25e-6
    c = op.material_c(10e9, 1e7, 90e-9) * (1 + 0.1 * np.arange(P.shape[0]) / P.shape[0])
    s = 1j * 2 * np.pi * 10e9 * op.MU0 * dx
    return m, P, fam, dx, c, s


@pytest.mark.parametrize("K,basis,fill", [((8, 8, 8), 3, 1.0), ((5, 3, 4), 3, 0.6),
                                          ((4, 4, 3), 5, 0.7), ((3, 5, 2), 5, 1.0),
                                          ((1, 6, 2), 5, 1.0), ((7, 1, 1), 3, 1.0)])
def test_dense_equals_fft_convolution(K, basis, fill):
    m, P, fam, dx, c, s = _setup(K, basis, 11, fill)
    x = wl.random_currents(12, basis * P.shape[0])
    yd = op.dense_matvec(m, basis, x, fam, s, c, dx)
    for L in [tuple(2 * k for k in K), tuple(2 * k - 1 for k in K), tuple(2 * k + 3 for k in K)]:
        yf = op.fft_matvec(m, basis, x, fam, L, s, c, dx)
        assert np.linalg.norm(yd - yf) <= 1e-14 * np.linalg.norm(yd)


@pytest.mark.parametrize("basis", [3, 5])
def test_operator_symmetric(basis):
    m, P, fam, dx, c, s = _setup((4, 3, 3), basis, 13, 0.8)
    N = basis * P.shape[0]
    u, v = wl.random_currents(1, N), wl.random_currents(2, N)
    Zu = op.dense_matvec(m, basis, u, fam, s, c, dx)
    Zv = op.dense_matvec(m, basis, v, fam, s, c, dx)
    assert abs(v @ Zu - u @ Zv) <= 1e-14 * abs(v @ Zu)


def test_planted_sign_error_is_caught(monkeypatch):
    """A dropped sign on the observer moment breaks the symmetry pin."""
    orig = op.block_terms

    def wrong(beta, alpha):
        return [(abs(c), n) for c, n in orig(beta, alpha)]
    monkeypatch.setattr(op, "block_terms", wrong)
    m, P, fam, dx, c, s = _setup((3, 3, 2), 5, 14, 1.0)
    N = 5 * P.shape[0]
    u, v = wl.random_currents(1, N), wl.random_currents(2, N)
    Zu = op.dense_matvec(m, 5, u, fam, s, c, dx)
    Zv = op.dense_matvec(m, 5, v, fam, s, c, dx)
    assert abs(v @ Zu - u @ Zv) > 1e-6 * abs(v @ Zu)


def test_toeplitz_translation_invariance():
    """A structure shifted inside a larger grid gives the same currents."""
    small = wl.random_mask(3, 3, 4, 2, fill=0.7)
    big = np.zeros((4, 7, 6), dtype=np.uint8)
    big[1:3, 2:6, 2:5] = small
    fam_s, fam_b = op.FamilyCache(3, 4, 2), op.FamilyCache(6, 7, 4)
    N = 5 * int(small.sum())
    x = wl.random_currents(4, N)
    ys = op.dense_matvec(small, 5, x, fam_s)
    yb = op.fft_matvec(big, 5, x, fam_b, (12, 14, 8))
    assert np.linalg.norm(ys - yb) <= 1e-14 * np.linalg.norm(ys)


def test_impulse_gives_toeplitz_column():
    K = (6, 5, 4)
    m = wl.full_box(*K)
    P = op.voxel_coords(m)
    fam = op.FamilyCache(*K)
    k0 = 37
    x = np.zeros(3 * P.shape[0], dtype=complex)
    x[P.shape[0] + k0] = 1.0  # y-component impulse
    y = op.fft_matvec(m, 3, x, fam, (12, 10, 8))
    col = fam.values("M0", P[k0] - P)
    assert np.allclose(y[P.shape[0]:2 * P.shape[0]], col, rtol=1e-13, atol=1e-17)
    assert np.abs(y[:P.shape[0]]).max() == 0 and np.abs(y[2 * P.shape[0]:]).max() == 0


def test_embedding_value_at_K_is_irrelevant():
    """For L = 2K the entry at index K of the circulant is never used by the
    cropped product (reading: set it to zero)."""
    K, L = (4, 4, 4), (8, 8, 8)
    m = wl.full_box(*K)
    P = op.voxel_coords(m)
    fam = op.FamilyCache(*K)
    x = wl.random_currents(6, P.shape[0])
    g = np.zeros((8, 8, 8), dtype=complex)
    g[P[:, 2], P[:, 1], P[:, 0]] = x
    E = op.embed(lambda o: fam.values("M0", o), K, L)
    y0 = np.fft.ifftn(np.fft.fftn(E) * np.fft.fftn(g))[P[:, 2], P[:, 1], P[:, 0]]
    E2 = E.copy()
    E2[4, :, :] = 3.7
    E2[:, 4, :] = -1.1
    E2[:, :, 4] = 2.5
    y1 = np.fft.ifftn(np.fft.fftn(E2) * np.fft.fftn(g))[P[:, 2], P[:, 1], P[:, 0]]
    assert np.linalg.norm(y0 - y1) <= 1e-14 * np.linalg.norm(y0)


def test_circulant_of_even_block_is_real():
    K, L = (6, 5, 4), (12, 10, 8)
    fam = op.FamilyCache(*K)
    Zh = np.fft.fftn(op.embed(lambda o: fam.values("M0", o), K, L))
    assert np.abs(Zh.imag).max() <= 1e-15 * np.abs(Zh).max()
    Zo = np.fft.fftn(op.embed(lambda o: fam.values("M1x", o), K, L))
    assert np.abs(Zo.real).max() <= 1e-15 * np.abs(Zo).max()


# ---------------------------------------------------------------- Tucker ----

def _circulant_M0(K, L):
    fam = op.FamilyCache(*K)
    Zh = np.fft.fftn(op.embed(lambda o: fam.values("M0", o), K, L)).real
    return np.transpose(Zh, (2, 1, 0))  # modes (x, y, z)


def test_tucker_full_rank_reproduces():
    O = _circulant_M0((6, 5, 4), (12, 10, 8))
    C, F = tucker.tucker_svd(O, 0.0)
    assert [f.shape[1] for f in F] == [12, 10, 8]
    assert np.linalg.norm(tucker.tucker_full(C, F) - O) <= 1e-14 * np.linalg.norm(O)


def test_tucker_separable_has_rank_one():
    rng = np.random.default_rng(3)
    a, b, c = rng.standard_normal(7), rng.standard_normal(5), rng.standard_normal(6)
    O = np.einsum("i,j,k->ijk", a, b, c)
    C, F = tucker.tucker_svd(O, 1e-8)
    assert [f.shape[1] for f in F] == [1, 1, 1]
    assert np.linalg.norm(tucker.tucker_full(C, F) - O) <= 1e-14 * np.linalg.norm(O)


@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-8])
def test_tucker_error_below_tolerance(tol):
    O = _circulant_M0((16, 16, 8), (32, 32, 16))
    C, F = tucker.tucker_svd(O, tol)
    err = np.linalg.norm(tucker.tucker_full(C, F) - O) / np.linalg.norm(O)
    assert err <= tol
    assert max(f.shape[1] for f in F) < 16   # genuinely compressed


def test_tucker_rank_nearly_constant_in_domain_size():
    """Sec. III.B: the maximum multilinear rank stays nearly constant as the
    domain grows."""
    r = []
    for K in [(8, 8, 4), (16, 16, 8), (32, 32, 8)]:
        O = _circulant_M0(K, tuple(2 * k for k in K))
        _, F = tucker.tucker_svd(O, 1e-6)
        r.append(max(f.shape[1] for f in F))
    assert r[-1] - r[0] <= 4, r
