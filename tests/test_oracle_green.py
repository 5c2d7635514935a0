"""Pins of the oracle's voxel-pair Green integrals (CPU only).

Each check compares the oracle with something other than itself: the
definition integrated a different way, classical constants, asymptotics.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import green

FOUR_PI = 4 * np.pi

# Mean reciprocal distance of two independent uniform points in the unit cube
# (classical closed-form constant); M0(0) is this over 4 pi (eq. 19 at l = k,
# unit voxel of App. B).
MEAN_INV_DIST_UNIT_CUBE = 1.8823126443896601


@pytest.mark.parametrize("pq", [(0, 0), (0, 1), (1, 1)])
def test_overlap_weights_match_definition(pq):
    p, q = pq
    for v in np.linspace(-1, 1, 17):
        lo, hi = max(-0.5, v - 0.5), min(0.5, v + 0.5)
        ref = integrate.quad(lambda s: s ** q * (s - v) ** p, lo, hi)[0] if hi > lo else 0.0
        assert abs(green.overlap_weight(pq, v) - ref) < 1e-15


def test_self_term_is_classical_constant():
    v = green.family_values("M0", [(0, 0, 0)])[0]
    assert abs(v * FOUR_PI - MEAN_INV_DIST_UNIT_CUBE) < 2e-15


def _brute_6d(name, d, n=8):
    """Direct tensor Gauss-Legendre over both voxels (no tent reduction)."""
    pqs = green.FAMILIES[name]
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * x
    w = 0.5 * w
    U = np.meshgrid(x, x, x, indexing="ij")
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    obs = [u.ravel() for u in U]
    Wv = W.ravel()
    tot = 0.0
    for j in range(Wv.size):  # loop over source points, vectorise observers
        src = [obs[a][j] for a in range(3)]
        r = np.sqrt(sum((d[a] + src[a] - obs[a]) ** 2 for a in range(3)))
        f = Wv / r
        for a in range(3):
            p, q = pqs[a]
            f = f * obs[a] ** p * src[a] ** q
        tot += Wv[j] * f.sum()
    return tot / FOUR_PI


@pytest.mark.parametrize("name", list(green.FAMILIES))
def test_families_match_6d_brute_force(name):
    for d in [(3, 0, 0), (2, 2, 1), (0, 3, 2), (4, 1, 3)]:
        ref = _brute_6d(name, d)
        v = green.family_values(name, [d])[0]
        scale = abs(green.family_values("M0", [d])[0])
        assert abs(v - ref) <= 1e-12 * scale, (name, d, v, ref)


def _tent_adaptive(d, eps=1e-12):
    """M0(d) by adaptive QUADPACK over the 8 tent boxes (independent of the
    oracle's Duffy / fixed Gauss-Legendre rules)."""
    tot = 0.0
    for bx in (-1, 0):
        for by in (-1, 0):
            for bz in (-1, 0):
                f = lambda z, y, x: ((1 - abs(x)) * (1 - abs(y)) * (1 - abs(z))
                                     / np.sqrt((d[0] + x) ** 2 + (d[1] + y) ** 2 + (d[2] + z) ** 2))
                tot += integrate.tplquad(f, bx, bx + 1, by, by + 1, bz, bz + 1,
                                         epsabs=eps, epsrel=eps)[0]
    return tot / FOUR_PI


@pytest.mark.slow
@pytest.mark.parametrize("d", [(1, 0, 0), (1, 1, 0)])
def test_near_singular_against_adaptive(d):
    v = green.family_values("M0", [d])[0]
    assert abs(v - _tent_adaptive(d)) < 1e-9 * v


def test_far_field_asymptotics():
    # M0: 4 pi |d| M0 = 1 - 7/(240 d^4) + O(d^-6) along an axis (the tent's
    # second moments vanish against the harmonic 1/r; the fourth-order term
    # follows from the MGF (sinh(D/2)/(D/2))^2 of the tent).
    for x in [12, 20, 40]:
        v = green.family_values("M0", [(x, 0, 0)])[0]
        assert abs(v * FOUR_PI * x - (1 - 7 / (240 * x ** 4))) < 5.0 / x ** 6
    # M1_x ~ (1/12) d/dx g ;  M2_x ~ -(1/144) d2/dx2 g  (second moments of the
    # source / observer-source overlap weights)
    for x in [15, 30]:
        g1 = -1 / (FOUR_PI * x ** 2)
        g2 = 2 / (FOUR_PI * x ** 3)
        v1 = green.family_values("M1x", [(x, 0, 0)])[0]
        v2 = green.family_values("M2x", [(x, 0, 0)])[0]
        assert abs(v1 / (g1 / 12) - 1) < 5.0 / x ** 2
        assert abs(v2 / (-g2 / 144) - 1) < 5.0 / x ** 2


def test_parity_and_permutation():
    rng = np.random.default_rng(5)
    offs = rng.integers(-6, 7, size=(30, 3))
    for name in green.FAMILIES:
        v = green.family_values(name, offs)
        for a in range(3):
            flip = offs.copy()
            flip[:, a] *= -1
            vf = green.family_values(name, flip)
            odd = name.startswith("M1") and name[2] == "xyz"[a]
            assert np.allclose(vf, -v if odd else v, rtol=1e-14, atol=1e-17)
    # axis permutation maps M0 to itself and M2x -> M2y
    v0 = green.family_values("M0", offs)
    assert np.allclose(green.family_values("M0", offs[:, [1, 0, 2]]), v0, rtol=1e-14)
    assert np.allclose(green.family_values("M2y", offs[:, [1, 0, 2]]),
                       green.family_values("M2x", offs), rtol=1e-13, atol=1e-18)


def test_quadrature_converged():
    """Every point-count tier agrees with a much finer rule."""
    offs = [(2, 0, 0), (2, 2, 2), (4, 1, 0), (9, 0, 3), (10, 10, 0), (31, 2, 1), (1, 0, 0), (1, 1, 1)]
    saved = green._points_for_distance
    try:
        base = {n: green.family_values(n, offs) for n in ("M0", "M1x", "M2z")}
        green._points_for_distance = lambda dist: 24
        fine = {n: green.family_values(n, offs) for n in ("M0", "M1x", "M2z")}
    finally:
        green._points_for_distance = saved
    for n in base:
        scale = np.abs(green.family_values("M0", offs))
        assert np.all(np.abs(base[n] - fine[n]) <= 2e-15 * scale), n


# ---------------------------------------------------------------------------
# Near-singular offsets (all |d_i| <= 1) of every family, against a reference
# that shares no step with the oracle's Duffy rule: the overlap weights are
# rebuilt here from their definition (integrals over the overlap of two unit
# intervals, as polynomials), the innermost z integral of
# w_z(z) / sqrt(rho^2 + (d_z + z)^2) is taken in closed form (antiderivatives
# of t^k / sqrt(rho^2 + t^2), k <= 3), and the remaining 2D integral, which has
# at most a logarithmic singularity at a corner, by adaptive QUADPACK.

def _weight_poly_from_definition(pq, lo):
    """w(v) = int s^q (s - v)^p ds over [max(-1/2, v - 1/2), min(1/2, v + 1/2)]
    as a polynomial in v on the half [lo, lo + 1] (lo = -1 or 0)."""
    P = np.polynomial.Polynomial
    v = P([0.0, 1.0])
    a, b = (v - 0.5, P([0.5])) if lo >= 0 else (P([-0.5]), v + 0.5)
    p, q = pq
    s_pow = {0: lambda x: x, 1: lambda x: x ** 2 / 2, 2: lambda x: x ** 3 / 3}
    # int s^q (s - v)^p ds, p, q in {0, 1}: expand (s - v)^p
    if p == 0:
        return s_pow[q](b) - s_pow[q](a)
    return (s_pow[q + 1](b) - s_pow[q + 1](a)) - v * (s_pow[q](b) - s_pow[q](a))


def _inner_closed_form(c, rho2, t0, t1):
    """int_{t0}^{t1} sum_k c_k t^k / sqrt(rho2 + t^2) dt (k <= 3), closed form."""
    assert rho2 > 0.0
    rho = np.sqrt(rho2)

    def F(t):
        s = np.sqrt(rho2 + t * t)
        ash = np.arcsinh(t / rho)
        return (c[0] * ash + c[1] * s + c[2] * (t * s - rho2 * ash) / 2
                + c[3] * s * (t * t - 2 * rho2) / 3)
    return F(t1) - F(t0)


def _family_semi_analytic(name, d, epsabs=1e-15):
    pqs = green.FAMILIES[name]
    P = np.polynomial.Polynomial
    tot = 0.0
    for lx in (-1.0, 0.0):
        wx = _weight_poly_from_definition(pqs[0], lx)
        for ly in (-1.0, 0.0):
            wy = _weight_poly_from_definition(pqs[1], ly)
            for lz in (-1.0, 0.0):
                wz = _weight_poly_from_definition(pqs[2], lz)(P([-float(d[2]), 1.0]))  # in t = d_z + z
                c = list(wz.coef) + [0.0] * (4 - len(wz.coef))
                t0, t1 = d[2] + lz, d[2] + lz + 1.0

                def f(y, x):
                    rho2 = (d[0] + x) ** 2 + (d[1] + y) ** 2
                    return wx(x) * wy(y) * _inner_closed_form(c, rho2, t0, t1)
                tot += integrate.dblquad(f, lx, lx + 1, ly, ly + 1, epsabs=epsabs, epsrel=1e-13)[0]
    return tot / FOUR_PI


NEAR_OFFSETS = [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)] + \
    [(-1, 0, 0), (0, -1, 1), (1, 0, -1), (-1, -1, -1)]


@pytest.mark.slow
@pytest.mark.parametrize("name", list(green.FAMILIES))
def test_near_families_against_semi_analytic(name):
    """App. A eqs. 19-21 at the offsets whose boxes touch the singular point:
    the oracle's Duffy rule against the independent reference above, to
    1e-14 of M0(0)."""
    scale = green.family_values("M0", [(0, 0, 0)])[0]
    v = green.family_values(name, NEAR_OFFSETS)
    for d, got in zip(NEAR_OFFSETS, v):
        ref = _family_semi_analytic(name, d)
        assert abs(got - ref) <= 1e-14 * scale, (name, d, got, ref)


def test_semi_analytic_reference_reduces_to_classical_constant():
    """The reference itself: M0(0) is the mean inverse distance of the unit cube."""
    v = _family_semi_analytic("M0", (0, 0, 0))
    assert abs(v * FOUR_PI - MEAN_INV_DIST_UNIT_CUBE) < 1e-14


def test_duffy_rule_converged():
    """The corner-box rule (n_ang, n_rad) = (20, 14) against (40, 28)."""
    offs = [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)] + [(-1, 1, 0)]
    saved = green._corner_box_integral
    try:
        base = {n: green.family_values(n, offs) for n in green.FAMILIES}
        green._corner_box_integral = lambda d, lo, hi, pqs: saved(d, lo, hi, pqs, n_ang=40, n_rad=28)
        fine = {n: green.family_values(n, offs) for n in green.FAMILIES}
    finally:
        green._corner_box_integral = saved
    scale = green.family_values("M0", [(0, 0, 0)])[0]
    for n in base:
        assert np.all(np.abs(base[n] - fine[n]) <= 1e-15 * scale), (n, np.abs(base[n] - fine[n]).max() / scale)
