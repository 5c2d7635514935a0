"""Pins of the oracle's saddle system and port model (CPU only): closed-form
circuits (a resistor voxel, the DC resistance of a bar, kinetic inductance
mu0 lambda^2 l / A), reciprocity, conservation and divergence-free fluxes."""
import numpy as np
import pytest

import workloads as wl
from oracle import circuit as cc
from oracle import green
from oracle import operator as op


def _dense_Z(mask, f, s0, lam, dx, basis=3):
    P = op.voxel_coords(mask)
    K = P.shape[0]
    fam = op.FamilyCache(mask.shape[2], mask.shape[1], mask.shape[0])
    c = op.material_c(f, s0, lam) * np.ones(K)
    s = 1j * 2 * np.pi * f * op.MU0 * dx
    return op.dense_rows(mask, basis, np.arange(basis * K), fam, s, c, dx)


def bar_ports(mask):
    """One port across the x-extent of a bar: + terminal on the -x faces of the
    first column, - terminal on the +x faces of the last column."""
    P = op.voxel_coords(mask)
    x0, x1 = P[:, 0].min(), P[:, 0].max()
    plus = [(k, 0) for k in range(P.shape[0]) if P[k, 0] == x0]
    minus = [(k, 1) for k in range(P.shape[0]) if P[k, 0] == x1]
    return plus, minus


def test_single_voxel_resistor():
    mask = wl.full_box(1, 1, 1)
    dx, f, s0, lam = 1e-6, 10e9, 1e7, 90e-9
    Z = _dense_Z(mask, f, s0, lam, dx)
    A, node_of, _ = cc.incidence(mask)
    pn = cc.port_nodes(mask, node_of, [([(0, 0)], [(0, 1)])])
    Y, X, free, b = cc.solve_ports(Z, A, pn)
    assert abs(Y[0, 0] - 1 / Z[0, 0]) <= 1e-14 * abs(Y[0, 0])


def test_bar_dc_resistance():
    """sigma0 = 1e7, no superconductivity (huge London depth), 1 Hz:
    Re Z_port = l / (sigma0 w t) (uniform current, series/parallel lines)."""
    Lx, Ly, Lz = 6, 2, 3
    mask = wl.full_box(Lx, Ly, Lz)
    dx, f, s0, lam = 1e-6, 1.0, 1e7, 1e3
    Z = _dense_Z(mask, f, s0, lam, dx)
    A, node_of, _ = cc.incidence(mask)
    pn = cc.port_nodes(mask, node_of, [bar_ports(mask)])
    Y, *_ = cc.solve_ports(Z, A, pn)
    R = (Lx * dx) / (s0 * (Ly * dx) * (Lz * dx))
    assert abs((1 / Y[0, 0]).real - R) <= 1e-9 * R


def test_bar_kinetic_inductance():
    """sigma0 = 0 and lambda^2 >> dx^2: L_port -> mu0 lambda^2 l / A plus the
    bar's uniform-current partial self-inductance (double sum of the same
    voxel-pair integrals)."""
    Lx, Ly, Lz = 8, 2, 2
    mask = wl.full_box(Lx, Ly, Lz)
    dx, f, s0, lam = 1e-6, 1e9, 0.0, 6e-6
    Z = _dense_Z(mask, f, s0, lam, dx)
    A, node_of, _ = cc.incidence(mask)
    pn = cc.port_nodes(mask, node_of, [bar_ports(mask)])
    Y, *_ = cc.solve_ports(Z, A, pn)
    w = 2 * np.pi * f
    Lport = (1 / Y[0, 0]).imag / w
    Lkin = op.MU0 * lam ** 2 * (Lx * dx) / ((Ly * dx) * (Lz * dx))
    P = op.voxel_coords(mask)
    Tsum = green.family_values("M0", (P[None, :, :] - P[:, None, :]).reshape(-1, 3)).sum()
    Lmag = op.MU0 * dx * Tsum / (Ly * Lz) ** 2
    assert abs(Lport - (Lkin + Lmag)) <= 1e-3 * Lport
    assert Lmag > 0.01 * Lkin  # the magnetic part is resolved, not negligible


def test_two_port_reciprocity_and_conservation():
    mask = np.zeros((2, 5, 6), dtype=np.uint8)
    mask[:, 0, :] = 1
    mask[:, 3:5, :] = 1
    dx, f, s0, lam = 0.5e-6, 5e9, 1e7, 90e-9
    Z = _dense_Z(mask, f, s0, lam, dx)
    A, node_of, _ = cc.incidence(mask)
    P = op.voxel_coords(mask)
    ports = []
    for ys in ([0], [3, 4]):
        plus = [(k, 0) for k in range(P.shape[0]) if P[k, 0] == 0 and P[k, 1] in ys]
        minus = [(k, 1) for k in range(P.shape[0]) if P[k, 0] == 5 and P[k, 1] in ys]
        ports.append((plus, minus))
    pn = cc.port_nodes(mask, node_of, ports)
    Y, X, free, b = cc.solve_ports(Z, A, pn)
    assert abs(Y[0, 1] - Y[1, 0]) <= 1e-12 * abs(Y[0, 1])
    assert abs(Y[0, 1]) > 1e-6 * abs(Y[0, 0])
    n = Z.shape[0]
    for p in range(2):
        kcl = A[free] @ X[:n, p]
        assert np.abs(kcl).max() <= 1e-12 * np.abs(X[:n, p]).max()


@pytest.mark.parametrize("basis", [3, 5])
def test_incidence_columns_are_divergence_free(basis):
    mask = wl.random_mask(4, 4, 3, 3, fill=0.6)
    A, _, _ = cc.incidence(mask, basis)
    # every basis function's drawn currents sum to zero (eq. 2 per voxel)
    assert np.abs(A.sum(axis=0)).max() == 0.0
