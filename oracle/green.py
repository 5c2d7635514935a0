"""Voxel-pair Green integrals by quadrature (oracle; test infrastructure only).

Definitions (Sec. II.A, App. A eqs. 19-21, App. B eqs. 24-27).  For two unit
voxels whose centres differ by the integer offset ``d`` (source minus
observer, in voxel units), with ``u`` the observer point and ``u'`` the source
point measured from their own voxel centres and ``g(r) = 1/(4 pi |r|)``:

    M0(d)   = int_{cube} int_{cube} g(d + u' - u) du' du          (eq. 19/24)
    M1_a(d) = int int u'_a g(d + u' - u) du' du                   (source moment)
    M2_a(d) = int int u_a u'_a g(d + u' - u) du' du               (eqs. 20-21 terms)

The physical entries are these times (Delta x)^5 for M0, (Delta x)^6 for M1,
(Delta x)^7 for M2 (change of variables of App. B).  The paper prints a minus
sign in front of the integrals of eqs. 19-21; the reading taken here is the
positive integral (the magnetic energy of a current distribution is positive).

Exact reduction used: substituting v = u' - u turns each 6D integral into the
3D integral  int_{[-1,1]^3} prod_i w_i(v_i) g(d + v) dv, where w_i is the 1D
overlap weight of the two unit intervals:
    (p, q) = (0, 0):  w(v) = 1 - |v|                   (tent)
    (p, q) = (0, 1):  w(v) = v (1 - |v|) / 2           (int u' over the overlap)
    (p, q) = (1, 1):  w(v) = -t/4 + t^2/2 - t^3/6,  t = 1 - |v|
with p, q the powers of u_a and u'_a.  Each weight is a polynomial on [-1, 0]
and on [0, 1], so the domain splits into 8 boxes on which the integrand is a
polynomial times g.  For integer offsets the singular point s = d + v = 0 is
either outside a box or at one of its corners; corner-singular boxes use the
Duffy pyramid map (which cancels the 1/r singularity), all other boxes use
tensor Gauss-Legendre with a point count chosen from the box's distance to
the singular point.
"""
from __future__ import annotations

import functools
import numpy as np

FOUR_PI = 4.0 * np.pi

# (p, q) powers per axis for each integral family.  M0 is the scalar kernel of
# the piecewise-constant blocks; M1_a / M2_a enter the blocks with the
# piecewise-linear basis functions of eqs. 5-6.
FAMILIES = {
    "M0": ((0, 0), (0, 0), (0, 0)),
    "M1x": ((0, 1), (0, 0), (0, 0)),
    "M1y": ((0, 0), (0, 1), (0, 0)),
    "M1z": ((0, 0), (0, 0), (0, 1)),
    "M2x": ((1, 1), (0, 0), (0, 0)),
    "M2y": ((0, 0), (1, 1), (0, 0)),
    "M2z": ((0, 0), (0, 0), (1, 1)),
}


def overlap_weight(pq, v):
    """1D overlap weight w(v) = int u'^q (u' - v)^p over |u'|<=1/2, |u'-v|<=1/2.

    Closed polynomial forms of the three weights used (derivation in the module
    docstring); pinned against direct numerical integration in the tests.
    """
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    inside = a <= 1.0
    if pq == (0, 0):
        w = 1.0 - a
    elif pq == (0, 1):
        w = v * (1.0 - a) / 2.0
    elif pq == (1, 1):
        t = 1.0 - a
        w = -t / 4.0 + t * t / 2.0 - t ** 3 / 6.0
    else:
        raise ValueError(pq)
    return np.where(inside, w, 0.0)


@functools.lru_cache(maxsize=None)
def _gl01(n):
    """Gauss-Legendre nodes and weights mapped to [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _points_for_distance(dist):
    """GL points per axis for a unit box at Euclidean distance ``dist`` (>=1)
    from the singular point.  Chosen so the Bernstein-ellipse bound of the
    nearest complex singularity is below 1e-17; verified in the tests by
    comparing against a finer rule."""
    if dist >= 30.0:
        return 5
    if dist >= 10.0:
        return 7
    if dist >= 4.0:
        return 9
    if dist >= 2.0:
        return 12
    return 18


def _regular_box_integral(d, lo, hi, pqs):
    """int over v in box [lo, hi] (per axis, within [-1,1]) of prod w(v) g(d+v),
    for a batch of offsets ``d`` (shape (N, 3)) sharing the same box; the box is
    assumed not to contain the singular point."""
    d = np.asarray(d, dtype=np.float64)
    # distance from singular point to the box in s = d + v coordinates
    s_lo = d + lo
    s_hi = d + hi
    gap = np.maximum(0.0, np.maximum(s_lo, -s_hi))
    dist = np.sqrt((gap * gap).sum(axis=1))
    out = np.zeros(d.shape[0])
    ns = np.array([_points_for_distance(x) for x in dist])
    for n in np.unique(ns):
        sel = np.nonzero(ns == n)[0]
        t, wt = _gl01(int(n))
        vx = lo[0] + (hi[0] - lo[0]) * t
        vy = lo[1] + (hi[1] - lo[1]) * t
        vz = lo[2] + (hi[2] - lo[2]) * t
        wx = wt * (hi[0] - lo[0]) * overlap_weight(pqs[0], vx)
        wy = wt * (hi[1] - lo[1]) * overlap_weight(pqs[1], vy)
        wz = wt * (hi[2] - lo[2]) * overlap_weight(pqs[2], vz)
        W = wx[:, None, None] * wy[None, :, None] * wz[None, None, :]
        for c0 in range(0, sel.size, 4096):
            idx = sel[c0:c0 + 4096]
            dd = d[idx]
            X = dd[:, 0, None, None, None] + vx[None, :, None, None]
            Y = dd[:, 1, None, None, None] + vy[None, None, :, None]
            Z = dd[:, 2, None, None, None] + vz[None, None, None, :]
            R = np.sqrt(X * X + Y * Y + Z * Z)
            out[idx] = (W[None] / R).reshape(idx.size, -1).sum(axis=1)
    return out / FOUR_PI


def _corner_box_integral(d, lo, hi, pqs, n_ang=20, n_rad=14):
    """Same integral for one offset whose box has the singular point s = 0 at a
    corner.  In s = d + v the box is prod [0,1] * sign_i; the Duffy pyramid map
    t = rho (1, eta, zeta) (and its two permutations) gives the regular integrand
    W(s) rho / (4 pi sqrt(1 + eta^2 + zeta^2)) on [0,1]^3."""
    d = np.asarray(d, dtype=np.float64)
    s_lo = d + lo
    s_hi = d + hi
    sign = np.where(s_hi > 0.5, 1.0, -1.0)  # box is [0,1] (sign +) or [-1,0] (sign -)
    ta, wa = _gl01(n_ang)
    tr, wr = _gl01(n_rad)
    total = 0.0
    for axis in range(3):
        # pyramid where coordinate `axis` is the largest: t_axis = rho
        rho = tr[:, None, None]
        e1 = ta[None, :, None]
        e2 = ta[None, None, :]
        others = [a for a in range(3) if a != axis]
        t = [None, None, None]
        t[axis] = rho * np.ones_like(e1 * e2)
        t[others[0]] = rho * e1
        t[others[1]] = rho * e2
        v = [sign[i] * t[i] - d[i] for i in range(3)]
        W = (overlap_weight(pqs[0], v[0]) * overlap_weight(pqs[1], v[1])
             * overlap_weight(pqs[2], v[2]))
        integrand = W * rho / np.sqrt(1.0 + e1 * e1 + e2 * e2)
        wts = wr[:, None, None] * wa[None, :, None] * wa[None, None, :]
        total += float((integrand * wts).sum())
    return total / FOUR_PI


def _boxes():
    for bx in (0, 1):
        for by in (0, 1):
            for bz in (0, 1):
                lo = np.array([-1.0 + bx, -1.0 + by, -1.0 + bz])
                yield lo, lo + 1.0


def family_values(name, offsets):
    """Family integral ``name`` (key of FAMILIES) at integer offsets (N, 3).

    Sec. II.A / App. A-B definitions, evaluated as described in the module
    docstring.  Returns float64 array of shape (N,).
    """
    pqs = FAMILIES[name]
    offs = np.atleast_2d(np.asarray(offsets, dtype=np.int64))
    out = np.zeros(offs.shape[0])
    near = np.all(np.abs(offs) <= 1, axis=1)
    df = offs.astype(np.float64)
    for lo, hi in _boxes():
        s_lo = df + lo
        s_hi = df + hi
        contains = np.all((s_lo <= 0.0) & (s_hi >= 0.0), axis=1)
        reg = ~contains
        if reg.any():
            out[reg] += _regular_box_integral(df[reg], lo, hi, pqs)
        for i in np.nonzero(contains)[0]:
            out[i] += _corner_box_integral(df[i], lo, hi, pqs)
    del near
    return out


def family_table(name, Kx, Ky, Kz):
    """Tabulate family ``name`` for offsets d in [0,Kx) x [0,Ky) x [0,Kz).

    Array index order is [dz, dy, dx] (x fastest), matching the voxel ordering
    used throughout (x fastest, then y, then z).
    """
    dz, dy, dx = np.meshgrid(np.arange(Kz), np.arange(Ky), np.arange(Kx), indexing="ij")
    offs = np.stack([dx.ravel(), dy.ravel(), dz.ravel()], axis=1)
    return family_values(name, offs).reshape(Kz, Ky, Kx)
