"""Dense Galerkin operator, circulant embedding and FFT convolution (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions (readings where the paper is silent):
  * voxels are ordered x fastest, then y, then z; the unknown vector is
    component-major, [I^x; I^y; I^z; (I^2D; I^3D)] (eq. 7);
  * basis functions carry total current: f^x = x_hat / dx^2 and the linear
    functions of eqs. 5-6 are divided by dx^2 as well, so the diagonal terms
    are c/dx, c/(6 dx), c/(2 dx) exactly as stated under eq. 9 and in eqs. 16-18;
  * with that normalisation every block is  j w mu dx * B(d)  with B built from
    the unit-voxel families of ``oracle.green`` (eq. 8, App. A, App. B);
  * mu = mu0 = 4 pi 1e-7 H/m (Sec. II.A takes mu = mu0).
"""
from __future__ import annotations

import numpy as np

from . import green

MU0 = 4.0e-7 * np.pi

# Basis functions per eqs. 4-6 in unit-voxel coordinates u (voxel centre at 0):
# each is a list of (vector component a, coefficient, power of u_a).
BASIS = {
    "x": [(0, 1.0, 0)],
    "y": [(1, 1.0, 0)],
    "z": [(2, 1.0, 0)],
    "2D": [(0, 1.0, 1), (1, -1.0, 1)],           # eq. 5
    "3D": [(0, 1.0, 1), (1, 1.0, 1), (2, -2.0, 1)],  # eq. 6
}
BASIS_SETS = {3: ["x", "y", "z"], 5: ["x", "y", "z", "2D", "3D"]}

_AX = "xyz"


def material_c(f_hz, sigma0, lam):
    """c = 1/sigma with the two-fluid conductivity sigma = sigma0 - j/(w mu lam^2)
    (eq. 3).  Returns complex128 broadcast over the inputs."""
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    sigma = np.asarray(sigma0, dtype=np.float64) - 1j / (w * MU0 * np.asarray(lam, dtype=np.float64) ** 2)
    return 1.0 / sigma


def material_ab(f_hz, sigma0, lam):
    """a and b of eqs. 22-23 (App. A); c = a + j w mu b."""
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    s0 = np.asarray(sigma0, dtype=np.float64)
    l2 = np.asarray(lam, dtype=np.float64) ** 2
    den = 1.0 + (s0 * w * MU0 * l2) ** 2
    a = s0 * (w * MU0 * l2) ** 2 / den
    b = l2 / den
    return a, b


def block_terms(beta, alpha):
    """Galerkin block (beta, alpha) of eq. 8 as a list of (coef, family name),
    derived from the basis definitions: the product f^beta_l . f^alpha_k picks
    matching vector components a; observer power p and source power q select
    the family (p,q)=(0,0) -> M0, (0,1) -> M1_a, (1,0) -> -M1_a (observer moment,
    by the substitution (u,u') -> (-u',-u)), (1,1) -> M2_a."""
    terms = []
    for (a, cb, p) in BASIS[beta]:
        for (a2, ca, q) in BASIS[alpha]:
            if a != a2:
                continue
            coef = cb * ca
            if (p, q) == (0, 0):
                terms.append((coef, "M0"))
            elif (p, q) == (0, 1):
                terms.append((coef, "M1" + _AX[a]))
            elif (p, q) == (1, 0):
                terms.append((-coef, "M1" + _AX[a]))
            else:
                terms.append((coef, "M2" + _AX[a]))
    return terms


def mass_coefficient(beta, alpha):
    """int_{unit voxel} f^beta . f^alpha du (unit coordinates); the diagonal
    term of block (beta, alpha) is c/dx times this (eqs. 9, 16-18)."""
    mom = {0: 1.0, 1: 0.0, 2: 1.0 / 12.0}
    s = 0.0
    for (a, cb, p) in BASIS[beta]:
        for (a2, ca, q) in BASIS[alpha]:
            if a == a2:
                # the three axis integrals: the power sits on axis a, others give 1
                s += cb * ca * mom[p + q]
    return s


def voxel_coords(mask):
    """Integer (x, y, z) coordinates of the non-empty voxels of ``mask``
    (array indexed [z, y, x]) in the compact order (x fastest)."""
    zz, yy, xx = np.nonzero(mask)
    order = np.lexsort((xx, yy, zz))
    return np.stack([xx[order], yy[order], zz[order]], axis=1)


class FamilyCache:
    """Family values at arbitrary offsets, computed on demand from full tables
    over [0, K) per axis and the parity of each family (M0, M2 even in every
    axis; M1_a odd in axis a, even in the others; pinned in the tests)."""

    def __init__(self, Kx, Ky, Kz):
        self.K = (Kx, Ky, Kz)
        self.tables = {}

    def table(self, name):
        if name not in self.tables:
            self.tables[name] = green.family_table(name, *self.K)
        return self.tables[name]

    def values(self, name, offsets):
        t = self.table(name)
        ad = np.abs(offsets)
        v = t[ad[..., 2], ad[..., 1], ad[..., 0]]
        if name.startswith("M1"):
            a = _AX.index(name[2])
            v = v * np.sign(offsets[..., a])
        return v


def dense_rows(mask, basis, rows, fam, scale_conv=1.0, diag_c=None, dx=1.0):
    """Rows of the dense operator Z (eq. 7 top-left block; eq. 8 layout).

    ``rows`` are global row indices into the component-major unknown vector
    (row = beta * K + l).  Entry (beta l, alpha k) = scale_conv * B^{beta alpha}(
    p_k - p_l) + delta_lk * mass(beta, alpha) * diag_c[l] / dx.  With
    scale_conv = j w mu dx this is the physical operator; scale_conv = 1 and
    diag_c = None give the bare unit-voxel convolution.
    """
    names = BASIS_SETS[basis]
    P = voxel_coords(mask)
    K = P.shape[0]
    rows = np.asarray(rows)
    out = np.zeros((rows.size, basis * K), dtype=np.complex128)
    for ri, row in enumerate(rows):
        b, l = divmod(int(row), K)
        off = P - P[l]  # source minus observer
        for a_i, alpha in enumerate(names):
            acc = np.zeros(K)
            for coef, fname in block_terms(names[b], alpha):
                acc += coef * fam.values(fname, off)
            out[ri, a_i * K:(a_i + 1) * K] = scale_conv * acc
            if diag_c is not None:
                out[ri, a_i * K + l] += mass_coefficient(names[b], alpha) * diag_c[l] / dx
    return out


def dense_matvec(mask, basis, x, fam, scale_conv=1.0, diag_c=None, dx=1.0, row_block=256):
    """y = Z x by plain dense summation, O(N^2) (the matrix-vector product that
    eq. 9 accelerates).  ``x`` has shape (basis*K,) or (nvec, basis*K)."""
    x = np.asarray(x, dtype=np.complex128)
    single = x.ndim == 1
    X = x[None] if single else x
    N = X.shape[1]
    Y = np.zeros_like(X)
    for r0 in range(0, N, row_block):
        rows = np.arange(r0, min(N, r0 + row_block))
        Zr = dense_rows(mask, basis, rows, fam, scale_conv, diag_c, dx)
        Y[:, rows] = X @ Zr.T
    return Y[0] if single else Y


def embed(B_of_offset, K, L):
    """Circulant embedding of a Toeplitz kernel (Sec. II.A, after eq. 8).

    The correlation y_m = sum_n B(n - m) x_n equals the circular convolution
    with h_j = B(-j) placed at j mod L for |j_i| < K_i and zero elsewhere
    (requires L_i >= 2 K_i - 1).  ``B_of_offset`` maps an (N,3) offset array to
    values.  Returns the real array E indexed [z, y, x] of shape L[::-1]."""
    Kx, Ky, Kz = K
    Lx, Ly, Lz = L
    jz, jy, jx = np.meshgrid(np.arange(-Kz + 1, Kz), np.arange(-Ky + 1, Ky),
                             np.arange(-Kx + 1, Kx), indexing="ij")
    offs = -np.stack([jx.ravel(), jy.ravel(), jz.ravel()], axis=1)
    vals = B_of_offset(offs)
    E = np.zeros((Lz, Ly, Lx))
    E[jz.ravel() % Lz, jy.ravel() % Ly, jx.ravel() % Lx] = vals
    return E


def spectrum_convolution(mask, H, x):
    """Bare eq. 9 product of one component with a given circulant spectrum H
    (array [Lz, Ly, Lx]): zero-pad x onto the L grid, FFT, multiply by H,
    inverse FFT, crop to the non-empty voxels.  Used with spectra rebuilt from
    Tucker factors (eq. 10) to check a compressed operator."""
    P = voxel_coords(mask)
    g = np.zeros(H.shape, dtype=np.complex128)
    g[P[:, 2], P[:, 1], P[:, 0]] = np.asarray(x, dtype=np.complex128)
    return np.fft.ifftn(H * np.fft.fftn(g))[P[:, 2], P[:, 1], P[:, 0]]


def fft_matvec(mask, basis, x, fam, L, scale_conv=1.0, diag_c=None, dx=1.0):
    """y = Z x through eq. 9 with numpy FFTs: every block's kernel is embedded
    and transformed, each I^alpha is zero-padded to L, the products are summed
    over alpha, inverse-transformed, cropped, and the diagonal term is added.
    Independent cross-check of ``dense_matvec``."""
    names = BASIS_SETS[basis]
    Kx, Ky, Kz = mask.shape[2], mask.shape[1], mask.shape[0]
    P = voxel_coords(mask)
    K = P.shape[0]
    x = np.asarray(x, dtype=np.complex128).reshape(basis, K)
    Xf = []
    for a in range(basis):
        g = np.zeros((L[2], L[1], L[0]), dtype=np.complex128)
        g[P[:, 2], P[:, 1], P[:, 0]] = x[a]
        Xf.append(np.fft.fftn(g))
    y = np.zeros((basis, K), dtype=np.complex128)
    for b in range(basis):
        acc = np.zeros_like(Xf[0])
        for a in range(basis):
            terms = block_terms(names[b], names[a])
            if not terms:
                continue
            def B(offs, terms=terms):
                return sum(c * fam.values(n, offs) for c, n in terms)
            H = np.fft.fftn(embed(B, (Kx, Ky, Kz), L))
            acc += H * Xf[a]
        conv = np.fft.ifftn(acc)
        y[b] = scale_conv * conv[P[:, 2], P[:, 1], P[:, 0]]
        if diag_c is not None:
            for a in range(basis):
                y[b] += mass_coefficient(names[b], names[a]) * diag_c / dx * x[a]
    return y.reshape(-1)
