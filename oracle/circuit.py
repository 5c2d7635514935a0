"""Saddle system, ports and direct solve (oracle; test infrastructure only).

Readings (the entries of A, Phi, V and I are defined in the cited VoxHenry
work, not in this paper):
  * nodes are the centres of the faces of non-empty voxels (Sec. II.A);
  * A[m, (k, beta)] is the current that basis (k, beta) draws from face node m
    into voxel k, i.e. minus its outward flux through that face.  For the
    piecewise-constant f^a (total current 1): +1 at the -a face, -1 at the +a
    face (eq. 7: A I = 0 is current conservation, eq. 2, at every node);
  * with the potential-gradient term of eq. 1, the first block row of eq. 7
    is Z I - A^T Phi = V; a port fixes Phi = 1 on its + terminal faces and
    Phi = 0 on its - terminal faces and on every other port's faces (these
    nodes are Dirichlet nodes); moving them to the right-hand side gives
        [Z  -A_F^T] [I    ]   [A_D^T Phi_D]
        [A_F   0  ] [Phi_F] = [     0     ]
  * the admittance Y_qp is the current entering port q's + terminal when
    port p is driven: Y_qp = b_q^T I^(p) with b_q = A_{q+}^T 1; the port
    impedance matrix is Y^-1 and the port inductance Im(Z)/w;
  * every connected conductor region with no Dirichlet node has one of its
    nodes grounded (Phi = 0): its conservation rows sum to zero, so the
    potential is defined only up to a constant there.
"""
from __future__ import annotations

import numpy as np

from . import operator as op

# face codes: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z
_AX = {0: 0, 1: 0, 2: 1, 3: 1, 4: 2, 5: 2}


def face_nodes(mask):
    """Unique face-centre nodes of the non-empty voxels.

    Returns (node_of, nodes): node_of[(axis, i, j, k)] -> node index, where
    (i, j, k) is the face's integer position (the face between voxels at
    coordinate c-1 and c along `axis` has coordinate c); nodes lists the keys
    in index order."""
    P = op.voxel_coords(mask)
    keys = []
    for p in P:
        for a in range(3):
            for s in (0, 1):
                q = list(p)
                q[a] += s
                keys.append((a, q[0], q[1], q[2]))
    uniq = sorted(set(keys))
    return {k: i for i, k in enumerate(uniq)}, uniq


def voxel_face_node(node_of, p, face):
    a = _AX[face]
    q = list(p)
    q[a] += face % 2
    return node_of[(a, q[0], q[1], q[2])]


def basis_face_flux(beta):
    """(face code, A entry) pairs of basis function beta of a voxel: the
    current it draws from each face node into the voxel (readings in the
    module docstring).  beta 0-2: f^x, f^y, f^z, +1 at the -a face and -1 at
    the +a face; 3: f^2D (eq. 5), -1/2 at both x faces and +1/2 at both y
    faces; 4: f^3D (eq. 6), -1/2 at the four x and y faces and +1 at both z
    faces (/dx^2 normalisation, so every function has zero net flux)."""
    if beta < 3:
        return [(2 * beta, 1.0), (2 * beta + 1, -1.0)]
    if beta == 3:
        return [(0, -0.5), (1, -0.5), (2, 0.5), (3, 0.5)]
    return [(0, -0.5), (1, -0.5), (2, -0.5), (3, -0.5), (4, 1.0), (5, 1.0)]


def incidence(mask, basis=3):
    """Dense incidence matrix A (M x basis*K), entries from basis_face_flux."""
    node_of, nodes = face_nodes(mask)
    P = op.voxel_coords(mask)
    K = P.shape[0]
    A = np.zeros((len(nodes), basis * K))
    for k, p in enumerate(P):
        for beta in range(basis):
            for f, a in basis_face_flux(beta):
                A[voxel_face_node(node_of, p, f), beta * K + k] += a
    return A, node_of, nodes


def ground_floating(A, dirichlet):
    """Dirichlet set extended by one node per connected region that has none."""
    M, N = A.shape
    parent = list(range(M))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i
    for col in range(N):
        ms = np.nonzero(A[:, col])[0]
        for m in ms[1:]:
            ra, rb = find(ms[0]), find(m)
            if ra != rb:
                parent[rb] = ra
    d = set(dirichlet)
    has = {find(m) for m in d}
    for m in range(M):
        r = find(m)
        if r not in has:
            d.add(m)
            has.add(r)
    return sorted(d)


def port_nodes(mask, node_of, ports):
    """ports: list of (plus_faces, minus_faces), each a list of (k, face)."""
    P = op.voxel_coords(mask)
    out = []
    for plus, minus in ports:
        out.append(([voxel_face_node(node_of, P[k], f) for k, f in plus],
                    [voxel_face_node(node_of, P[k], f) for k, f in minus]))
    return out


def saddle_system(Z, A, dirichlet):
    """Dense saddle matrix [[Z, -A_F^T], [A_F, 0]] on the free nodes."""
    M = A.shape[0]
    free = np.setdiff1d(np.arange(M), dirichlet)
    AF = A[free]
    n = Z.shape[0]
    Kmat = np.zeros((n + free.size, n + free.size), dtype=np.complex128)
    Kmat[:n, :n] = Z
    Kmat[:n, n:] = -AF.T
    Kmat[n:, :n] = AF
    return Kmat, free


def solve_ports(Z, A, pnodes, extra_dirichlet=()):
    """Direct (LU) solve for every port excitation.

    Returns (Y, X, free, b): admittance matrix Y[q, p], solutions X[:, p]
    (currents then free-node potentials), the free node list and the port
    vectors b[:, q] = A_{q+}^T 1."""
    dir_nodes = set(extra_dirichlet)
    for plus, minus in pnodes:
        dir_nodes.update(plus)
        dir_nodes.update(minus)
    dirichlet = ground_floating(A, sorted(dir_nodes))
    Kmat, free = saddle_system(Z, A, dirichlet)
    n = Z.shape[0]
    npt = len(pnodes)
    b = np.zeros((n, npt))
    for q, (plus, _) in enumerate(pnodes):
        b[:, q] = A[plus].sum(axis=0)
    rhs = np.zeros((Kmat.shape[0], npt), dtype=np.complex128)
    rhs[:n] = b
    X = np.linalg.solve(Kmat, rhs)
    Y = b.T @ X[:n]
    return Y, X, free, b
