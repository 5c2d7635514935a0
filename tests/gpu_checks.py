"""Checks of port solutions shared by the GPU tests (not a test module).

check_solution: the residual of the saddle system of eq. 7 evaluated with the
oracle's face-flux entries of A (every current row and every free node),
the library supplying only Z I, and the admittance as the current entering
each + terminal.
"""
import numpy as np
import torch

from oracle import circuit as cc
from oracle import operator as op


def _node_index(mask):
    """(K, 6) node index of every voxel face in the library's node order
    (face grid: x faces, then y faces, then z faces, each with x fastest,
    then y, then z; only faces of non-empty voxels are nodes)."""
    Kz, Ky, Kx = mask.shape
    P = op.voxel_coords(mask)
    dims = [(Kx + 1, Ky, Kz), (Kx, Ky + 1, Kz), (Kx, Ky, Kz + 1)]
    off = np.cumsum([0] + [a * b * c for a, b, c in dims])
    ids = np.zeros((P.shape[0], 6), dtype=np.int64)
    for f in range(6):
        a, s = divmod(f, 2)
        q = P.copy()
        q[:, a] += s
        X, Y, _ = dims[a]
        ids[:, f] = off[a] + (q[:, 2] * Y + q[:, 1]) * X + q[:, 0]
    used = np.unique(ids)
    return np.searchsorted(used, ids), used.size


def check_solution(p, mask, basis, ports, X, Y, rre, cols):
    """Residual of eq. 7 from the oracle's face fluxes (all rows) and the
    admittance as terminal currents, for the port columns `cols`."""
    K = p.K
    CK = basis * K
    node, M = _node_index(mask)
    assert M == p.M
    plus = [np.unique([node[k, f] for k, f in pl]) for pl, _ in ports]
    Xh = X.cpu().numpy()
    I = Xh[:, :CK].reshape(-1, basis, K)
    ZI = p.matvec(torch.from_numpy(np.ascontiguousarray(I[cols])).to(X.device), [0] * len(cols)).cpu().numpy()
    terminals = np.unique(np.concatenate([node[k, f][None] for pl, mi in ports for k, f in pl + mi]))
    free = np.ones(M, dtype=bool)
    free[terminals] = False
    for ci, q in enumerate(cols):
        phi = Xh[q, CK:].copy()
        phi[plus[q]] = 1.0
        inj = np.zeros(M, dtype=np.complex128)
        top = ZI[ci].copy()
        bvec = np.zeros((basis, K))
        hot = np.zeros(M)
        hot[plus[q]] = 1.0
        for beta in range(basis):
            for f, a in cc.basis_face_flux(beta):
                np.add.at(inj, node[:, f], a * I[q, beta])
                top[beta] -= a * phi[node[:, f]]
                bvec[beta] += a * hot[node[:, f]]
        res = np.sqrt(np.sum(np.abs(top) ** 2) + np.sum(np.abs(inj[free]) ** 2)) / np.linalg.norm(bvec)
        print(f"[check] port {q}: residual of eq. 7 with the oracle's fluxes {res:.2e}", flush=True)
        assert res <= 1.5 * rre, (q, res)
        Yq = np.array([inj[pl].sum() for pl in plus])
        assert np.abs(Yq - Y[:, q]).max() <= 1e-10 * np.abs(Y).max(), q
