"""Adjoint matvec, adjoint solve and the gradient of port inductance with
respect to the per-voxel kinetic parameter p = lambda^-2 (eq. 3): against the
oracle's dense adjoint and against central finite differences."""
import numpy as np
import pytest

import workloads as wl
from oracle import circuit as cc
from oracle import operator as op

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

F, S0 = 8e9, 1e7


def bend_like(seed=1003):
    """Two coupled strips over a ground slab; per-voxel London depth drawn
    uniformly in 80-120 nm (stand-in for the bend workload, which needs the
    piecewise-linear basis)."""
    mask = np.zeros((6, 8, 14), dtype=np.uint8)
    mask[0:2, :, :] = 1
    mask[4:6, 1:3, :] = 1
    mask[4:6, 5:7, :] = 1
    P = op.voxel_coords(mask)
    ports = []
    for ys in ([1, 2], [5, 6]):
        sel = [k for k in range(P.shape[0]) if P[k, 2] >= 4 and P[k, 1] in ys]
        ports.append(([(k, 0) for k in sel if P[k, 0] == 0], [(k, 1) for k in sel if P[k, 0] == 13]))
    lam = np.random.default_rng(seed).uniform(80e-9, 120e-9, P.shape[0])
    return mask, ports, lam


def _problem(mask, ports, lam, dx):
    import paper_2105_08627_amd as svh
    p = svh.Problem(mask, dx)
    p.set_material([F], np.full(lam.size, S0), lam, per_voxel=True)
    p.setup_tensors()
    p.set_ports(ports)
    return p


def test_adjoint_matvec_dot_test():
    import paper_2105_08627_amd as svh
    mask = wl.random_mask(9, 10, 7, 5, fill=0.6)
    p = svh.Problem(mask, 0.5e-6)
    p.set_material([F], S0, 90e-9)
    p.setup_tensors()
    dev = torch.device("cuda")
    u = torch.from_numpy(wl.random_currents(1, (1, 3, p.K))).to(dev)
    v = torch.from_numpy(wl.random_currents(2, (1, 3, p.K))).to(dev)
    a = torch.sum(v * p.matvec(u, [0])).item()
    b = torch.sum(u * p.matvec_adjoint(v, [0])).item()
    assert abs(a - b) <= 1e-13 * abs(a)


def test_gradient_matches_dense_adjoint():
    dx = 0.25e-6
    mask, ports, lam = bend_like()
    p = _problem(mask, ports, lam, dx)
    X, Y, info = p.solve(0, rre=1e-12)
    Xa, Ya, info_a = p.solve(0, rre=1e-12, transpose=True)
    dY = p.port_gradient(0, X, Xa).cpu().numpy()
    # oracle: dense saddle system and its transpose, solved directly
    K = p.K
    fam = op.FamilyCache(mask.shape[2], mask.shape[1], mask.shape[0])
    c = op.material_c(F, S0, lam)
    w = 2 * np.pi * F
    Z = op.dense_rows(mask, 3, np.arange(3 * K), fam, 1j * w * op.MU0 * dx, c, dx)
    A, node_of, _ = cc.incidence(mask)
    pn = cc.port_nodes(mask, node_of, ports)
    dirn = sorted({m for pl, mi in pn for m in pl + mi})
    dirn = cc.ground_floating(A, dirn)
    Kmat, free = cc.saddle_system(Z, A, dirn)
    b = np.stack([A[pl].sum(axis=0) for pl, _ in pn], axis=1)
    rhs = np.zeros((Kmat.shape[0], len(pn)), dtype=complex)
    rhs[:3 * K] = b
    Xo = np.linalg.solve(Kmat, rhs)[:3 * K]
    Yadj = np.linalg.solve(Kmat.T, rhs)[:3 * K]
    dz = 1j * c ** 2 / (w * op.MU0 * dx)
    ref = np.zeros((len(pn), len(pn), K), dtype=complex)
    for q in range(len(pn)):
        for pp in range(len(pn)):
            s = (Yadj[:, q] * Xo[:, pp]).reshape(3, K).sum(axis=0)
            ref[q, pp] = -s * dz
    err = np.abs(dY - ref).max() / np.abs(ref).max()
    print("gradient vs dense adjoint", err, info["iterations"], info_a["iterations"])
    assert err <= 1e-8


def test_inductance_gradient_vs_finite_differences():
    """dL/dp_k through the autograd function against central differences
    (step 1e-4 relative) on 8 seeded voxels, solves to relative residual 1e-12."""
    from paper_2105_08627_amd.autograd import port_inductance
    dx = 0.25e-6
    mask, ports, lam = bend_like()
    p = _problem(mask, ports, lam, dx)
    dev = torch.device("cuda")
    pv = torch.tensor(lam ** -2.0, dtype=torch.float64, device=dev, requires_grad=True)
    L = port_inductance(p, pv, S0, F, rre=1e-12)
    loss = L[0, 0] + 0.5 * L[0, 1]
    loss.backward()
    g = pv.grad.cpu().numpy()
    rng = np.random.default_rng(1003)
    for k in rng.choice(p.K, size=8, replace=False):
        h = 1e-4 * pv[k].item()
        vals = []
        for sgn in (+1, -1):
            pp = pv.detach().clone()
            pp[k] += sgn * h
            Lk = port_inductance(p, pp, S0, F, rre=1e-12)
            vals.append((Lk[0, 0] + 0.5 * Lk[0, 1]).item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(g[k] - fd) <= 1e-3 * abs(g[k]) + 1e-6 * np.abs(g).max(), (k, g[k], fd)


def test_port_inductance_and_contraction_through_the_abi():
    """svh_port_inductance (Z = Y^-1, L = Im Z / w) and svh_gradient_contract
    (W = Z^T G Z^T formed in the library) against the same algebra written
    out here with numpy on the library's own Y and dY."""
    dx = 0.25e-6
    mask, ports, lam = bend_like()
    p = _problem(mask, ports, lam, dx)
    X, Y, _ = p.solve(0, rre=1e-12)
    Xa, _, _ = p.solve(0, rre=1e-12, transpose=True)
    dY = p.port_gradient(0, X, Xa)
    Z, L = p.port_inductance(0, Y)
    w = 2 * np.pi * F
    Zref = np.linalg.inv(Y)
    assert np.abs(Z - Zref).max() <= 1e-13 * np.abs(Zref).max()
    assert np.abs(L - Zref.imag / w).max() <= 1e-13 * np.abs(Zref.imag / w).max()
    G = np.array([[1.0, 0.5], [-0.25, 2.0]])
    g = p.gradient_contract(0, Y, G, dY).cpu().numpy()
    W = Zref.T @ G @ Zref.T
    ref = -np.imag(np.einsum("ab,abk->k", W, dY.cpu().numpy())) / w
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


def test_autograd_backward_uses_the_forward_material():
    """Two forward calls with different materials before the first backward:
    the first backward must still give the gradient of its own forward."""
    from paper_2105_08627_amd.autograd import port_inductance
    dx = 0.25e-6
    mask, ports, lam = bend_like()
    p = _problem(mask, ports, lam, dx)
    dev = torch.device("cuda")
    pv1 = torch.tensor(lam ** -2.0, dtype=torch.float64, device=dev, requires_grad=True)
    L1 = port_inductance(p, pv1, S0, F, rre=1e-12)
    pv2 = torch.tensor((1.3 * lam) ** -2.0, dtype=torch.float64, device=dev, requires_grad=True)
    L2 = port_inductance(p, pv2, S0, F, rre=1e-12)
    L1[0, 0].backward()
    g_interleaved = pv1.grad.cpu().numpy()
    pv3 = torch.tensor(lam ** -2.0, dtype=torch.float64, device=dev, requires_grad=True)
    port_inductance(p, pv3, S0, F, rre=1e-12)[0, 0].backward()
    g_fresh = pv3.grad.cpu().numpy()
    assert np.abs(g_interleaved - g_fresh).max() <= 1e-9 * np.abs(g_fresh).max()
    del L2
