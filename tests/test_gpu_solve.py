"""GPU port solve (FGMRES on the saddle system, eq. 7, with the preconditioner
of eqs. 12-15) against the oracle's dense LU solve of the same system."""
import numpy as np
import pytest

import workloads as wl
from oracle import circuit as cc
from oracle import operator as op

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

F, S0, LAM = 5e9, 1e7, 90e-9


def strips(nstrip=2, length=10, width=2, thick=2, gap=2, ground=False):
    """Parallel x-directed strips, one port each (+ at x = 0, - at the far end),
    optionally over a ground slab two voxels below."""
    Ky = nstrip * (width + gap)
    Kz = thick + (4 if ground else 0)
    mask = np.zeros((Kz, Ky, length), dtype=np.uint8)
    z0 = 4 if ground else 0
    for i in range(nstrip):
        mask[z0:z0 + thick, i * (width + gap):i * (width + gap) + width, :] = 1
    if ground:
        mask[0:2, :, :] = 1
    P = op.voxel_coords(mask)
    ports = []
    for i in range(nstrip):
        ys = range(i * (width + gap), i * (width + gap) + width)
        sel = lambda k: P[k, 1] in ys and P[k, 2] >= z0
        plus = [(k, 0) for k in range(P.shape[0]) if sel(k) and P[k, 0] == 0]
        minus = [(k, 1) for k in range(P.shape[0]) if sel(k) and P[k, 0] == length - 1]
        ports.append((plus, minus))
    return mask, ports


def _oracle(mask, ports, dx):
    P = op.voxel_coords(mask)
    K = P.shape[0]
    fam = op.FamilyCache(mask.shape[2], mask.shape[1], mask.shape[0])
    c = op.material_c(F, S0, LAM) * np.ones(K)
    Z = op.dense_rows(mask, 3, np.arange(3 * K), fam, 1j * 2 * np.pi * F * op.MU0 * dx, c, dx)
    A, node_of, _ = cc.incidence(mask)
    pn = cc.port_nodes(mask, node_of, ports)
    Y, X, free, b = cc.solve_ports(Z, A, pn)
    return Y, X[:3 * K]


def _gpu(mask, ports, dx, transpose=False, restart=50):
    import paper_2105_08627_amd as svh
    p = svh.Problem(mask, dx)
    p.set_material([F], S0, LAM)
    p.setup_tensors()
    p.set_ports(ports)
    X, Y, info = p.solve(0, rre=1e-10, restart=restart, maxit=400, transpose=transpose)
    return p, X.cpu().numpy(), Y, info


@pytest.mark.parametrize("case", [dict(nstrip=1, length=8), dict(nstrip=2, length=10),
                                  dict(nstrip=3, length=12, ground=True)])
def test_port_solve_matches_dense_lu(case):
    dx = 0.5e-6
    mask, ports = strips(**case)
    Yo, Io = _oracle(mask, ports, dx)
    p, X, Y, info = _gpu(mask, ports, dx)
    print(case, info["iterations"], info["inner_iterations"], info["relres"])
    assert info["converged"] and info["relres"] <= 1e-10 * 2
    K3 = 3 * p.K
    for q in range(len(ports)):
        e = np.linalg.norm(X[q, :K3] - Io[:, q]) / np.linalg.norm(Io[:, q])
        assert e <= 1e-8, (q, e)
    assert np.abs(Y - Yo).max() <= 1e-8 * np.abs(Yo).max()
    assert np.abs(Y - Y.T).max() <= 1e-8 * np.abs(Y).max()  # reciprocity


def test_restarts_converge():
    """A short restart length forces several restart cycles."""
    dx = 0.5e-6
    mask, ports = strips(nstrip=2, length=10, ground=True)
    Yo, _ = _oracle(mask, ports, dx)
    p, X, Y, info = _gpu(mask, ports, dx, restart=3)
    assert info["restarts"] > 1 and info["converged"]
    assert np.abs(Y - Yo).max() <= 1e-8 * np.abs(Yo).max()


def test_adjoint_solution_identity():
    """K^T y = [b; 0] is solved by y = [x_I; -x_Phi] because Z is symmetric."""
    dx = 0.5e-6
    mask, ports = strips(nstrip=2, length=10)
    p, X, Y, info = _gpu(mask, ports, dx)
    _, Xt, Yt, info_t = _gpu(mask, ports, dx, transpose=True)
    K3 = 3 * p.K
    assert info_t["converged"]
    assert np.linalg.norm(Xt[:, :K3] - X[:, :K3]) <= 1e-9 * np.linalg.norm(X[:, :K3])
    assert np.linalg.norm(Xt[:, K3:] + X[:, K3:]) <= 1e-9 * np.linalg.norm(X[:, K3:])
    assert np.abs(Yt - Y).max() <= 1e-9 * np.abs(Y).max()


def test_fp32_refinement_matches_fp64_and_oracle():
    """FP32 operator inside FP64 iterative refinement reaches the FP64
    tolerance; its admittance matches the FP64 solve and the dense oracle."""
    import paper_2105_08627_amd as svh
    dx = 0.5e-6
    mask, ports = strips(nstrip=3, length=12, ground=True)
    Yo, Io = _oracle(mask, ports, dx)
    p = svh.Problem(mask, dx)
    p.set_material([F], S0, LAM)
    p.setup_tensors()
    p.tucker_compress(1e-10)
    p.set_ports(ports)
    X64, Y64, i64 = p.solve(0, rre=1e-10, restart=30)
    Xir, Yir, iir = p.solve(0, rre=1e-10, restart=30, refine=True)
    print("fp64", i64, "ir", iir)
    assert iir["converged"] and iir["refinement_steps"] >= 2
    assert iir["relres"] <= 2e-10
    assert np.abs(Yir - Y64).max() <= 1e-8 * np.abs(Y64).max()
    assert np.abs(Yir - Yo).max() <= 1e-8 * np.abs(Yo).max()


def test_graph_replay_equals_eager():
    """The preconditioner's CG block replayed from a HIP graph (many replays
    with eager kernels and synchronisations between them) gives bitwise the
    same solution as launching every kernel directly."""
    import paper_2105_08627_amd as svh
    dx = 0.5e-6
    mask, ports = strips(nstrip=2, length=10, ground=True)
    p = svh.Problem(mask, dx)
    p.set_material([F], S0, LAM)
    p.setup_tensors()
    p.set_ports(ports)
    p.set_graphs(False)
    Xe, Ye, ie = p.solve(0, rre=1e-10)
    p.set_graphs(True)
    for _ in range(3):
        Xg, Yg, ig = p.solve(0, rre=1e-10)
        assert torch.equal(Xe, Xg)
        assert ig["inner_iterations"] == ie["inner_iterations"]


@pytest.mark.parametrize("basis", [3, 5])
def test_multigrid_schur_preconditioner(basis):
    """The aggregation multigrid V-cycle (default) and the Jacobi diagonal
    precondition the same Schur-complement CG: same admittance to the solve
    tolerance, far fewer inner iterations; matches the dense LU oracle."""
    import paper_2105_08627_amd as svh
    dx = 0.5e-6
    if basis == 3:
        mask, ports = strips(nstrip=3, length=24, ground=True)
    else:
        mask, ports = wl.square_bend(3, 14)
    res = {}
    for kind in ("jacobi", "amg"):
        p = svh.Problem(mask, dx, basis=basis)
        p.set_material([F], S0, LAM)
        p.setup_tensors()
        p.set_ports(ports)
        p.set_schur_precond(kind)
        X, Y, info = p.solve(0, rre=1e-10, restart=50, maxit=400)
        assert info["converged"], (kind, info)
        res[kind] = (Y, info["inner_iterations"], info["iterations"])
    print(basis, {k: v[1:] for k, v in res.items()})
    Yj, Ya = res["jacobi"][0], res["amg"][0]
    assert np.abs(Ya - Yj).max() <= 1e-8 * np.abs(Yj).max()
    assert res["amg"][1] < res["jacobi"][1]
    if basis == 3:
        Yo, _ = _oracle(mask, ports, dx)
        assert np.abs(Ya - Yo).max() <= 1e-8 * np.abs(Yo).max()
