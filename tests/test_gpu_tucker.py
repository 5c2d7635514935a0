"""The library's Tucker compression against the oracle's Algorithm 1.

The library computes the Tucker factors of the circulant spectrum through the
weighted Toeplitz tensor (a different route to the same HOSVD), so
  * its multilinear ranks must equal those of the oracle's Algorithm 1
    (``oracle.tucker.tucker_svd``) run on fftn(embed(T)), the spectrum itself;
  * its truncated operator must equal the oracle's product with the oracle's
    own truncated reconstruction (eq. 10) far below the truncation error: the
    HOSVD projection onto the leading singular subspaces is unique, so the two
    differ only by rounding and SVD accuracy;
  * the restored circulant kernel, observed through impulse responses of the
    bare convolution (E at the offsets the cropped product reads), differs
    from the exact one by at most tol * ||E||_F: with unnormalised DFTs
    ||dE||_F = ||dZ||_F / sqrt(Lt) <= tol ||Z||_F / sqrt(Lt) = tol ||E||_F.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import operator as op
from oracle import tucker

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU test needs a device"
    return torch.device("cuda")


@pytest.fixture(scope="module")
def exact():
    """Exact spectrum of the 16 x 16 x 8 grid (L = 32 x 32 x 16) from the oracle."""
    K = (16, 16, 8)
    L = (32, 32, 16)
    fam = op.FamilyCache(*K)
    E = op.embed(lambda o: fam.values("M0", o), K, L)
    Z = np.fft.fftn(E)
    assert np.abs(Z.imag).max() <= 1e-15 * np.abs(Z.real).max()
    return K, L, E, Z.real


def _bare(p, x, dev):
    xt = torch.from_numpy(np.asarray(x, dtype=np.complex128)).to(dev).contiguous()
    y = p.matvec(xt, [-1] * x.shape[0])
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("zstep", ["fft", "direct", "fused"])
@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-8])
def test_ranks_and_reconstruction_match_algorithm_1(dev, exact, tol, zstep):
    import paper_2105_08627_amd as svh
    K, L, E, Z = exact
    mask = wl.full_box(*K)
    p = svh.Problem(mask, 0.25e-6)
    p.set_material([10e9], 1e7, 90e-9)
    p.setup_tensors()
    p.set_zstep(zstep)
    assert tuple(p.L) == L
    ranks, bound = p.tucker_compress(tol)
    core, F = tucker.tucker_svd(Z, tol)  # numpy axes (z, y, x)
    ranks_oracle = (F[2].shape[1], F[1].shape[1], F[0].shape[1])
    print("ranks library", ranks, "oracle", ranks_oracle, "bound", bound)
    assert tuple(ranks) == ranks_oracle
    Zt = tucker.tucker_full(core, F)
    err_spec = np.linalg.norm(Zt - Z) / np.linalg.norm(Z)
    assert err_spec <= tol

    # truncated operator: library vs the oracle's product with its own Zt
    x = wl.random_currents(2300, (1, 3, p.K))
    y = _bare(p, x, dev)[0]
    ref = np.stack([op.spectrum_convolution(mask, Zt, x[0, a]) for a in range(3)])
    d = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"tol {tol:g} {zstep}: library vs oracle-truncated operator {d:.2e} (truncation {err_spec:.2e})")
    assert d <= 1e-3 * tol

    # restored kernel through impulse responses at the first and last voxel
    imp = np.zeros((2, 3, p.K), dtype=np.complex128)
    imp[0, 0, 0] = 1.0
    imp[1, 0, p.K - 1] = 1.0
    r = _bare(p, imp, dev)[:, 0].real
    P = op.voxel_coords(mask)
    Lx, Ly, Lz = L
    got, want = [], []
    for i, src in enumerate((P[0], P[-1])):
        off = P - src  # observer minus source: the product reads E at -(source - observer)
        got.append(r[i])
        want.append(E[off[:, 2] % Lz, off[:, 1] % Ly, off[:, 0] % Lx])
    dE = np.linalg.norm(np.concatenate(got) - np.concatenate(want))
    print(f"impulse responses: |dE| / |E| = {dE / np.linalg.norm(E):.2e}")
    assert dE <= tol * np.linalg.norm(E)
