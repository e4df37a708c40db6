"""Batched Krylov kernels of the library (h2_krylov_dots / h2_krylov_update)
against FP64 numpy, real and complex, with strided basis storage."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05665_amd import h2  # noqa: E402


@pytest.mark.parametrize("cx", [False, True])
@pytest.mark.parametrize("r,m,nvec,n", [(1, 1, 1, 1), (3, 8, 5, 1000), (16, 31, 31, 70001)])
def test_dots_and_update(cx, r, m, nvec, n):
    rng = np.random.default_rng(r * 100 + nvec)
    Q = rng.standard_normal((r, m, n))
    W = rng.standard_normal((r, n))
    if cx:
        Q = Q + 1j * rng.standard_normal(Q.shape)
        W = W + 1j * rng.standard_normal(W.shape)
    Qd, Wd = torch.tensor(Q, device="cuda"), torch.tensor(W, device="cuda")
    h = h2.h2_krylov_dots(Qd, Wd, nvec).cpu().numpy()
    ref = np.einsum("rik,rk->ri", Q[:, :nvec].conj(), W)
    assert np.abs(h - ref).max() <= 1e-12 * np.abs(ref).max()
    hd = torch.tensor(ref, device="cuda")
    h2.h2_krylov_update(Qd, hd, Wd, -0.5)
    out = Wd.cpu().numpy()
    ref2 = W - 0.5 * np.einsum("ri,rik->rk", ref, Q[:, :nvec])
    assert np.abs(out - ref2).max() <= 1e-12 * np.abs(ref2).max()
    # deterministic
    assert np.array_equal(h2.h2_krylov_dots(Qd, Wd, nvec).cpu().numpy(), h2.h2_krylov_dots(Qd, Wd, nvec).cpu().numpy())
