"""The product captured in a HIP graph (through torch.cuda.CUDAGraph on the
capturing stream): every replay gives bitwise the eager result, with eager
products and host synchronisations between the replays, for the single-vector
and the many-right-hand-side paths.  The product path issues no memset, no
allocation and no synchronisation, so it can be captured; the many-RHS
workspaces are allocated by the first (eager) call."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import h2_inputs as I  # noqa: E402
from paper_2203_05665_amd import h2  # noqa: E402


@pytest.mark.parametrize("storage,nrhs", [("f64", 1), ("f32", 1), ("f32", 40)])
def test_graph_replays_match_eager(storage, nrhs):
    print("graph", storage, nrhs, flush=True)
    V, T = I.mesh_for("sphere", 5)
    n = T.shape[0]
    A = h2.H2Matrix(V, T, order=4, leaf=64, eta=0.5, storage=storage)
    try:
        xs = I.random_vector(n, 11, "normal", nrhs) if nrhs > 1 else I.random_vector(n, 11, "normal")
        x = torch.tensor(xs, dtype=torch.float64, device="cuda")
        if nrhs > 1:
            x = x.t().contiguous().t()            # n x R, Fortran order
        ref = A.matvec(x, torch.zeros_like(x))
        torch.cuda.synchronize()
        ref = ref.clone()
        y = torch.zeros_like(x)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            A.matvec(x, y)                          # warm-up on the side stream
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            A.matvec(x, y)
        other = torch.zeros_like(x)
        for rep in range(4):
            y.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(y, ref), "replay %d differs from the eager product" % rep
            other.zero_()
            A.matvec(x, other)                      # eager work between replays
            torch.cuda.synchronize()
            assert torch.equal(other, ref)
        del g
    finally:
        A.close()
