"""gabp_residual_noalloc (the entry point for callers that cannot allocate) against
gabp_residual through the C ABI: same r and same norms, on two calls in a row, the second
on a smaller system, and again after a call on the larger one (the static array keeps the
last call's contents, which must not leak into the next)."""
import numpy as np
import pytest

from paper_1904_04093_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_04093_amd import gabp
    gabp.load()
    return gabp


def _case(n, seed, **kw):
    a, _ = W.precision_at_scale(n)
    r = W.rng(700, seed)
    b = torch.as_tensor(r.uniform(-1, 1, a.n)).cuda()
    x = torch.as_tensor(r.uniform(-1, 1, a.n)).cuda()
    return a, b, x


@pytest.mark.parametrize("colour", [False, True])
def test_noalloc_residual_equals_residual(B, colour):
    cases = [_case(300, 0), _case(37, 1), _case(300, 2)]     # large, smaller, large again
    solvers = [B.Solver.from_csr(a, colour=W.grid_colouring(int(round(np.sqrt(a.n))))
                                 if colour else None,
                                 schedule="redblack" if colour else "flood")
               for a, _, _ in cases]
    for (a, b, x), s in zip(cases, solvers):
        for tr in (False, True):
            r_ref, n_ref = s.residual(b, x, transposed=tr)
            r = torch.full((a.n,), np.nan, dtype=torch.float64, device="cuda")
            nrm = torch.full((3,), np.nan, dtype=torch.float64, device="cuda")
            s.residual_noalloc(b, x, r, nrm, transposed=tr)
            torch.cuda.synchronize()
            assert torch.equal(r, r_ref), (a.n, tr)
            assert np.array_equal(nrm.cpu().numpy(), np.array(n_ref)), (a.n, tr)
            # norms only, no residual vector
            nrm2 = torch.full((3,), np.nan, dtype=torch.float64, device="cuda")
            s.residual_noalloc(b, x, None, nrm2, transposed=tr)
            torch.cuda.synchronize()
            assert torch.equal(nrm2, nrm)


def test_noalloc_residual_in_a_captured_graph(B):
    """The call allocates nothing and never synchronises, so it can be captured; the
    replays after eager work between them give the eager result each time."""
    a, b, x = _case(200, 3)
    s = B.Solver.from_csr(a)
    r_ref, n_ref = s.residual(b, x)
    r = torch.zeros(a.n, dtype=torch.float64, device="cuda")
    nrm = torch.zeros(3, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        s.residual_noalloc(b, x, r, nrm)
    other, small = _case(37, 4), None
    s_small = B.Solver.from_csr(other[0])
    for rep in range(3):
        r.fill_(np.nan)
        nrm.fill_(np.nan)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r, r_ref), rep
        assert np.array_equal(nrm.cpu().numpy(), np.array(n_ref)), rep
        small = s_small.residual(other[1], other[2])      # eager work in between
        torch.cuda.synchronize()
    assert small is not None
