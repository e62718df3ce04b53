"""The Sec. 5 test problems as generated: second-order central differences of each PDE with
its manufactured solution must converge to that solution at rate h^2 (no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from paper_1904_04093_amd import workloads as W


def _err(name, n, **kw):
    a, b, exact = W.sec5_problem(name, n, **kw)
    m = sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.n)).tocsc()
    return float(np.abs(spl.spsolve(m, b) - exact).max())


@pytest.mark.parametrize("name,kw", [("stand_alone", {}), ("boundary_layers", dict(eps=0.02)),
                                     ("inner_layers", dict(eps=0.015)),
                                     ("stretched", dict(p=20, eta=0.5, eps=1e-6))])
def test_sec5_problems_converge_at_second_order(name, kw):
    e = [_err(name, n, **kw) for n in (63, 127, 255)]
    for coarse, fine in zip(e, e[1:]):
        assert 3.7 < coarse / fine < 4.3, e


def test_sec5_hierarchy_shapes():
    levels, b = W.sec5_hierarchy("inner_layers", 6, 1, eps=0.01)
    assert [a.n for a in levels] == [63 ** 2, 31 ** 2, 15 ** 2, 7 ** 2, 3 ** 2, 1]
    assert b.shape == (63 ** 2,)
