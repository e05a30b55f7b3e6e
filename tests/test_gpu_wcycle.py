"""The W-cycle (two level-(l+1) cycles on an intermediate level, the second
on the residual of the first): one application against the oracle's
W-cycle on the GPU's interpolation bases, solves to 1e-10, and its graph
capture."""
import pytest
import torch

import workloads as W
from oracle.krylov import norm
from tests.gpu_util import dev, empty, host, oracle_from_gpu, relerr, say, to_params
from tests.test_gpu_hierarchy import Setup, _p

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


@pytest.fixture(scope="module")
def three_w(dd):
    dims = (16, 16, 16, 16)
    p = _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 4])
    S = Setup(dd, dims, p, m0=-0.25, seed=733)
    S.Hw = dd.build_hierarchy(S.ctx, to_params(dd, p, dd.F64, cycle="W"), dev(S.tv))
    torch.cuda.synchronize()
    return S


def test_w_cycle_parity(dd, three_w):
    S = three_w
    OH = oracle_from_gpu(dd, S.Hw, S.op, S.p, cycle="W")
    b = W.gaussian_spinor(S.dims, 734)
    ref = OH.cycle(0, b)
    z = empty(b.shape)
    dd.precondition(S.Hw, dev(b), z)
    e = relerr(host(z), ref)
    say(f"  W-cycle relerr {e:.2e}")
    assert e < 1e-9


@pytest.mark.parametrize("graph", [0, 1])
def test_w_cycle_solves(dd, three_w, graph):
    S = three_w
    P = to_params(dd, S.p, dd.F32, cycle="W")
    P.graph = graph
    H = dd.build_hierarchy(S.ctx, P, dev(S.tv))
    b = W.gaussian_spinor(S.dims, 735, nrhs=2)
    z = empty(b.shape)
    rc, st = dd.solve(H, dev(b), z, nrhs=2)
    say(f"  W-cycle graph={graph}: its {[x['outer_iters'] for x in st]}")
    assert rc == dd.OK
    zz = host(z)
    for r in range(2):
        assert norm(b[r] - S.op.apply(zz[r])) / norm(b[r]) <= 1e-10
