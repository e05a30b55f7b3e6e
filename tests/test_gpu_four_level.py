"""Four levels with a per-level SAP block shape (the coarse level whose 2^4
blocks would come in odd counts takes smaller blocks; here 1^4 on a 2^4
level) and a non-bipartite coarsest lattice (1^4, full GMRES): one K-cycle
against the oracle (FP64, 1e-9 as for three levels) and certified solves."""
import numpy as np
import pytest

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


def _four():
    return _p(4, [(4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2)], [4, 4, 4],
              sap_blocks=[(2, 2, 2, 2), (2, 2, 2, 2), (1, 1, 1, 1)])


@pytest.fixture(scope="module")
def four(dd):
    return Setup(dd, (16, 16, 16, 16), _four(), m0=-0.25, seed=321)


def test_four_level_shapes(dd, four):
    assert dd.level_info(four.H, 3) == ((1, 1, 1, 1), 8)
    assert dd.level_info(four.H, 2) == ((2, 2, 2, 2), 8)


def test_four_level_cycle_parity(dd, four):
    OH = oracle_from_gpu(dd, four.H, four.op, four.p)
    b = W.gaussian_spinor(four.dims, 901)
    z = empty(b.shape)
    dd.precondition(four.H, dev(b), z)
    e = relerr(host(z), OH.cycle(0, b))
    say(f"  four-level cycle relerr {e:.2e}")
    assert e < 1e-9


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_four_level_solve(dd, four, prec):
    P = getattr(dd, prec)
    H = four.H if P == dd.F64 else dd.build_hierarchy(four.ctx, to_params(dd, four.p, P), dev(four.tv))
    zstar = W.gaussian_spinor(four.dims, 902)
    b = four.op.apply(zstar)
    z = empty(b.shape)
    rc, st = dd.solve(H, dev(b), z)
    zz = host(z)
    res = norm(b - four.op.apply(zz)) / norm(b)
    say(f"  four-level solve {prec}: rc={rc} {st[0]} oracle relres={res:.2e}")
    assert rc == dd.OK and res <= 1e-10
    assert relerr(zz, zstar) < 1e-8


def test_odd_block_count_rejected(dd, four):
    """2^4 blocks on the 2^4 level give one block per direction: rejected"""
    p = _p(4, [(4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2)], [4, 4, 4])
    with pytest.raises(dd.DDAMGError) as ei:
        dd.build_hierarchy(four.ctx, to_params(dd, p), dev(four.tv))
    assert ei.value.status == dd.EINVAL
