"""FP64 CGNR on the GPU against the oracle's CGNR (Sec. 4): same iteration
count up to rounding, solutions agreeing to the tolerance's scale, the
residual bound met with the oracle's operator; a batch equals its systems
solved alone; the iteration limit and a zero right-hand side."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.dirac import WilsonClover
from oracle.krylov import cgnr, norm
from tests.gpu_util import dev, empty, host, relerr, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


@pytest.fixture(scope="module")
def lat(dd):
    dims = (8, 8, 8, 8)
    U = W.links(dims, 0.5, 811)
    op = WilsonClover(U, -0.2, 1.0)
    ctx = dd.create(dims, -0.2, 1.0, dev(U))
    b = W.gaussian_spinor(dims, 812, nrhs=3)
    return dims, op, ctx, b


def test_cgnr_matches_oracle(dd, lat):
    dims, op, ctx, b = lat
    st = {}
    xo = cgnr(op.apply, op.apply_dagger, b[0], 1e-10, 5000, stats=st)
    z = empty(b[:1].shape)
    rc, sg = dd.cgnr(ctx, dev(b[:1]), z, tol=1e-10)
    zz = host(z)[0]
    say(f"  CGNR iterations: oracle {st['iters']}, GPU {sg[0]['outer_iters']}, rel. diff {relerr(zz, xo):.1e}")
    assert rc == dd.OK
    assert abs(sg[0]["outer_iters"] - st["iters"]) <= 2
    assert relerr(zz, xo) <= 1e-8
    res = norm(b[0] - op.apply(zz)) / norm(b[0])
    assert res <= 1e-10 and abs(res - sg[0]["true_relres"]) <= 1e-12


def test_cgnr_batch_equals_alone(dd, lat):
    dims, op, ctx, b = lat
    z3 = empty(b.shape)
    rc, s3 = dd.cgnr(ctx, dev(b), z3, nrhs=3, tol=1e-10)
    assert rc == dd.OK
    zz3 = host(z3)
    for r in range(3):
        z1 = empty(b[:1].shape)
        rc1, s1 = dd.cgnr(ctx, dev(b[r:r + 1]), z1, tol=1e-10)
        assert s1[0]["outer_iters"] == s3[r]["outer_iters"]
        assert relerr(zz3[r], host(z1)[0]) <= 1e-13
        assert norm(b[r] - op.apply(zz3[r])) / norm(b[r]) <= 1e-10


def test_cgnr_limits(dd, lat):
    dims, op, ctx, b = lat
    z = empty(b[:1].shape)
    rc, st = dd.cgnr(ctx, dev(b[:1]), z, tol=1e-10, max_iter=5)
    assert rc == dd.ENOCONV and st[0]["outer_iters"] == 5 and st[0]["status"] == dd.ENOCONV
    zb = np.zeros_like(b[:2])
    zb[1] = b[1]
    z2 = empty(zb.shape)
    rc, st = dd.cgnr(ctx, dev(zb), z2, nrhs=2, tol=1e-10)
    assert rc == dd.OK and st[0]["outer_iters"] == 0
    assert np.all(host(z2)[0] == 0)
    with pytest.raises(dd.DDAMGError):
        dd.cgnr(ctx, dev(b[:1]), z, tol=0.0)
