"""Edge cases of the solve entry point: an initial guess that already
solves the system (no iteration), a zero right-hand side (zero solution),
a non-finite right-hand side (DDAMG_ENONFINITE, the other systems of the
batch unaffected), a restart limit too small for the tolerance
(DDAMG_ENOCONV with a finite iterate), and parameter validation."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.krylov import norm
from tests.gpu_util import dev, empty, host, relerr, say, to_params
from tests.test_gpu_hierarchy import Setup, _p

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


@pytest.fixture(scope="module")
def two(dd):
    return Setup(dd, (8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [4]), prec=dd.F32)


def test_initial_guess_that_solves(dd, two):
    zstar = W.gaussian_spinor(two.dims, 1001)
    b = two.op.apply(zstar)
    z = dev(zstar)
    rc, st = dd.solve(two.H, dev(b), z)
    say(f"  exact initial guess: {st[0]}")
    assert rc == dd.OK and st[0]["outer_iters"] == 0
    assert relerr(host(z), zstar) < 1e-12


def test_zero_rhs_in_a_batch(dd, two):
    zstar = W.gaussian_spinor(two.dims, 1002, nrhs=3)
    b = np.stack([two.op.apply(x) for x in zstar])
    b[1] = 0
    z = dev(W.gaussian_spinor(two.dims, 1003, nrhs=3))   # a nonzero guess for the zero system
    rc, st = dd.solve(two.H, dev(b), z, nrhs=3)
    zz = host(z)
    say(f"  zero rhs in a batch: {[s['status'] for s in st]} its {[s['outer_iters'] for s in st]}")
    assert rc == dd.OK
    assert np.all(zz[1] == 0)
    for r in (0, 2):
        assert norm(b[r] - two.op.apply(zz[r])) / norm(b[r]) <= 1e-10


def test_nonfinite_rhs(dd, two):
    zstar = W.gaussian_spinor(two.dims, 1004, nrhs=2)
    b = np.stack([two.op.apply(x) for x in zstar])
    b[0, 0, 0, 0, 0, 0] = np.nan
    z = empty(b.shape)
    rc, st = dd.solve(two.H, dev(b), z, nrhs=2)
    say(f"  non-finite rhs: rc={rc} statuses {[s['status'] for s in st]}")
    assert rc == dd.ENONFINITE
    assert st[0]["status"] == dd.ENONFINITE and st[1]["status"] == dd.OK
    assert norm(b[1] - two.op.apply(host(z)[1])) / norm(b[1]) <= 1e-10


def test_restart_limit(dd, two):
    p = dict(two.p, tol=1e-14, max_restarts=1)
    H = dd.build_hierarchy(two.ctx, to_params(dd, p, dd.F32), dev(two.tv))
    b = W.gaussian_spinor(two.dims, 1005)
    z = empty(b.shape)
    rc, st = dd.solve(H, dev(b), z)
    say(f"  restart limit: rc={rc} {st[0]}")
    assert rc == dd.ENOCONV and st[0]["status"] == dd.ENOCONV and st[0]["restarts"] == 1
    zz = host(z)
    assert np.all(np.isfinite(zz))
    assert norm(b - two.op.apply(zz)) / norm(b) < 1e-3


@pytest.mark.parametrize("field,value", [("batch", 0), ("batch", 33), ("half_storage", 2), ("nkv", 40),
                                         ("levels", 5)])
def test_parameter_validation(dd, two, field, value):
    P = to_params(dd, two.p, dd.F32)
    setattr(P, field, value)
    with pytest.raises(dd.DDAMGError) as ei:
        dd.build_hierarchy(two.ctx, P, dev(two.tv))
    assert ei.value.status == dd.EINVAL


def test_stagnation_ends_the_solve(dd, two):
    """A tolerance below what FP64 reaches: once a restart cycle no longer
    reduces the recomputed residual, the solve stops with ENOCONV instead of
    running out its 100 restarts, and the iterate it returns is the
    converged one."""
    p = dict(two.p, tol=1e-18, max_restarts=100)
    H = dd.build_hierarchy(two.ctx, to_params(dd, p, dd.F32), dev(two.tv))
    b = W.gaussian_spinor(two.dims, 1006)
    z = empty(b.shape)
    rc, st = dd.solve(H, dev(b), z)
    say(f"  stagnation: rc={rc} {st[0]}")
    assert rc == dd.ENOCONV and st[0]["status"] == dd.ENOCONV
    assert st[0]["restarts"] < 20
    zz = host(z)
    assert norm(b - two.op.apply(zz)) / norm(b) < 1e-13
