"""Batched solver: several systems advance through the outer FGMRES, the
K-cycle, the coarsest odd-even GMRES and the setup together, each with its
own Krylov scalars and stopping tests.

Checks: the batched preconditioner equals the oracle's cycle system by
system (the oracle runs each system alone); a batched solve reaches the
certified tolerance for every right-hand side with the same iteration
counts as one-at-a-time solves and the same solutions up to the solve
tolerance; the 12 spin-colour point sources solved in one batch with the
FP32 (and FP16-storage) preconditioner; a setup that smooths its test
vectors in batches builds the same interpolation as one that takes them one
at a time."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.krylov import norm
from tests.gpu_util import dev, empty, export_P, host, oracle_from_gpu, relerr, say, to_params
from tests.test_gpu_hierarchy import Setup, _p

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


@pytest.fixture(scope="module")
def three(dd):
    return Setup(dd, (16, 16, 16, 16), _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 4]), m0=-0.25, seed=99)


def _params(dd, S, prec, batch, half=False):
    P = to_params(dd, S.p, prec, half=half)
    P.batch = batch
    return P


def test_batched_precondition_matches_oracle_cycle(dd, three):
    OH = oracle_from_gpu(dd, three.H, three.op, three.p)
    nrhs = 4
    b = W.gaussian_spinor(three.dims, 701, nrhs=nrhs)
    z = empty(b.shape)
    dd.precondition(three.H, dev(b), z, nrhs=nrhs)
    got = host(z)
    for r in range(nrhs):
        e = relerr(got[r], OH.cycle(0, b[r]))
        say(f"  batched cycle system {r}: relerr {e:.2e}")
        assert e < 1e-9


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_batched_solve_equals_single_solves(dd, three, prec):
    P = getattr(dd, prec)
    nrhs = 5
    zstar = W.gaussian_spinor(three.dims, 801, nrhs=nrhs)
    b = np.stack([three.op.apply(x) for x in zstar])
    res = {}
    for batch in (1, nrhs):
        H = dd.build_hierarchy(three.ctx, _params(dd, three, P, batch), dev(three.tv))
        z = empty(b.shape)
        rc, st = dd.solve(H, dev(b), z, nrhs=nrhs)
        assert rc == dd.OK
        res[batch] = (host(z), st)
        say(f"  {prec} batch={batch}: its {[s['outer_iters'] for s in st]} "
            f"kcycle {[s['kcycle_iters'] for s in st]} coarsest {[s['coarsest_iters'] for s in st]}")
    (z1, st1), (zb, stb) = res[1], res[nrhs]
    for r in range(nrhs):
        rr = norm(b[r] - three.op.apply(zb[r])) / norm(b[r])
        assert rr <= 1e-10 and stb[r]["true_relres"] <= 1e-10
        assert abs(stb[r]["outer_iters"] - st1[r]["outer_iters"]) <= 1
        assert relerr(zb[r], z1[r]) < 1e-8
        assert relerr(zb[r], zstar[r]) < 1e-8


@pytest.mark.parametrize("half", [False, True])
def test_point_sources_one_batch(dd, half):
    dims = (16, 16, 16, 16)
    p = _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [8, 8], n_inv=2, nu=3)
    S = Setup(dd, dims, p, eps=0.5, m0=-0.42, csw=1.0, seed=4711, prec=dd.F32, half=half)
    P = _params(dd, S, dd.F32, 12, half=half)
    H = dd.build_hierarchy(S.ctx, P, dev(S.tv))
    b = W.point_sources(dims)
    z = empty(b.shape)
    rc, st = dd.solve(H, dev(b), z, nrhs=12)
    zz = host(z)
    say(f"  point sources half={half}: its {[s['outer_iters'] for s in st]}")
    assert rc == dd.OK
    for r in range(12):
        rr = norm(b[r] - S.op.apply(zz[r])) / norm(b[r])
        assert rr <= 1e-10, (r, rr)


def test_batched_setup_matches_unbatched(dd, three):
    Ps = {}
    for batch in (1, 4):
        H = dd.build_hierarchy(three.ctx, _params(dd, three, dd.F64, batch), dev(three.tv))
        Ps[batch] = export_P(dd, H, 0, 4)
    e = relerr(Ps[4], Ps[1])
    say(f"  setup batch 4 vs 1: P relerr {e:.2e}")
    assert e < 1e-8
