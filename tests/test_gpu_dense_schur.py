"""The coarsest odd-even Schur system held as a dense matrix (coarse_dense = 1,
the default on small coarsest levels) against the oracle's odd-even coarsest
solve, through one cycle of a two-level hierarchy whose coarsest level has
the 16^3x32 workload's coarsest shape (2^3x4 sites, 40 components: a
640-unknown Schur system), and the solves with the dense and the sparse
Schur product side by side."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.dirac import WilsonClover
from oracle.krylov import norm
from oracle.sap import sap_sweep
from tests.gpu_util import dev, empty, host, oracle_from_gpu, relerr, say, to_params

pytestmark = pytest.mark.gpu

DIMS = (8, 8, 8, 16)


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


@pytest.fixture(scope="module")
def case(dd):
    p = dict(W.DEFAULT_PARAMS)
    p.update(levels=2, agg=[(4, 4, 4, 4)], ntv=[20], n_inv=1, nu=2)
    U = W.links(DIMS, 0.5, 4321)
    op = WilsonClover(U, -0.3, 1.0)
    ctx = dd.create(DIMS, -0.3, 1.0, dev(U))
    tv = W.test_vectors(DIMS, 12, 20, 4322)
    say(f"two-level dims={DIMS} ntv=20: coarsest 2^3x4 x 40")
    return dd, p, op, ctx, tv


def _hier(case, prec, dense):
    dd, p, op, ctx, tv = case
    P = to_params(dd, p, prec)
    P.coarse_dense = dense
    H = dd.build_hierarchy(ctx, P, dev(tv))
    torch.cuda.synchronize()
    return H


@pytest.mark.parametrize("dense", [1, 0])
def test_cycle_parity_dense_and_sparse(case, dense):
    dd, p, op, ctx, tv = case
    H = _hier(case, dd.F64, dense)
    assert dd.level_info(H, 1) == ((2, 2, 2, 4), 40)
    OH = oracle_from_gpu(dd, H, op, p)
    b = W.gaussian_spinor(DIMS, 71)
    ref = OH.cycle(0, b)
    z = empty(b.shape)
    dd.precondition(H, dev(b), z)
    e = relerr(host(z), ref)
    say(f"  coarse_dense={dense}: one cycle relerr {e:.2e}")
    assert e < 1e-9


def test_solves_dense_and_sparse(case):
    dd, p, op, ctx, tv = case
    zstar = W.gaussian_spinor(DIMS, 72, nrhs=3)
    b = np.stack([op.apply(zstar[r]) for r in range(3)])
    its = {}
    for dense in (1, 0):
        H = _hier(case, dd.F32, dense)
        z = empty(b.shape)
        rc, st = dd.solve(H, dev(b), z, nrhs=3)
        assert rc == dd.OK
        zz = host(z)
        for r in range(3):
            res = norm(b[r] - op.apply(zz[r])) / norm(b[r])
            assert res <= 1e-10 and st[r]["true_relres"] <= 1e-10
        # the path taken: the 640-unknown dense Schur matrix, or none
        assert all(s["coarsest_dense"] == (640 if dense else 0) for s in st)
        its[dense] = [s["outer_iters"] for s in st]
        say(f"  coarse_dense={dense}: outer iterations {its[dense]}, "
            f"coarsest {[s['coarsest_iters'] for s in st]}")
    assert all(abs(a - c) <= 1 for a, c in zip(its[1], its[0]))


def test_fp32_cycle_dense_against_sparse(case):
    """The FP32 dense Schur product (the matrix copy the FP32 and FP16
    preconditioners use) against the sparse FP32 product, one cycle on the
    same hierarchy data: equal up to FP32 rounding (1e-5)."""
    dd, p, op, ctx, tv = case
    b = W.gaussian_spinor(DIMS, 73, nrhs=2)
    zd, zs = empty(b.shape), empty(b.shape)
    dd.precondition(_hier(case, dd.F32, 1), dev(b), zd, nrhs=2)
    dd.precondition(_hier(case, dd.F32, 0), dev(b), zs, nrhs=2)
    for r in range(2):
        e = relerr(host(zd)[r], host(zs)[r])
        say(f"  FP32 cycle, dense against sparse Schur product: relerr {e:.2e}")
        assert e < 1e-5


def test_coarse_dense_validation(case):
    dd, p, op, ctx, tv = case
    P = to_params(dd, p, dd.F32)
    P.coarse_dense = 2
    with pytest.raises(dd.DDAMGError) as e:
        dd.build_hierarchy(ctx, P, dev(tv))
    assert e.value.status == dd.EINVAL


def test_components_n20(case):
    """Restriction, prolongation, D_c and the fine SAP of the same hierarchy
    (N = 20 on an 8^3x16 lattice) against the oracle, one by one."""
    dd, p, op, ctx, tv = case
    H = _hier(case, dd.F64, 1)
    OH = oracle_from_gpu(dd, H, op, p)
    agg = OH.aggs[0]
    v = W.gaussian_spinor(DIMS, 81)
    c = W.gaussian_field(agg.cdims, 40, 82)
    out = empty(c.shape)
    dd.restrict(H, 0, dev(v), out, prec=dd.F64)
    er = relerr(host(out), agg.restrict(v))
    f = dev(v)
    dd.prolong(H, 0, dev(c), f, prec=dd.F64)
    ep = relerr(host(f), v + agg.prolong(c))
    o2 = empty(c.shape)
    dd.apply_Dc(H, 1, dev(c), o2, prec=dd.F64)
    ed = relerr(host(o2), OH.ops[1].apply(c))
    b = W.gaussian_spinor(DIMS, 83)
    ref = sap_sweep(op, b, np.zeros_like(b), (2, 2, 2, 2), 3)
    z = empty(b.shape)
    dd.sap_smooth(H, 0, dev(b), z, 1, prec=dd.F64)
    es = relerr(host(z), ref)
    say(f"  N=20: restrict {er:.2e} prolong {ep:.2e} D_c {ed:.2e} fine SAP {es:.2e}")
    assert max(er, ep, ed) < 1e-12 and es < 1e-12
