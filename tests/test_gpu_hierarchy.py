"""GPU parity of the multilevel components against the FP64 oracle through
the C ABI: interpolation P (aggregation, Sec. 1), Galerkin D_c = P^H D P,
restriction / prolongation, SAP on fine and coarse levels, one cycle
(Alg. 1 / Alg. 2) and full solves to 1e-10 (Tab. 1).

Setup results (test vectors) have no unique value, so the oracle is rebuilt
from the GPU's exported bases, or the GPU imports the oracle's vectors."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import multigrid as mg
from oracle.aggregation import Aggregation
from oracle.dirac import WilsonClover
from oracle.galerkin import galerkin
from oracle.krylov import norm
from oracle.lattice import shape
from oracle.sap import sap_sweep
from tests.gpu_util import (dev, empty, export_Dc, export_P, host, oracle_from_gpu, relerr, say,
                            to_params)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


def _p(levels, agg, ntv, n_inv=1, nu=2, **kw):
    p = dict(W.DEFAULT_PARAMS)
    p.update(levels=levels, agg=agg, ntv=ntv, n_inv=n_inv, nu=nu, **kw)
    return p


class Setup:
    def __init__(self, dd, dims, p, eps=0.5, m0=-0.3, csw=1.0, seed=1234, prec=None, half=False):
        say(f"hierarchy dims={dims} levels={p['levels']} ntv={p['ntv']}")
        self.dims, self.p = dims, p
        self.U = W.links(dims, eps, seed)
        self.op = WilsonClover(self.U, m0, csw)
        self.ctx = dd.create(dims, m0, csw, dev(self.U))
        self.tv = W.test_vectors(dims, 12, p["ntv"][0], seed + 1)
        self.H = dd.build_hierarchy(self.ctx, to_params(dd, p, prec, half=half), dev(self.tv))
        torch.cuda.synchronize()


@pytest.fixture(scope="module")
def two(dd):
    return Setup(dd, (8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [4]))


@pytest.fixture(scope="module")
def three(dd):
    return Setup(dd, (16, 16, 16, 16), _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 4]), m0=-0.25, seed=99)


def test_interpolation_orthonormal(dd, two):
    Pc = export_P(dd, two.H, 0, 4)
    agg = Aggregation(two.dims, (4, 4, 4, 4), Pc)      # re-orthonormalise in the oracle
    assert np.max(np.abs(agg.columns() - Pc)) < 1e-12


def test_import_test_vectors_matches_oracle_P_and_Dc(dd, two):
    rng = np.random.Generator(np.random.PCG64(5))
    tv = rng.standard_normal((4,) + shape(two.dims) + (12, 2)) @ np.array([1, 1j])
    dd.import_test_vectors(two.H, 0, dev(tv))
    agg = Aggregation(two.dims, (4, 4, 4, 4), tv)
    got = export_P(dd, two.H, 0, 4)
    e = np.max(np.abs(got - agg.columns()))
    say(f"  P max abs diff {e:.2e}")
    assert e < 1e-12
    Dc = galerkin(two.op, agg)
    G = export_Dc(dd, two.H, 1)
    ref = np.concatenate([Dc.S[..., None, :, :], np.moveaxis(Dc.F, 0, -3), np.moveaxis(Dc.B, 0, -3)],
                         axis=-3)
    e = relerr(G, ref)
    say(f"  D_c relerr {e:.2e}")
    assert e < 1e-12


def test_restrict_prolong(dd, two):
    agg = Aggregation(two.dims, (4, 4, 4, 4), export_P(dd, two.H, 0, 4))
    v = W.gaussian_spinor(two.dims, 11)
    c = W.gaussian_field(agg.cdims, 8, 12)
    for prec, tol in ((dd.F64, 1e-13), (dd.F32, 1e-6)):
        out = empty(c.shape)
        dd.restrict(two.H, 0, dev(v), out, prec=prec)
        assert relerr(host(out), agg.restrict(v)) < tol
        f = dev(v)
        dd.prolong(two.H, 0, dev(c), f, prec=prec)
        assert relerr(host(f), v + agg.prolong(c)) < tol


def test_coarse_apply_and_sap(dd, two):
    OH = oracle_from_gpu(dd, two.H, two.op, two.p)
    Dc = OH.ops[1]
    v = W.gaussian_field(Dc.dims, Dc.d, 21)
    for prec, tol in ((dd.F64, 1e-13), (dd.F32, 1e-5)):
        out = empty(v.shape)
        dd.apply_Dc(two.H, 1, dev(v), out, prec=prec)
        e = relerr(host(out), Dc.apply(v))
        say(f"  apply_Dc prec={prec} relerr={e:.2e}")
        assert e < tol


def test_fine_sap_parity(dd, two):
    b = W.gaussian_spinor(two.dims, 31)
    z0 = W.gaussian_spinor(two.dims, 32)
    ref = z0
    for _ in range(2):
        ref = sap_sweep(two.op, b, ref, (2, 2, 2, 2), 3)
    for prec, tol in ((dd.F64, 1e-12), (dd.F32, 1e-5)):
        z = dev(z0)
        dd.sap_smooth(two.H, 0, dev(b), z, 2, prec=prec)
        e = relerr(host(z), ref)
        say(f"  fine SAP prec={prec} relerr={e:.2e}")
        assert e < tol


def test_coarse_sap_parity(dd, three):
    OH = oracle_from_gpu(dd, three.H, three.op, three.p)
    Dc = OH.ops[1]
    b = W.gaussian_field(Dc.dims, Dc.d, 41)
    z0 = W.gaussian_field(Dc.dims, Dc.d, 42)
    ref = sap_sweep(Dc, b, z0, (2, 2, 2, 2), 3)
    for prec, tol in ((dd.F64, 1e-12), (dd.F32, 1e-5)):
        z = dev(z0)
        dd.sap_smooth(three.H, 1, dev(b), z, 1, prec=prec)
        e = relerr(host(z), ref)
        say(f"  coarse SAP prec={prec} relerr={e:.2e}")
        assert e < tol


def test_second_level_galerkin(dd, three):
    OH = oracle_from_gpu(dd, three.H, three.op, three.p)
    D2 = OH.ops[2]
    G = export_Dc(dd, three.H, 2)
    ref = np.concatenate([D2.S[..., None, :, :], np.moveaxis(D2.F, 0, -3), np.moveaxis(D2.B, 0, -3)],
                         axis=-3)
    e = relerr(G, ref)
    say(f"  level-2 D_c relerr {e:.2e}")
    assert e < 1e-12


@pytest.mark.parametrize("which", ["two", "three"])
def test_one_cycle_parity(dd, which, request):
    S = request.getfixturevalue(which)
    OH = oracle_from_gpu(dd, S.H, S.op, S.p)
    b = W.gaussian_spinor(S.dims, 51)
    ref = OH.cycle(0, b)
    z = empty(b.shape)
    dd.precondition(S.H, dev(b), z)
    e = relerr(host(z), ref)
    say(f"  cycle {which} relerr {e:.2e}")
    assert e < 1e-9


@pytest.mark.parametrize("which", ["two", "three"])
@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_solve_known_solution(dd, which, prec, request):
    S = request.getfixturevalue(which)
    P = getattr(dd, prec)
    H = S.H if P == dd.F64 else dd.build_hierarchy(S.ctx, to_params(dd, S.p, P), dev(S.tv))
    zstar = W.gaussian_spinor(S.dims, 61)
    b = S.op.apply(zstar)
    z = empty(b.shape)
    rc, st = dd.solve(H, dev(b), z)
    zz = host(z)
    res = norm(b - S.op.apply(zz)) / norm(b)
    err = norm(zz - zstar) / norm(zstar)
    say(f"  solve {which} {prec}: rc={rc} {st[0]} oracle relres={res:.2e} err={err:.2e}")
    assert rc == dd.OK
    assert res <= 1e-10 and st[0]["true_relres"] <= 1e-10
    assert err < 1e-8
