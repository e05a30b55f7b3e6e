"""FP16 storage of the preconditioner's operator data (links, clover, P_l,
coarse D_l) with FP32 arithmetic: every level operation of such a hierarchy
against the FP64 oracle, and full solves that still reach the outer FP64
tolerance of Tab. 1.

Tolerances: binary16 has unit roundoff u = 2^-11 ~ 4.9e-4, and each stored
operator entry carries a relative error of at most u; a sum of products
whose terms are not strongly cancelling then has a relative error of a few
u.  Apply, restriction and prolongation are checked to 4u ~ 2e-3, smoothers
(a few dependent applications) to 1e-2.  The same results also have to lie
above the FP32 level (1e-5), which shows that the FP16 copies were read."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.aggregation import Aggregation
from oracle.krylov import norm
from oracle.sap import sap_sweep
from tests.gpu_util import dev, empty, export_P, host, oracle_from_gpu, relerr, say, to_params
from tests.test_gpu_hierarchy import Setup, _p

pytestmark = pytest.mark.gpu

U16 = 2.0 ** -11
APPLY_TOL = 4 * U16
SMOOTH_TOL = 1e-2
FP32_LEVEL = 1e-5


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


@pytest.fixture(scope="module")
def two_h(dd):
    return Setup(dd, (8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [4]), prec=dd.F32, half=True)


@pytest.fixture(scope="module")
def three_h(dd):
    return Setup(dd, (16, 16, 16, 16), _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 4]), m0=-0.25, seed=99,
                 prec=dd.F32, half=True)


def _in_band(e, tol):
    return FP32_LEVEL < e < tol


def test_half_needs_fp32_preconditioner(dd, two_h):
    P = to_params(dd, two_h.p, dd.F64, half=True)
    with pytest.raises(dd.DDAMGError) as ei:
        dd.build_hierarchy(two_h.ctx, P, dev(two_h.tv))
    assert ei.value.status == dd.EINVAL


def test_half_fine_apply(dd, two_h):
    v = W.gaussian_spinor(two_h.dims, 71)
    out = empty(v.shape)
    dd.apply_Dc(two_h.H, 0, dev(v), out, prec=dd.F32)
    e = relerr(host(out), two_h.op.apply(v))
    say(f"  FP16-stored D relerr {e:.2e}")
    assert _in_band(e, APPLY_TOL)


def test_half_restrict_prolong(dd, two_h):
    agg = Aggregation(two_h.dims, (4, 4, 4, 4), export_P(dd, two_h.H, 0, 4))
    v = W.gaussian_spinor(two_h.dims, 72)
    c = W.gaussian_field(agg.cdims, 8, 73)
    out = empty(c.shape)
    dd.restrict(two_h.H, 0, dev(v), out, prec=dd.F32)
    e = relerr(host(out), agg.restrict(v))
    say(f"  FP16-stored restrict relerr {e:.2e}")
    assert _in_band(e, APPLY_TOL)
    f = empty(v.shape)
    f.zero_()
    dd.prolong(two_h.H, 0, dev(c), f, prec=dd.F32)
    e = relerr(host(f), agg.prolong(c))
    say(f"  FP16-stored prolong relerr {e:.2e}")
    assert _in_band(e, APPLY_TOL)


def test_half_coarse_apply_and_restrict(dd, three_h):
    OH = oracle_from_gpu(dd, three_h.H, three_h.op, three_h.p)
    for lvl in (1, 2):
        Dc = OH.ops[lvl]
        v = W.gaussian_field(Dc.dims, Dc.d, 80 + lvl)
        out = empty(v.shape)
        dd.apply_Dc(three_h.H, lvl, dev(v), out, prec=dd.F32)
        e = relerr(host(out), Dc.apply(v))
        say(f"  FP16-stored D_{lvl} relerr {e:.2e}")
        assert _in_band(e, APPLY_TOL)
    agg = OH.aggs[1]
    v = W.gaussian_field(OH.ops[1].dims, OH.ops[1].d, 84)
    out = empty((*agg.cdims, OH.ops[2].d))
    dd.restrict(three_h.H, 1, dev(v), out, prec=dd.F32)
    e = relerr(host(out), agg.restrict(v))
    say(f"  FP16-stored coarse restrict relerr {e:.2e}")
    assert _in_band(e, APPLY_TOL)


def test_half_smoothers(dd, three_h):
    OH = oracle_from_gpu(dd, three_h.H, three_h.op, three_h.p)
    b = W.gaussian_spinor(three_h.dims, 91)
    z0 = W.gaussian_spinor(three_h.dims, 92)
    z = dev(z0)
    dd.sap_smooth(three_h.H, 0, dev(b), z, 1, prec=dd.F32)
    e = relerr(host(z), sap_sweep(three_h.op, b, z0, (2, 2, 2, 2), 3))
    say(f"  FP16-stored fine SAP relerr {e:.2e}")
    assert _in_band(e, SMOOTH_TOL)
    Dc = OH.ops[1]
    b = W.gaussian_field(Dc.dims, Dc.d, 93)
    z0 = W.gaussian_field(Dc.dims, Dc.d, 94)
    z = dev(z0)
    dd.sap_smooth(three_h.H, 1, dev(b), z, 1, prec=dd.F32)
    e = relerr(host(z), sap_sweep(Dc, b, z0, (2, 2, 2, 2), 3))
    say(f"  FP16-stored coarse SAP relerr {e:.2e}")
    assert _in_band(e, SMOOTH_TOL)


@pytest.mark.parametrize("which", ["two_h", "three_h"])
def test_half_solve_known_solution(dd, which, request):
    S = request.getfixturevalue(which)
    zstar = W.gaussian_spinor(S.dims, 61)
    b = S.op.apply(zstar)
    z = empty(b.shape)
    rc, st = dd.solve(S.H, dev(b), z)
    zz = host(z)
    res = norm(b - S.op.apply(zz)) / norm(b)
    err = norm(zz - zstar) / norm(zstar)
    say(f"  FP16-storage solve {which}: rc={rc} {st[0]} oracle relres={res:.2e} err={err:.2e}")
    assert rc == dd.OK
    assert res <= 1e-10 and st[0]["true_relres"] <= 1e-10
    assert err < 1e-8


@pytest.mark.parametrize("half", [False, True])
def test_fp16_directions_solve(dd, three_h, half):
    """outer directions stored in FP16 with a per-site scale: the solve still
    reaches the certified tolerance (D is applied to the stored values)"""
    P = to_params(dd, three_h.p, dd.F32, half=half, half_dirs=True)
    H = dd.build_hierarchy(three_h.ctx, P, dev(three_h.tv))
    zstar = W.gaussian_spinor(three_h.dims, 62, nrhs=3)
    b = np.stack([three_h.op.apply(x) for x in zstar])
    z = empty(b.shape)
    rc, st = dd.solve(H, dev(b), z, nrhs=3)
    zz = host(z)
    say(f"  FP16 directions (half storage {half}): its {[s['outer_iters'] for s in st]}")
    assert rc == dd.OK
    for r in range(3):
        assert norm(b[r] - three_h.op.apply(zz[r])) / norm(b[r]) <= 1e-10
        assert relerr(zz[r], zstar[r]) < 1e-8

