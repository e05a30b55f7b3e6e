"""FP16 fine-level spinors in the solve's preconditioner (half_spinors):
the SAP colour passes, the restriction and the prolongation on FP16 fields
with one FP32 scale per site, against the FP64 oracle; the preconditioner
against the FP32-spinor one; solves certified by the oracle's operator.

Tolerances: every stored spinor component carries an error of at most
u = 2^-11 times its site's largest component, on top of the FP16 operator
entries (relative error u each).  A restriction or prolongation (one
encoded input or output, FP16 P) is then within a few u: 4u ~ 2e-3, as for
FP16 operator storage alone; a SAP sweep (inputs encoded, z re-encoded
after each colour pass, a few dependent applications) within 1e-2.  The
results must also lie above the FP32 level (1e-5), which shows that the
FP16 spinors were the ones read."""
import numpy as np
import pytest

import workloads as W
from oracle.aggregation import Aggregation
from oracle.krylov import norm
from oracle.sap import sap_sweep
from tests.gpu_util import dev, empty, export_P, host, relerr, say, to_params
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


def _hs_params(dd, p, hs=True):
    P = to_params(dd, p, dd.F32, half=True)
    P.half_spinors = 1 if hs else 0
    return P


class HSetup(Setup):
    def __init__(self, dd, dims, p, **kw):
        super().__init__(dd, dims, p, prec=dd.F32, half=True, **kw)
        self.H = dd.build_hierarchy(self.ctx, _hs_params(dd, p), dev(self.tv))


@pytest.fixture(scope="module")
def two_s(dd):
    return HSetup(dd, (8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [4]))


@pytest.fixture(scope="module")
def three_s(dd):
    return HSetup(dd, (16, 16, 16, 16), _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 4]), m0=-0.25, seed=99)


def _in_band(e, tol):
    return FP32_LEVEL < e < tol


def test_f16s_sap_sweep(dd, three_s):
    b = W.gaussian_spinor(three_s.dims, 191, nrhs=3)
    z0 = W.gaussian_spinor(three_s.dims, 192, nrhs=3)
    z = dev(z0)
    dd.sap_smooth(three_s.H, 0, dev(b), z, 1, nrhs=3, prec=dd.F16S)
    zz = host(z)
    for r in range(3):
        e = relerr(zz[r], sap_sweep(three_s.op, b[r], z0[r], (2, 2, 2, 2), 3))
        say(f"  FP16-spinor SAP sweep, field {r}: relerr {e:.2e}")
        assert _in_band(e, SMOOTH_TOL)
    # two sweeps from z = 0 (the smoother as the cycle runs it)
    z = empty(b.shape)
    z.zero_()
    dd.sap_smooth(three_s.H, 0, dev(b), z, 2, nrhs=3, prec=dd.F16S)
    ref = sap_sweep(three_s.op, b[1], sap_sweep(three_s.op, b[1], np.zeros_like(b[1]), (2, 2, 2, 2), 3),
                    (2, 2, 2, 2), 3)
    e = relerr(host(z)[1], ref)
    say(f"  two sweeps from zero: relerr {e:.2e}")
    assert _in_band(e, SMOOTH_TOL)


@pytest.mark.parametrize("nrhs", [2, 12])
def test_f16s_restrict_prolong(dd, two_s, nrhs):
    """(12 fields: the matrix-core kernels)"""
    agg = Aggregation(two_s.dims, (4, 4, 4, 4), export_P(dd, two_s.H, 0, 4))
    v = W.gaussian_spinor(two_s.dims, 172, nrhs=nrhs)
    c = W.gaussian_field(agg.cdims, 8, 173, nrhs=nrhs)
    out = empty(c.shape)
    dd.restrict(two_s.H, 0, dev(v), out, nrhs=nrhs, prec=dd.F16S)
    for r in range(nrhs):
        e = relerr(host(out)[r], agg.restrict(v[r]))
        say(f"  FP16-spinor restrict relerr {e:.2e}")
        assert _in_band(e, APPLY_TOL)
    # prolongation adds the decoded FP16 field P c to the canonical one
    f0 = W.gaussian_spinor(two_s.dims, 174, nrhs=nrhs)
    f = dev(f0)
    dd.prolong(two_s.H, 0, dev(c), f, nrhs=nrhs, prec=dd.F16S)
    for r in range(nrhs):
        pc = agg.prolong(c[r])
        e = norm(host(f)[r] - f0[r] - pc) / norm(pc)
        say(f"  FP16-spinor prolong relerr {e:.2e}")
        assert _in_band(e, APPLY_TOL)


def test_f16s_preconditioner_close_to_fp32_spinors(dd, three_s):
    """The same hierarchy data (FP16 operators) with FP32 spinors: the two
    preconditioners differ by the spinor rounding only."""
    H32 = dd.build_hierarchy(three_s.ctx, _hs_params(dd, three_s.p, hs=False), dev(three_s.tv))
    b = W.gaussian_spinor(three_s.dims, 181, nrhs=2)
    z16, z32 = empty(b.shape), empty(b.shape)
    dd.precondition(three_s.H, dev(b), z16, nrhs=2)
    dd.precondition(H32, dev(b), z32, nrhs=2)
    for r in range(2):
        e = relerr(host(z16)[r], host(z32)[r])
        say(f"  preconditioner FP16 vs FP32 spinors: relerr {e:.2e}")
        assert FP32_LEVEL < e < 2e-2


@pytest.mark.parametrize("which", ["two_s", "three_s"])
def test_f16s_solve_known_solution(dd, which, request):
    S = request.getfixturevalue(which)
    zstar = W.gaussian_spinor(S.dims, 161, nrhs=3)
    b = np.stack([S.op.apply(x) for x in zstar])
    z = empty(b.shape)
    rc, st = dd.solve(S.H, dev(b), z, nrhs=3)
    zz = host(z)
    H32 = dd.build_hierarchy(S.ctx, _hs_params(dd, S.p, hs=False), dev(S.tv))
    z32 = empty(b.shape)
    rc32, st32 = dd.solve(H32, dev(b), z32, nrhs=3)
    its, its32 = [s["outer_iters"] for s in st], [s["outer_iters"] for s in st32]
    say(f"  {which}: outer iterations FP16 spinors {its}, FP32 spinors {its32}")
    assert rc == dd.OK and rc32 == dd.OK
    for r in range(3):
        res = norm(b[r] - S.op.apply(zz[r])) / norm(b[r])
        assert res <= 1e-10 * 1.01 and st[r]["true_relres"] <= 1e-10
        assert relerr(zz[r], zstar[r]) < 1e-8
        assert its[r] <= its32[r] + 2


def test_f16s_validation(dd, two_s):
    P = _hs_params(dd, two_s.p)
    P.mu = 1
    with pytest.raises(dd.DDAMGError) as e:
        dd.build_hierarchy(two_s.ctx, P, dev(two_s.tv))
    assert e.value.status == dd.EINVAL
    P = _hs_params(dd, two_s.p)
    P.half_storage = 0
    with pytest.raises(dd.DDAMGError) as e:
        dd.build_hierarchy(two_s.ctx, P, dev(two_s.tv))
    assert e.value.status == dd.EINVAL
    v = W.gaussian_spinor(two_s.dims, 175)
    H32 = dd.build_hierarchy(two_s.ctx, _hs_params(dd, two_s.p, hs=False), dev(two_s.tv))
    with pytest.raises(dd.DDAMGError) as e:
        dd.sap_smooth(H32, 0, dev(v), empty(v.shape), 1, prec=dd.F16S)
    assert e.value.status == dd.EINVAL and "half_spinors" in str(e.value)
    c = W.gaussian_field((2, 2, 2, 2), 8, 178)
    with pytest.raises(dd.DDAMGError) as e:
        dd.prolong(two_s.H, 0, dev(c), dev(v), prec=dd.F16S, layout=dd.NATIVE)
    assert e.value.status == dd.EINVAL and "canonical" in str(e.value)
    with pytest.raises(dd.DDAMGError) as e:
        dd.apply_Dc(two_s.H, 0, dev(v), empty(v.shape), prec=dd.F16S)
    assert e.value.status == dd.EINVAL


def test_f16s_native_form(dd, two_s):
    """The native FP16 form (entries, then site scales, in one buffer): a
    round trip through it is the FP16 rounding of the field, and SAP and
    restriction on it give the canonical-layout calls' results exactly."""
    import torch
    n0, V = 12 * 8 ** 4, 8 ** 4
    b = W.gaussian_spinor(two_s.dims, 176, nrhs=2)
    z0 = W.gaussian_spinor(two_s.dims, 177, nrhs=2)
    nb = torch.empty(2 * (n0 + V), dtype=torch.float32, device="cuda")
    nz = torch.empty_like(nb)
    dd.to_native(two_s.ctx, None, 0, dev(b), nb, nrhs=2, prec=dd.F16S)
    dd.to_native(two_s.ctx, None, 0, dev(z0), nz, nrhs=2, prec=dd.F16S)
    back = empty(b.shape)
    dd.from_native(two_s.ctx, None, 0, nb, back, nrhs=2, prec=dd.F16S)
    e = relerr(host(back), b)
    say(f"  FP16 form round trip relerr {e:.2e}")
    assert 1e-6 < e < U16
    dd.sap_smooth(two_s.H, 0, nb, nz, 1, nrhs=2, prec=dd.F16S, layout=dd.NATIVE)
    zn = empty(b.shape)
    dd.from_native(two_s.ctx, None, 0, nz, zn, nrhs=2, prec=dd.F16S)
    zc = dev(z0)
    dd.sap_smooth(two_s.H, 0, dev(b), zc, 1, nrhs=2, prec=dd.F16S)
    assert np.array_equal(host(zn), host(zc))
    cc = empty((2, 2, 2, 2, 2, 8))
    c32 = torch.empty(2 * 16 * 8, dtype=torch.complex64, device="cuda")
    dd.restrict(two_s.H, 0, nb, c32, nrhs=2, prec=dd.F16S, layout=dd.NATIVE)
    dd.restrict(two_s.H, 0, dev(b), cc, nrhs=2, prec=dd.F16S)
    assert np.array_equal(c32.cpu().numpy().astype(np.complex128), host(cc).reshape(-1))
