"""The C-ABI additions: the FP16-storage precision at the call level, the
solve statistics (setup time, per-level times, algorithmic bytes and
flops, the error against a reference solution, the dense coarsest Schur
order), and the setup's check for test vectors that cannot be
orthonormalised accurately."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.dirac import WilsonClover
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
def three(dd):
    return Setup(dd, (16, 16, 16, 16), _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 4]), m0=-0.25, seed=777,
                 prec=dd.F32, half=True)


def test_apply_D_f16_storage(dd, three):
    """DDAMG_F16: binary16 links and clover, FP32 arithmetic: within the
    FP16-storage band of the oracle (entries rounded at 2^-11 relative)."""
    psi = W.gaussian_spinor(three.dims, 7701, nrhs=2)
    ref = np.stack([three.op.apply(x) for x in psi])
    out = empty(psi.shape)
    dd.apply_D(three.ctx, dev(psi), out, nrhs=2, prec=dd.F16)
    e = relerr(host(out), ref)
    say(f"  apply_D F16 relerr {e:.2e}")
    assert 1e-6 < e < 2e-3
    # level calls of a half-storage hierarchy accept F16 (and read the same copies as F32)
    dims1, d1 = dd.level_info(three.H, 1)
    v = W.gaussian_field(dims1, d1, 7702)
    o16, o32 = empty(v.shape), empty(v.shape)
    dd.apply_Dc(three.H, 1, dev(v), o16, prec=dd.F16)
    dd.apply_Dc(three.H, 1, dev(v), o32, prec=dd.F32)
    assert np.array_equal(host(o16), host(o32))


def test_f16_needs_half_storage(dd):
    S = Setup(dd, (8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [4]), prec=dd.F32)
    v = W.gaussian_field((2, 2, 2, 2), 8, 7703)
    with pytest.raises(dd.DDAMGError) as e:
        dd.apply_Dc(S.H, 1, dev(v), empty(v.shape), prec=dd.F16)
    assert e.value.status == dd.EINVAL


def test_solve_stats_fields(dd, three):
    zstar = W.gaussian_spinor(three.dims, 7704, nrhs=2)
    b = np.stack([three.op.apply(x) for x in zstar])
    for prof in (0, 1):
        P = to_params(dd, three.p, dd.F32, half=True)
        P.profile_levels = prof
        H = dd.build_hierarchy(three.ctx, P, dev(three.tv))
        z = empty(b.shape)
        rc, st = dd.solve_ex(H, dev(b), z, z_ref=dev(zstar), nrhs=2)
        zz = host(z)
        say(f"  profile_levels={prof}: {st[0]}")
        assert rc == dd.OK
        for r in range(2):
            err = norm(zz[r] - zstar[r]) / norm(zstar[r])
            assert abs(st[r]["err_vs_ref"] - err) <= 1e-6 * err + 1e-14
            assert st[r]["t_setup_s"] > 0 and st[r]["bytes"] > 0 and st[r]["flops"] > 0
            assert st[r]["coarsest_dense"] == 0 or st[r]["coarsest_dense"] % 8 == 0
            tl = st[r]["t_level_s"]
            if prof:
                assert all(t > 0 for t in tl[:3]) and tl[3] == 0
                assert sum(tl) <= st[r]["seconds"] * 1.05
            else:
                assert tl == [0, 0, 0, 0]
        # without a reference the error field is -1
        z.zero_()
        rc, st2 = dd.solve(H, dev(b), z, nrhs=2)
        assert st2[0]["err_vs_ref"] == -1


def test_nearly_dependent_test_vectors_rejected(dd, three):
    """Test vectors that are dependent on an aggregate to within rounding
    cannot be orthonormalised accurately by Cholesky QR: the import fails
    with EINVAL instead of producing an inaccurate P; a well separated set
    still matches the oracle."""
    from oracle.aggregation import Aggregation
    from tests.gpu_util import export_P
    S = Setup(dd, (8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [4]), prec=dd.F64)
    tv = W.test_vectors(S.dims, 12, 4, 7705)
    bad = tv.copy()
    bad[3] = bad[2] + 1e-9 * tv[3]
    with pytest.raises(dd.DDAMGError) as e:
        dd.import_test_vectors(S.H, 0, dev(bad))
    assert e.value.status == dd.EINVAL and "dependent" in str(e.value)
    ok = tv.copy()
    ok[3] = ok[2] + 1e-3 * tv[3]
    dd.import_test_vectors(S.H, 0, dev(ok))
    e2 = np.max(np.abs(export_P(dd, S.H, 0, 4) - Aggregation(S.dims, (4, 4, 4, 4), ok).columns()))
    say(f"  conditioned 1e-3 set: P max abs diff {e2:.2e}")
    assert e2 < 1e-9
