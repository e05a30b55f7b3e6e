"""Handles whose device memory is a caller-owned (torch) workspace: the
query's count is what the build takes, nothing else is allocated on the
device during the build and the solves, and the results equal those of the
library-owned handles."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.dirac import WilsonClover
from oracle.krylov import norm
from tests.gpu_util import dev, empty, host, say, to_params
from tests.test_gpu_hierarchy import _p

pytestmark = pytest.mark.gpu

DIMS = (16, 16, 16, 16)
M0, CSW = -0.25, 1.0


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("half", [0, 1])
def test_solve_in_torch_workspace(dd, half):
    p = _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 4], n_inv=2)
    prec = dd.F32
    P = to_params(dd, p, prec, half=bool(half))
    U = W.links(DIMS, 0.5, 4242)
    op = WilsonClover(U, M0, CSW)
    tv = dev(W.test_vectors(DIMS, 12, 4, 4243))
    zstar = W.gaussian_spinor(DIMS, 4244, nrhs=2)
    b = dev(np.stack([op.apply(x) for x in zstar]))
    Ud = dev(U)

    # library-owned handles
    ctx0 = dd.create(DIMS, M0, CSW, Ud)
    H0 = dd.build_hierarchy(ctx0, P, tv)
    z0 = empty(zstar.shape)
    rc0, st0 = dd.solve(H0, b, z0, nrhs=2)
    assert rc0 == dd.OK
    v1 = dev(W.gaussian_field((4, 4, 4, 4), 8, 4245, nrhs=2))
    o0 = empty(tuple(v1.shape))
    dd.apply_Dc(H0, 1, v1, o0, nrhs=2, prec=dd.F64)

    cb, hb = dd.workspace_bytes(DIMS, M0, CSW, P, nrhs_max=2)
    say(f"  half={half}: context {cb / 2**20:.1f} MiB, hierarchy {hb / 2**20:.1f} MiB")
    wc = torch.empty(cb, dtype=torch.uint8, device="cuda")
    wh = torch.empty(hb, dtype=torch.uint8, device="cuda")
    z = empty(zstar.shape)
    o = empty(tuple(v1.shape))
    free0 = _free()
    ctx = dd.create_ws(DIMS, M0, CSW, Ud, wc, params=P, nrhs_max=2)
    H = dd.build_hierarchy_ws(ctx, P, tv, wh, nrhs_max=2)
    rc, st = dd.solve(H, b, z, nrhs=2)
    dd.apply_Dc(H, 1, v1, o, nrhs=2, prec=dd.F64)
    drop = free0 - _free()
    say(f"  device memory taken outside the workspaces: {drop / 2**20:.1f} MiB")
    assert drop < 32 * 2**20 < (cb + hb) // 8
    assert rc == dd.OK
    for r in range(2):
        assert st[r]["outer_iters"] == st0[r]["outer_iters"]
        assert st[r]["kcycle_iters"] == st0[r]["kcycle_iters"]
    zz, zz0 = host(z), host(z0)
    assert np.max(np.abs(zz - zz0)) <= 1e-12 * np.max(np.abs(zz0))
    assert np.array_equal(host(o), host(o0))
    # certified by the oracle's FP64 operator
    for r in range(2):
        res = norm(host(b)[r] - op.apply(zz[r])) / norm(host(b)[r])
        assert res <= 1e-10 * 1.01
    del H, ctx
    torch.cuda.synchronize()


def test_workspace_exhaustion_is_an_error(dd):
    """Work beyond the count draws on the rest of the workspace: ENOMEM when
    there is none (here an FP64 canonical-layout call on an FP32 hierarchy,
    whose scratch was counted at FP32), and the handle stays usable."""
    p = _p(2, [(4, 4, 4, 4)], [4], n_inv=1)
    dims = (8, 8, 8, 8)
    P = to_params(dd, p, dd.F32)
    U = W.links(dims, 0.5, 515)
    cb, hb = dd.workspace_bytes(dims, M0, CSW, P, nrhs_max=1)
    wc = torch.empty(cb, dtype=torch.uint8, device="cuda")
    wh = torch.empty(hb, dtype=torch.uint8, device="cuda")
    ctx = dd.create_ws(dims, M0, CSW, dev(U), wc, params=P, nrhs_max=1)
    H = dd.build_hierarchy_ws(ctx, P, dev(W.test_vectors(dims, 12, 4, 516)), wh, nrhs_max=1)
    x = dev(W.gaussian_spinor(dims, 517, nrhs=1))
    ref = WilsonClover(U, M0, CSW).apply(host(x)[0])
    with pytest.raises(dd.DDAMGError) as e:
        dd.apply_Dc(H, 0, x, empty(tuple(x.shape)), nrhs=1, prec=dd.F64)
    assert e.value.status == dd.ENOMEM and "workspace" in str(e.value)
    y = empty(tuple(x.shape))
    dd.apply_Dc(H, 0, x, y, nrhs=1, prec=dd.F32)
    assert np.max(np.abs(host(y)[0] - ref)) <= 1e-5 * np.max(np.abs(ref))
