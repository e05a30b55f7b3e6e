"""ddamg_apply_D_noalloc (the entry point that allocates nothing) against
ddamg_apply_D with the canonical layout, through the C ABI: two calls in a
row, the second on a smaller input, in FP64 and FP32; and the size limit
rejected on the host."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import dev, empty, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_matches_apply_D(dd):
    big, small = (8, 8, 8, 16), (4, 4, 8, 8)
    ctxs = {}
    for dims in (big, small):
        U = W.links(dims, 0.5, 7000 + dims[3])
        ctxs[dims] = dd.create(dims, -0.3, 1.0, dev(U))
    for prec, tol in ((dd.F64, 1e-13), (dd.F32, 1e-6)):
        for dims, nrhs in ((big, 3), (small, 1)):
            say(f"  noalloc apply_D prec={prec} dims={dims} nrhs={nrhs}")
            psi = W.gaussian_spinor(dims, 7100 + nrhs, nrhs=nrhs)
            ref = empty(psi.shape)
            dd.apply_D(ctxs[dims], dev(psi), ref, nrhs=nrhs, prec=prec)
            out = empty(psi.shape)
            dd.apply_D_noalloc(ctxs[dims], dev(psi), out, nrhs=nrhs, prec=prec)
            e = _rel(host(out), host(ref))
            say(f"    relerr vs ddamg_apply_D {e:.2e}")
            assert e <= tol


def test_noalloc_size_limit(dd):
    dims = (16, 16, 16, 16)
    U = W.links(dims, 0.5, 7200)
    ctx = dd.create(dims, -0.3, 1.0, dev(U))
    # 2 fields x 65536 sites x 192 bytes = 25 MB per right-hand side in FP64
    nrhs = dd.NOALLOC_SCRATCH_BYTES // (2 * 65536 * 192) + 1
    x = empty((nrhs,) + (16, 16, 16, 16, 12))
    y = empty(x.shape)
    with pytest.raises(dd.DDAMGError) as ei:
        dd.apply_D_noalloc(ctx, x, y, nrhs=nrhs, prec=dd.F64)
    assert ei.value.status == dd.EINVAL and "staging" in str(ei.value)
    dd.apply_D_noalloc(ctx, x[:1], y[:1], nrhs=1, prec=dd.F64)
    torch.cuda.synchronize()
