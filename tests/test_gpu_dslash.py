"""GPU parity of the Wilson-clover stencil (the operator of eq. (1)) against
the FP64 oracle, through the C ABI.  Tolerances: 1e-13 relative in FP64,
1e-5 in FP32 (norm-wise over the whole field)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.dirac import WilsonClover
from oracle.lattice import shape
from tests.gpu_util import dev, empty, host, relerr, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


CASES = [((4, 4, 4, 8), 0.5, -0.3, 0.0), ((4, 4, 4, 8), 0.5, -0.3, 1.0),
         ((8, 4, 12, 4), 0.4, -0.4, 1.3), ((8, 8, 8, 8), 0.6, -0.2, 1.0)]


@pytest.mark.parametrize("dims,eps,m0,csw", CASES)
def test_apply_D_parity(dd, dims, eps, m0, csw):
    say(f"apply_D parity dims={dims} csw={csw}")
    U = W.links(dims, eps, 1000 + sum(dims))
    op = WilsonClover(U, m0, csw)
    psi = W.gaussian_spinor(dims, 77, nrhs=2)
    ref = np.stack([op.apply(p) for p in psi])
    ctx = dd.create(dims, m0, csw, dev(U))
    for prec, tol in ((dd.F64, 1e-13), (dd.F32, 1e-5)):
        out = empty(psi.shape)
        dd.apply_D(ctx, dev(psi), out, nrhs=2, prec=prec)
        got = host(out)
        for r in range(2):
            e = relerr(got[r], ref[r])
            say(f"  prec={prec} rhs={r} relerr={e:.3e}")
            assert e <= tol


def test_native_layout_roundtrip_and_apply(dd):
    dims = (4, 8, 4, 4)
    U = W.links(dims, 0.5, 5)
    ctx = dd.create(dims, -0.3, 1.0, dev(U))
    psi = W.gaussian_spinor(dims, 6, nrhs=3)
    x = dev(psi)
    V = int(np.prod(dims))
    for prec, cdt in ((dd.F64, torch.complex128), (dd.F32, torch.complex64)):
        nat = torch.zeros((3, V * 12), dtype=cdt, device="cuda")
        dd.to_native(ctx, None, 0, x, nat, nrhs=3, prec=prec)
        back = empty(psi.shape)
        dd.from_native(ctx, None, 0, nat, back, nrhs=3, prec=prec)
        if prec == dd.F64:
            assert np.array_equal(host(back), psi)
        else:
            assert np.array_equal(host(back), psi.astype(np.complex64).astype(np.complex128))
        # native apply equals canonical apply bit for bit
        nout = torch.zeros_like(nat)
        dd.apply_D(ctx, nat, nout, nrhs=3, prec=prec, layout=dd.NATIVE)
        a = empty(psi.shape)
        dd.from_native(ctx, None, 0, nout, a, nrhs=3, prec=prec)
        b = empty(psi.shape)
        dd.apply_D(ctx, dev(host(back)), b, nrhs=3, prec=prec)
        assert np.array_equal(host(a), host(b))


def test_apply_D_full_size_16x32(dd):
    """The 16^3x32 clover workload (eps 0.5, m0 -0.4, c_sw 1): whole field."""
    cfg = W.CONFIGS["clover16x32_3lvl"]
    dims = cfg["dims"]
    say(f"apply_D full-size {dims}")
    U = W.links(dims, cfg["eps"], cfg["seed_links"])
    op = WilsonClover(U, cfg["m0"], cfg["csw"])
    psi = W.gaussian_spinor(dims, cfg["seed_rhs"])
    ref = op.apply(psi)
    ctx = dd.create(dims, cfg["m0"], cfg["csw"], dev(U))
    for prec, tol in ((dd.F64, 1e-13), (dd.F32, 1e-5)):
        out = empty(psi.shape)
        dd.apply_D(ctx, dev(psi), out, prec=prec)
        e = relerr(host(out), ref)
        say(f"  prec={prec} relerr={e:.3e}")
        assert e <= tol


@pytest.mark.parametrize("name", ["clover32x64_3lvl_12rhs"])
def test_apply_D_sampled_full_size(dd, name):
    """The 32^3x64 workload's operator on three fields in one launch (the
    batched launch of its 12-source solves), FP64 and FP32, checked on 64
    sampled sites per field against the oracle's site-by-site evaluation
    (the whole-lattice oracle is too slow at 2.1 M sites)."""
    from oracle.dirac import apply_at_sites
    cfg = W.CONFIGS[name]
    dims = cfg["dims"]
    say(f"apply_D sampled full-size {dims}")
    U = W.links(dims, cfg["eps"], cfg["seed_links"])
    psi = W.gaussian_spinor(dims, cfg["seed_rhs"], nrhs=3)
    ctx = dd.create(dims, cfg["m0"], cfg["csw"], dev(U))
    rng = np.random.Generator(np.random.PCG64(2024))
    sites = [tuple(int(rng.integers(0, e)) for e in dims) for _ in range(64)]
    refs = [apply_at_sites(U, cfg["m0"], cfg["csw"], psi[r], sites) for r in range(3)]
    for prec, tol in ((dd.F64, 1e-13), (dd.F32, 1e-5)):
        out = empty(psi.shape)
        dd.apply_D(ctx, dev(psi), out, nrhs=3, prec=prec)
        o = host(out)
        for r in range(3):
            got = np.array([o[r, t, z, y, x] for (x, y, z, t) in sites])
            e = relerr(got, refs[r])
            say(f"  prec={prec} field {r}: sampled relerr={e:.3e}")
            assert e <= tol


def test_bad_arguments_raise(dd):
    dims = (4, 4, 4, 4)
    U = W.links(dims, 0.5, 9)
    ctx = dd.create(dims, -0.3, 1.0, dev(U))
    x = empty((int(np.prod(dims)), 12))
    with pytest.raises(dd.DDAMGError) as e:
        dd.apply_D(ctx, x, x)
    assert e.value.status == dd.EINVAL
    with pytest.raises(dd.DDAMGError):
        dd.apply_D(ctx, x, empty(x.shape), prec=7)
