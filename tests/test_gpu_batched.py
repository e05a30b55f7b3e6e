"""Batched right-hand sides: every level operation of the C ABI applied to
nrhs fields in one batched launch (the link, clover, interpolation and
coarse-operator entries are loaded once per site and used for all fields
of the batch), compared field by field with the FP64 oracle.  Batch sizes
cover the per-thread chunking (4 fields per thread in FP32, 2 in FP64, and
the remainders) and the matrix-core path of the coarse operator (FP32,
8 or more fields, components per site a multiple of 4).

Tolerances as for single fields: 1e-13 (FP64) and 1e-5 (FP32) for the
operators and transfers, 1e-12 / 1e-5 for the smoothers; FP16 storage
4 u_16 ~ 2e-3."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.aggregation import Aggregation
from oracle.dirac import WilsonClover
from oracle.sap import sap_sweep
from tests.gpu_util import dev, empty, export_P, host, oracle_from_gpu, relerr, say, to_params
from tests.test_gpu_hierarchy import Setup, _p

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-5}       # by precision code (F64 = 0, F32 = 1)
HALF_TOL = 4 * 2.0 ** -11


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


@pytest.fixture(scope="module")
def wide(dd):
    """two levels on 8^4 with 20 test vectors: a 2^4 coarse lattice with
    d = 40 (three 16-row matrix-core tiles, the last one partial)"""
    return Setup(dd, (8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [20]), prec=dd.F32)


@pytest.fixture(scope="module")
def wide_half(dd):
    return Setup(dd, (8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [20]), prec=dd.F32, half=True)


@pytest.fixture(scope="module")
def three(dd):
    return Setup(dd, (16, 16, 16, 16), _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 4]), m0=-0.25, seed=99)


def _check(got, ref, tol, what):
    for r in range(ref.shape[0]):
        e = relerr(got[r], ref[r])
        assert e <= tol, f"{what}: field {r} relerr {e:.3e} > {tol}"
    say(f"  {what}: {ref.shape[0]} fields, max relerr "
        f"{max(relerr(got[r], ref[r]) for r in range(ref.shape[0])):.2e}")


@pytest.mark.parametrize("nrhs", [3, 5, 12])
def test_batched_apply_D(dd, nrhs):
    dims = (8, 4, 8, 8)
    U = W.links(dims, 0.5, 4242)
    op = WilsonClover(U, -0.3, 1.0)
    psi = W.gaussian_spinor(dims, 4243, nrhs=nrhs)
    ref = np.stack([op.apply(p) for p in psi])
    ctx = dd.create(dims, -0.3, 1.0, dev(U))
    for prec in (dd.F64, dd.F32):
        out = empty(psi.shape)
        dd.apply_D(ctx, dev(psi), out, nrhs=nrhs, prec=prec)
        _check(host(out), ref, TOL[prec], f"apply_D nrhs={nrhs} prec={prec}")


def test_batched_apply_D_native_matches_single(dd):
    """the native batched call equals nrhs single-field calls in FP64 up to
    the rounding of a different contraction of the same sums"""
    dims = (4, 8, 4, 8)
    U = W.links(dims, 0.4, 17)
    ctx = dd.create(dims, -0.2, 1.0, dev(U))
    nrhs, V = 6, int(np.prod(dims))
    psi = dev(W.gaussian_spinor(dims, 18, nrhs=nrhs))
    nat = torch.zeros((nrhs, V * 12), dtype=torch.complex128, device="cuda")
    dd.to_native(ctx, None, 0, psi, nat, nrhs=nrhs, prec=dd.F64)
    outb = torch.zeros_like(nat)
    dd.apply_D(ctx, nat, outb, nrhs=nrhs, prec=dd.F64, layout=dd.NATIVE)
    for r in range(nrhs):
        o1 = torch.zeros_like(nat[r])
        dd.apply_D(ctx, nat[r].contiguous(), o1, nrhs=1, prec=dd.F64, layout=dd.NATIVE)
        e = float(torch.linalg.vector_norm(o1 - outb[r]) / torch.linalg.vector_norm(o1))
        assert e <= 1e-15, e


@pytest.mark.parametrize("nrhs", [3, 12, 20])
def test_batched_coarse_apply_d40(dd, wide, nrhs):
    OH = oracle_from_gpu(dd, wide.H, wide.op, wide.p)
    Dc = OH.ops[1]
    v = W.gaussian_field(Dc.dims, Dc.d, 300 + nrhs, nrhs=nrhs)
    ref = np.stack([Dc.apply(x) for x in v])
    for prec in (dd.F64, dd.F32):
        out = empty(v.shape)
        dd.apply_Dc(wide.H, 1, dev(v), out, nrhs=nrhs, prec=prec)
        _check(host(out), ref, TOL[prec], f"apply_Dc d=40 nrhs={nrhs} prec={prec}")


def test_batched_coarse_apply_half(dd, wide_half):
    OH = oracle_from_gpu(dd, wide_half.H, wide_half.op, wide_half.p)
    Dc = OH.ops[1]
    v = W.gaussian_field(Dc.dims, Dc.d, 401, nrhs=12)
    ref = np.stack([Dc.apply(x) for x in v])
    out = empty(v.shape)
    dd.apply_Dc(wide_half.H, 1, dev(v), out, nrhs=12, prec=dd.F32)
    _check(host(out), ref, HALF_TOL, "apply_Dc FP16 storage nrhs=12")


def test_batched_transfers(dd, three):
    nrhs = 7
    agg = Aggregation(three.dims, (4, 4, 4, 4), export_P(dd, three.H, 0, 4))
    v = W.gaussian_spinor(three.dims, 501, nrhs=nrhs)
    c = W.gaussian_field(agg.cdims, 8, 502, nrhs=nrhs)
    rref = np.stack([agg.restrict(x) for x in v])
    pref = np.stack([v[r] + agg.prolong(c[r]) for r in range(nrhs)])
    for prec in (dd.F64, dd.F32):
        out = empty(c.shape)
        dd.restrict(three.H, 0, dev(v), out, nrhs=nrhs, prec=prec)
        _check(host(out), rref, 1e-13 if prec == dd.F64 else 1e-6, f"restrict fine prec={prec}")
        f = dev(v)
        dd.prolong(three.H, 0, dev(c), f, nrhs=nrhs, prec=prec)
        _check(host(f), pref, 1e-13 if prec == dd.F64 else 1e-6, f"prolong fine prec={prec}")
    OH = oracle_from_gpu(dd, three.H, three.op, three.p)
    a1 = OH.aggs[1]
    v1 = W.gaussian_field(OH.ops[1].dims, OH.ops[1].d, 503, nrhs=nrhs)
    c1 = W.gaussian_field(a1.cdims, 8, 504, nrhs=nrhs)
    rref = np.stack([a1.restrict(x) for x in v1])
    pref = np.stack([v1[r] + a1.prolong(c1[r]) for r in range(nrhs)])
    for prec in (dd.F64, dd.F32):
        out = empty(c1.shape)
        dd.restrict(three.H, 1, dev(v1), out, nrhs=nrhs, prec=prec)
        _check(host(out), rref, 1e-13 if prec == dd.F64 else 1e-6, f"restrict coarse prec={prec}")
        f = dev(v1)
        dd.prolong(three.H, 1, dev(c1), f, nrhs=nrhs, prec=prec)
        _check(host(f), pref, 1e-13 if prec == dd.F64 else 1e-6, f"prolong coarse prec={prec}")


def test_batched_smoothers(dd, three):
    nrhs = 6
    b = W.gaussian_spinor(three.dims, 601, nrhs=nrhs)
    z0 = W.gaussian_spinor(three.dims, 602, nrhs=nrhs)
    ref = np.stack([sap_sweep(three.op, b[r], z0[r], (2, 2, 2, 2), 3) for r in range(nrhs)])
    for prec, tol in ((dd.F64, 1e-12), (dd.F32, 1e-5)):
        z = dev(z0)
        dd.sap_smooth(three.H, 0, dev(b), z, 1, nrhs=nrhs, prec=prec)
        _check(host(z), ref, tol, f"fine SAP prec={prec}")
    OH = oracle_from_gpu(dd, three.H, three.op, three.p)
    Dc = OH.ops[1]
    b = W.gaussian_field(Dc.dims, Dc.d, 603, nrhs=nrhs)
    z0 = W.gaussian_field(Dc.dims, Dc.d, 604, nrhs=nrhs)
    ref = np.stack([sap_sweep(Dc, b[r], z0[r], (2, 2, 2, 2), 3) for r in range(nrhs)])
    for prec, tol in ((dd.F64, 1e-12), (dd.F32, 1e-5)):
        z = dev(z0)
        dd.sap_smooth(three.H, 1, dev(b), z, 1, nrhs=nrhs, prec=prec)
        _check(host(z), ref, tol, f"coarse SAP prec={prec}")


@pytest.mark.parametrize("nrhs", [12, 20])
def test_batched_transfers_matrix_cores(dd, nrhs):
    """Batches of 8 or more fields take the matrix-core restriction and
    prolongation (16 fields per launch chunk, here one full chunk and one of
    4 after it): against the oracle at FP32 accuracy, with N = 20 test
    vectors (two 16-column tiles, the second partly empty).  Tolerance: each
    coarse entry of the restriction sums 96 FP32 products per 2^4 block and
    then 16 block sums, so its rounding error is typically
    (sqrt(96) + sqrt(16)) u ~ 8e-7 (u = 2^-24), at most a few times that:
    4e-6."""
    S = Setup(dd, (8, 8, 8, 16), _p(2, [(4, 4, 4, 4)], [20]), prec=dd.F32)
    agg = Aggregation(S.dims, (4, 4, 4, 4), export_P(dd, S.H, 0, 20))
    v = W.gaussian_spinor(S.dims, 511, nrhs=nrhs)
    c = W.gaussian_field(agg.cdims, 40, 512, nrhs=nrhs)
    rref = np.stack([agg.restrict(x) for x in v])
    pref = np.stack([v[r] + agg.prolong(c[r]) for r in range(nrhs)])
    out = empty(c.shape)
    dd.restrict(S.H, 0, dev(v), out, nrhs=nrhs, prec=dd.F32)
    _check(host(out), rref, 4e-6, f"restrict fine on the matrix cores, nrhs={nrhs}")
    f = dev(v)
    dd.prolong(S.H, 0, dev(c), f, nrhs=nrhs, prec=dd.F32)
    _check(host(f), pref, 4e-6, f"prolong fine on the matrix cores, nrhs={nrhs}")
    # FP16 interpolation (FP32 arithmetic): within the FP16-storage band
    P16 = to_params(dd, S.p, dd.F32, half=True)
    H16 = dd.build_hierarchy(S.ctx, P16, dev(S.tv))
    a16 = Aggregation(S.dims, (4, 4, 4, 4), export_P(dd, H16, 0, 20))
    out = empty(c.shape)
    dd.restrict(H16, 0, dev(v), out, nrhs=nrhs, prec=dd.F16)
    e = max(np.linalg.norm(host(out)[r] - a16.restrict(v[r])) / np.linalg.norm(a16.restrict(v[r]))
            for r in range(nrhs))
    say(f"  FP16 P, matrix cores: restrict relerr {e:.2e}")
    assert 1e-5 < e < 4 * 2.0 ** -11
