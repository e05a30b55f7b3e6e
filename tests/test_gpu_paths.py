"""Kernel paths that only the larger workloads reach, each compared with the
FP64 oracle on the same seeded inputs at the smallest lattice that takes
the path:

* the coarse Galerkin product D_{l+1} = P_l^H D_l P_l (Sec. 1, Sec. 2) with
  one and with four columns of P per workgroup, including a test-vector
  count that is not a multiple of four;
* the coarse SAP smoother (Sec. 2, Tab. 1) with 3^4 blocks (81 sites: more
  than one wavefront per block);
* coarse operators with 56 components per site (28 test vectors, the
  four-level workload's coarsest level), applied by the per-site kernel and
  by the matrix-core kernel, and the odd-even coarsest solve (Sec. 3) on
  them with the dense and the sparse Schur product;
* the extra fresh test vectors of a level that has more of them than the
  level above (the initial setup, Alg. 3), against the oracle's setup;
* a non-bipartite coarsest lattice with 40 components per site (GMRES on
  the full coarsest system, Sec. 3).

The GPU imports test vectors drawn by the seeded generators (so P and D_c
are defined by the oracle's inputs), or the oracle is rebuilt from the
GPU's exported bases where the setup itself is under test."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import multigrid as mg
from oracle.aggregation import Aggregation
from oracle.dirac import WilsonClover
from oracle.galerkin import galerkin
from oracle.krylov import norm
from oracle.sap import sap_sweep
from tests.gpu_util import (dev, empty, export_Dc, export_P, host, oracle_from_gpu, relerr, say,
                            to_params)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


def _p(levels, agg, ntv, **kw):
    p = dict(W.DEFAULT_PARAMS)
    p.update(levels=levels, agg=agg, ntv=ntv, n_inv=0, nu=2)
    p.update(kw)
    return p


def _nine(D):
    return np.concatenate([D.S[..., None, :, :], np.moveaxis(D.F, 0, -3), np.moveaxis(D.B, 0, -3)], axis=-3)


# ---------------------------------------------------------------------------
# 24^4 fine lattice: level 1 is 6^4 x 8 (3^4 SAP blocks, 3^4 aggregates),
# level 2 is 2^4 x 12
# ---------------------------------------------------------------------------
DIMS24 = (24, 24, 24, 24)


@pytest.fixture(scope="module")
def lat24(dd):
    say(f"lattice {DIMS24}: links and oracle operator")
    U = W.links(DIMS24, 0.5, 2401)
    op = WilsonClover(U, -0.3, 0.0)
    ctx = dd.create(DIMS24, -0.3, 0.0, dev(U))
    tv0 = W.test_vectors(DIMS24, 12, 4, 2402)
    tv1 = W.test_vectors((6, 6, 6, 6), 8, 6, 2403)
    extra = W.test_vectors((6, 6, 6, 6), 8, 2, 2406)   # level 1 has 6 vectors, 4 come from level 0
    say("  oracle P_0, D_1")
    A0 = Aggregation(DIMS24, (4, 4, 4, 4), tv0)
    D1 = galerkin(op, A0)
    say("  oracle P_1, D_2")
    A1 = Aggregation((6, 6, 6, 6), (3, 3, 3, 3), tv1)
    D2 = galerkin(D1, A1)
    return dict(ctx=ctx, op=op, tv0=tv0, tv1=tv1, extra=extra, D1=D1, D2=D2)


def _hier24(dd, L, cols):
    p = _p(3, [(4, 4, 4, 4), (3, 3, 3, 3)], [4, 6], sap_blocks=[(2, 2, 2, 2), (3, 3, 3, 3)])
    P = to_params(dd, p, dd.F64)
    P.galerkin_cols = cols
    H = dd.build_hierarchy(L["ctx"], P, dev(L["tv0"]), dev(L["extra"]))
    dd.import_test_vectors(H, 0, dev(L["tv0"]))
    dd.import_test_vectors(H, 1, dev(L["tv1"]))
    torch.cuda.synchronize()
    return H


@pytest.mark.timeout(600)
@pytest.mark.parametrize("cols", [1, 4])
def test_coarse_galerkin_column_groups(dd, lat24, cols):
    """D_2 = P_1^H D_1 P_1 on 81-site aggregates with 6 test vectors (one
    full group of four columns and one of two), one or four columns per
    workgroup, against the oracle's Galerkin product; D_1 too."""
    H = _hier24(dd, lat24, cols)
    assert dd.level_info(H, 1) == ((6, 6, 6, 6), 8)
    assert dd.level_info(H, 2) == ((2, 2, 2, 2), 12)
    e1 = relerr(export_Dc(dd, H, 1), _nine(lat24["D1"]))
    e2 = relerr(export_Dc(dd, H, 2), _nine(lat24["D2"]))
    say(f"  galerkin_cols={cols}: D_1 relerr {e1:.2e}, D_2 relerr {e2:.2e}")
    assert e1 < 1e-12 and e2 < 1e-12


@pytest.mark.timeout(600)
def test_coarse_sap_3x3x3x3_blocks(dd, lat24):
    """One SAP step on the 6^4 level with 3^4 blocks (2^4 blocks of 81 sites)
    against the oracle's SAP on its own D_1, single and batched."""
    H = _hier24(dd, lat24, 0)
    D1 = lat24["D1"]
    b = W.gaussian_field(D1.dims, D1.d, 2404, nrhs=3)
    z0 = W.gaussian_field(D1.dims, D1.d, 2405, nrhs=3)
    ref = np.stack([sap_sweep(D1, b[r], z0[r], (3, 3, 3, 3), 3) for r in range(3)])
    for prec, tol in ((dd.F64, 1e-12), (dd.F32, 1e-5)):
        for nb in (1, 3):
            z = dev(z0[:nb])
            dd.sap_smooth(H, 1, dev(b[:nb]), z, 1, nrhs=nb, prec=prec)
            e = relerr(host(z), ref[:nb])
            say(f"  3^4-block coarse SAP prec={prec} nrhs={nb}: relerr {e:.2e}")
            assert e < tol


# ---------------------------------------------------------------------------
# 56 components per site: 16^4 fine, N = 4 then 28
# ---------------------------------------------------------------------------
DIMS16 = (16, 16, 16, 16)


@pytest.fixture(scope="module")
def d56(dd):
    say("d = 56: 16^4 fine, N = 4 / 28")
    U = W.links(DIMS16, 0.5, 5601)
    op = WilsonClover(U, -0.25, 1.0)
    ctx = dd.create(DIMS16, -0.25, 1.0, dev(U))
    p = _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 28], coarse_eps=1e-8, coarse_restart=30, coarse_max_restarts=40)
    tv0 = W.test_vectors(DIMS16, 12, 4, 5602)
    tv1 = W.test_vectors((4, 4, 4, 4), 8, 28, 5603)
    extra = W.test_vectors((4, 4, 4, 4), 8, 24, 5606)   # level 1 has 28 vectors, 4 come from level 0
    OH = mg.Hierarchy(op, p)
    OH.tv[0] = tv0
    OH.build_level(0)
    OH.tv[1] = tv1
    OH.build_level(1)
    return dict(ctx=ctx, op=op, p=p, tv0=tv0, tv1=tv1, extra=extra, OH=OH)


def _hier56(dd, c, prec, dense=1):
    P = to_params(dd, c["p"], prec)
    P.coarse_dense = dense
    H = dd.build_hierarchy(c["ctx"], P, dev(c["tv0"]), dev(c["extra"]))
    dd.import_test_vectors(H, 0, dev(c["tv0"]))
    dd.import_test_vectors(H, 1, dev(c["tv1"]))
    torch.cuda.synchronize()
    return H


def test_d56_coarse_apply(dd, d56):
    """D_2 with 56 components per site: per-site kernel (1 field, FP64 and
    FP32) and matrix-core kernel (12 fields, FP32)."""
    H = _hier56(dd, d56, dd.F32)
    assert dd.level_info(H, 2) == ((2, 2, 2, 2), 56)
    D2 = d56["OH"].ops[2]
    assert relerr(export_Dc(dd, H, 2), _nine(D2)) < 1e-12
    v = W.gaussian_field(D2.dims, 56, 5604, nrhs=12)
    ref = np.stack([D2.apply(x) for x in v])
    for prec, nb, tol in ((dd.F64, 1, 1e-13), (dd.F32, 1, 1e-5), (dd.F32, 12, 1e-5), (dd.F64, 12, 1e-13)):
        out = empty(v[:nb].shape)
        dd.apply_Dc(H, 2, dev(v[:nb]), out, nrhs=nb, prec=prec)
        e = relerr(host(out), ref[:nb])
        say(f"  d=56 apply prec={prec} nrhs={nb}: relerr {e:.2e}")
        assert e < tol


@pytest.mark.parametrize("dense", [1, 0])
def test_d56_one_cycle(dd, d56, dense):
    """One K-cycle with the d = 56 coarsest level (odd-even Schur system,
    self blocks of 56 x 56 inverted on the device), dense and sparse Schur
    product, against the oracle (FP64)."""
    H = _hier56(dd, d56, dd.F64, dense)
    b = W.gaussian_spinor(DIMS16, 5605)
    ref = d56["OH"].cycle(0, b)
    z = empty(b.shape)
    dd.precondition(H, dev(b), z)
    e = relerr(host(z), ref)
    say(f"  d=56 one cycle (dense={dense}): relerr {e:.2e}")
    assert e < 1e-9


def test_four_level_extra_test_vectors_initial_setup(dd):
    """Four levels, N = 4 / 4 / 28: level 2 takes the 4 restricted vectors
    and 24 fresh ones (Alg. 3 with more vectors than the level above).  The
    initial setup (no iterative phase) of the GPU in FP64 against the
    oracle's from the same inputs: interpolations on every level; then one
    cycle against the oracle on the GPU's bases (coarsest 1^4 x 56, GMRES on
    the full system)."""
    p = _p(4, [(4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2)], [4, 4, 28],
           sap_blocks=[(2, 2, 2, 2), (2, 2, 2, 2), (1, 1, 1, 1)])
    U = W.links(DIMS16, 0.5, 5701)
    op = WilsonClover(U, -0.25, 1.0)
    ctx = dd.create(DIMS16, -0.25, 1.0, dev(U))
    tv0 = W.test_vectors(DIMS16, 12, 4, 5702)
    extra = W.test_vectors((2, 2, 2, 2), 8, 24, 5703)
    H = dd.build_hierarchy(ctx, to_params(dd, p, dd.F64), dev(tv0), dev(extra))
    assert dd.level_info(H, 3) == ((1, 1, 1, 1), 56)
    say("  oracle initial setup")
    OH = mg.Hierarchy(op, p)
    mg.initial_setup(OH, 0, tv0, {2: extra})
    for l in range(3):
        e = relerr(export_P(dd, H, l, p["ntv"][l]), OH.aggs[l].columns())
        say(f"  level {l} interpolation relerr {e:.2e}")
        assert e < 1e-10
    OG = oracle_from_gpu(dd, H, op, p)
    b = W.gaussian_spinor(DIMS16, 5704)
    z = empty(b.shape)
    dd.precondition(H, dev(b), z)
    e = relerr(host(z), OG.cycle(0, b))
    say(f"  four-level cycle relerr {e:.2e}")
    assert e < 1e-9


# ---------------------------------------------------------------------------
# non-bipartite coarsest with 40 components: 12^4 fine, 3^4 coarsest
# ---------------------------------------------------------------------------
def test_nonbipartite_d40_coarsest(dd):
    dims = (12, 12, 12, 12)
    p = _p(2, [(4, 4, 4, 4)], [20])
    U = W.links(dims, 0.5, 4001)
    op = WilsonClover(U, -0.3, 1.0)
    ctx = dd.create(dims, -0.3, 1.0, dev(U))
    tv0 = W.test_vectors(dims, 12, 20, 4002)
    H = dd.build_hierarchy(ctx, to_params(dd, p, dd.F64), dev(tv0))
    dd.import_test_vectors(H, 0, dev(tv0))
    assert dd.level_info(H, 1) == ((3, 3, 3, 3), 40)
    OH = mg.Hierarchy(op, p)
    OH.tv[0] = tv0
    OH.build_level(0)
    assert not OH.coarsest.bipartite
    b = W.gaussian_spinor(dims, 4003)
    z = empty(b.shape)
    dd.precondition(H, dev(b), z)
    e = relerr(host(z), OH.cycle(0, b))
    say(f"  non-bipartite d=40 one cycle relerr {e:.2e}")
    assert e < 1e-9
    H32 = dd.build_hierarchy(ctx, to_params(dd, p, dd.F32), dev(tv0))
    zs = W.gaussian_spinor(dims, 4004)
    bb = op.apply(zs)
    z = empty(bb.shape)
    rc, st = dd.solve(H32, dev(bb), z)
    zz = host(z)
    res = norm(bb - op.apply(zz)) / norm(bb)
    say(f"  FP32-preconditioned solve rc={rc} {st[0]} oracle relres {res:.2e}")
    assert rc == dd.OK and res <= 1e-10 and relerr(zz, zs) < 1e-8
