"""Runtime re-blocking of a coarse level's SAP (ddamg_set_sap_block) against
the oracle's SAP with the new blocks, its validation, and the autotuner:
the search returns a valid choice, stores it in the cache and reads it back
from there, and the tuned hierarchy still solves to 1e-10."""
import json

import pytest
import torch

import workloads as W
from oracle.krylov import norm
from oracle.sap import sap_sweep
from tests.gpu_util import dev, empty, host, oracle_from_gpu, relerr, say
from tests.test_gpu_hierarchy import Setup, _p

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


@pytest.fixture(scope="module")
def three(dd):
    # level 1 is 4^3 x 8: several valid block shapes
    return Setup(dd, (16, 16, 16, 32), _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 4]), m0=-0.25, seed=123,
                 prec=dd.F32)


def test_reblocked_coarse_sap_parity(dd, three):
    OH = oracle_from_gpu(dd, three.H, three.op, three.p)
    Dc = OH.ops[1]
    b = W.gaussian_field(Dc.dims, Dc.d, 51)
    z0 = W.gaussian_field(Dc.dims, Dc.d, 52)
    for blk in ((2, 2, 2, 4), (2, 2, 2, 1), (2, 2, 2, 2)):
        dd.set_sap_block(three.H, 1, blk)
        ref = sap_sweep(Dc, b, z0, blk, 3)
        for prec, tol in ((dd.F64, 1e-12), (dd.F32, 1e-5)):
            z = dev(z0)
            dd.sap_smooth(three.H, 1, dev(b), z, 1, prec=prec)
            e = relerr(host(z), ref)
            say(f"  SAP blocks {blk} prec={prec} relerr={e:.2e}")
            assert e < tol


def test_set_sap_block_validation(dd, three):
    for level, blk in ((1, (3, 3, 3, 3)), (1, (2, 2, 4, 2)), (1, (2, 2, 2, 8)), (0, (2, 2, 2, 2)),
                       (2, (2, 2, 2, 2))):
        with pytest.raises(dd.DDAMGError) as e:
            dd.set_sap_block(three.H, level, blk)
        assert e.value.status == dd.EINVAL
    dd.set_sap_block(three.H, 1, (2, 2, 2, 2))


def test_tune_search_cache_and_solve(dd, three, tmp_path):
    cache = tmp_path / "tune.json"
    b = W.gaussian_spinor(three.dims, 61, nrhs=2)
    r1 = dd.tune(three.H, dev(b), nrhs=2, cache=cache)
    say(f"  tuned: {r1}")
    assert not r1["from_cache"]
    blk = r1["sap_block_l"][0]
    dims1 = (4, 4, 4, 8)
    assert all(d % x == 0 and (d // x) % 2 == 0 for d, x in zip(dims1, blk))
    assert 1 <= r1["batch"] <= 2
    text = cache.read_text()
    entries = json.loads(text)
    assert len(entries) == 1
    (key, val), = entries.items()
    assert "|nrhs2" in key and val["sap_block_l"][:4] == blk and val["batch"] == r1["batch"]
    r2 = dd.tune(three.H, dev(b), nrhs=2, cache=cache)
    assert r2["from_cache"] and r2["sap_block_l"] == r1["sap_block_l"] and r2["batch"] == r1["batch"]
    z = empty(b.shape)
    rc, st = dd.solve(three.H, dev(b), z, nrhs=2)
    assert rc == dd.OK
    zz = host(z)
    for r in range(2):
        assert norm(b[r] - three.op.apply(zz[r])) / norm(b[r]) <= 1e-10
