"""Concurrent solves of independent systems on lattices of different sizes
(ddamg_solve_many): every system's result and iteration count equal those
of ddamg_solve on the same hierarchy alone, every solution meets the FP64
residual bound with the oracle's operator, and the argument checks."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.dirac import WilsonClover
from oracle.krylov import norm
from tests.gpu_util import dev, empty, host, relerr, say, to_params
from tests.test_gpu_hierarchy import _p

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


class System:
    def __init__(self, dd, dims, p, eps, m0, csw, seed, nrhs, cycle):
        say(f"system dims={dims} levels={p['levels']} agg={p['agg']} cycle={cycle} nrhs={nrhs}")
        self.dims, self.nrhs = dims, nrhs
        U = W.links(dims, eps, seed)
        self.op = WilsonClover(U, m0, csw)
        self.ctx = dd.create(dims, m0, csw, dev(U))
        tv = W.test_vectors(dims, 12, p["ntv"][0], seed + 1)
        self.H = dd.build_hierarchy(self.ctx, to_params(dd, p, dd.F32, cycle=cycle), dev(tv))
        self.b = W.gaussian_spinor(dims, seed + 2, nrhs=nrhs)
        torch.cuda.synchronize()


@pytest.fixture(scope="module")
def systems(dd):
    return [
        # two-level Wilson, K-cycle, two right-hand sides
        System(dd, (8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [8], n_inv=2), 0.4, -0.3, 0.0, 31, 2, "K"),
        # three-level clover, V-cycle
        System(dd, (16, 16, 16, 16), _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [8, 8]), 0.5, -0.3, 1.0, 41, 1, "V"),
        # 6^4 second level with 3^4 SAP blocks, 3^4 coarsest lattice (no odd-even split)
        System(dd, (24, 24, 24, 24),
               _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [8, 8], sap_blocks=[(2, 2, 2, 2), (3, 3, 3, 3)]),
               0.45, -0.3, 1.0, 51, 1, "V"),
    ]


def test_many_equals_one_at_a_time(dd, systems):
    single = []
    for s in systems:
        z = empty(s.b.shape)
        rc, st = dd.solve(s.H, dev(s.b), z, nrhs=s.nrhs)
        assert rc == dd.OK
        single.append((host(z), st))
        say(f"  alone {s.dims}: its {[x['outer_iters'] for x in st]}")
    bs = [dev(s.b) for s in systems]
    zs = [empty(s.b.shape) for s in systems]
    rc, st = dd.solve_many([s.H for s in systems], bs, zs, nrhs=[s.nrhs for s in systems])
    assert rc == dd.OK
    assert len(st) == sum(s.nrhs for s in systems)
    k = 0
    for s, z, (z1, st1) in zip(systems, zs, single):
        zz = host(z)
        e = relerr(zz, z1)
        its = [x["outer_iters"] for x in st[k:k + s.nrhs]]
        say(f"  together {s.dims}: its {its}, rel. diff to alone {e:.1e}")
        assert its == [x["outer_iters"] for x in st1]
        assert e <= 1e-14
        for r in range(s.nrhs):
            res = norm(s.b[r] - s.op.apply(zz[r])) / norm(s.b[r])
            assert res <= 1e-10
            assert abs(res - st[k + r]["true_relres"]) <= 1e-12
            assert st[k + r]["status"] == dd.OK
        k += s.nrhs


def test_many_twice_in_a_row(dd, systems):
    """A second call reuses the hierarchies' streams; a system can be left out."""
    two = systems[1:]
    zs = [empty(s.b.shape) for s in two]
    for _ in range(2):
        for z in zs:
            z.zero_()
        rc, st = dd.solve_many([s.H for s in two], [dev(s.b) for s in two], zs)
        assert rc == dd.OK
    for s, z in zip(two, zs):
        assert norm(s.b[0] - s.op.apply(host(z)[0])) / norm(s.b[0]) <= 1e-10


def test_many_argument_checks(dd, systems):
    s = systems[0]
    b, z = dev(s.b), empty(s.b.shape)
    with pytest.raises(dd.DDAMGError) as e:
        dd.solve_many([s.H, s.H], [b, b], [z, z], nrhs=[2, 2])
    assert e.value.status == dd.EINVAL
    with pytest.raises(dd.DDAMGError) as e:
        dd.solve_many([s.H], [b], [b], nrhs=[2])
    assert e.value.status == dd.EINVAL
