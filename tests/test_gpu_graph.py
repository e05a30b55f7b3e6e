"""The graph-captured preconditioner (params.graph = 1): the coarsest GMRES
with its scalars on the device gives the host-driven solve's iteration
counts and solution up to rounding; graph replays give identical results
call after call; batches of different sizes (new captures after the
buffers grow) and concurrent solves on several hierarchies each capture
their own graph; parameter checks."""
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


class Pair:
    """Two hierarchies from the same links and test vectors, one solving
    host-driven, the other with the graph-captured preconditioner."""

    def __init__(self, dd, dims, p, eps, m0, csw, seed, cycle):
        say(f"pair dims={dims} levels={p['levels']} cycle={cycle}")
        self.dims = dims
        U = W.links(dims, eps, seed)
        self.op = WilsonClover(U, m0, csw)
        self.ctx = dd.create(dims, m0, csw, dev(U))
        tv = dev(W.test_vectors(dims, 12, p["ntv"][0], seed + 1))
        P0 = to_params(dd, p, dd.F32, cycle=cycle)
        P1 = to_params(dd, p, dd.F32, cycle=cycle)
        P1.graph = 1
        self.Hh = dd.build_hierarchy(self.ctx, P0, tv)
        self.Hg = dd.build_hierarchy(self.ctx, P1, tv)
        self.b = W.gaussian_spinor(dims, seed + 2, nrhs=3)
        torch.cuda.synchronize()

    def solve(self, dd, H, nrhs=1):
        z = empty(self.b[:nrhs].shape)
        rc, st = dd.solve(H, dev(self.b[:nrhs]), z, nrhs=nrhs)
        assert rc == dd.OK
        return host(z), st


COARSE = dict(coarse_restart=16, coarse_max_restarts=2)


@pytest.fixture(scope="module")
def three(dd):
    return Pair(dd, (16, 16, 16, 16), _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [8, 8], **COARSE), 0.5, -0.3, 1.0,
                61, "V")


@pytest.fixture(scope="module")
def two(dd):
    return Pair(dd, (8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [8], **COARSE), 0.4, -0.3, 0.0, 71, "K")


@pytest.mark.parametrize("which", ["three", "two"])
def test_graph_matches_host_driven(dd, which, request):
    P = request.getfixturevalue(which)
    zh, sh = P.solve(dd, P.Hh)
    zg, sg = P.solve(dd, P.Hg)
    say(f"  {which}: host its {sh[0]['outer_iters']} coarsest {sh[0]['coarsest_iters']}, "
        f"graph its {sg[0]['outer_iters']} coarsest {sg[0]['coarsest_iters']}, rel. diff {relerr(zg, zh):.1e}")
    assert sg[0]["outer_iters"] == sh[0]["outer_iters"]
    assert abs(sg[0]["coarsest_iters"] - sh[0]["coarsest_iters"]) <= 2
    assert relerr(zg, zh) <= 1e-8
    for z in (zh, zg):
        assert norm(P.b[0] - P.op.apply(z[0])) / norm(P.b[0]) <= 1e-10


def test_graph_replays_identical(dd, three):
    z1, s1 = three.solve(dd, three.Hg)
    z2, s2 = three.solve(dd, three.Hg)
    z3, s3 = three.solve(dd, three.Hg)
    assert np.array_equal(z1, z2) and np.array_equal(z1, z3)
    assert s1[0]["outer_iters"] == s2[0]["outer_iters"] == s3[0]["outer_iters"]
    assert s1[0]["coarsest_iters"] == s2[0]["coarsest_iters"] == s3[0]["coarsest_iters"]


def test_graph_batch_sizes(dd, three):
    """1, 3, then 1 right-hand sides: the batch of 3 grows the buffers (the
    graph for 1 is captured again afterwards); each system of the batch gets
    the iterations it gets alone."""
    z1, s1 = three.solve(dd, three.Hg, 1)
    z3, s3 = three.solve(dd, three.Hg, 3)
    z1b, s1b = three.solve(dd, three.Hg, 1)
    say(f"  batch of 3: its {[x['outer_iters'] for x in s3]}")
    assert relerr(z3[0], z1[0]) <= 1e-8
    assert np.array_equal(z1, z1b)
    for r in range(3):
        assert norm(three.b[r] - three.op.apply(z3[r])) / norm(three.b[r]) <= 1e-10
    assert s3[0]["outer_iters"] == s1[0]["outer_iters"]


def test_graph_concurrent(dd, three, two):
    zs = [empty(three.b[:1].shape), empty(two.b[:1].shape)]
    rc, st = dd.solve_many([three.Hg, two.Hg], [dev(three.b[:1]), dev(two.b[:1])], zs)
    assert rc == dd.OK
    for P, z in zip((three, two), zs):
        zz = host(z)
        assert norm(P.b[0] - P.op.apply(zz[0])) / norm(P.b[0]) <= 1e-10


def test_graph_needs_vcycle(dd, three):
    p = _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [8, 8], **COARSE)
    P = to_params(dd, p, dd.F32, cycle="K")
    P.graph = 1
    with pytest.raises(dd.DDAMGError) as e:
        dd.build_hierarchy(three.ctx, P, dev(W.test_vectors(three.dims, 12, 8, 5)))
    assert e.value.status == dd.EINVAL
