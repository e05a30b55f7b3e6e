"""ddamg_solve_batch: the outer FGMRES of several hierarchies with its
scalars on the device, one HIP graph per outer step over all of them, and
per-system device convergence flags.  Each system's result is the one the
host-driven solve of the same hierarchy gives (the same arithmetic: equal
iteration counts, solutions within the solve tolerance), certified by the
oracle's FP64 operator."""
import numpy as np
import pytest

import workloads as W
from oracle.dirac import WilsonClover
from oracle.krylov import norm
from tests.gpu_util import dev, empty, host, relerr, say, to_params
from tests.test_gpu_hierarchy import _p

pytestmark = pytest.mark.gpu

# the coarsest GMRES of a captured V-cycle: restart length and cycles
COARSE = (8, 1)


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


def _graph_params(dd, p, cycle="V"):
    P = to_params(dd, p, dd.F32, cycle=cycle)
    P.graph = 1
    P.coarse_restart, P.coarse_max_restarts = COARSE
    return P


@pytest.fixture(scope="module")
def systems(dd):
    """Three lattices of different sizes and masses, two and three levels."""
    specs = [((8, 8, 8, 8), _p(2, [(4, 4, 4, 4)], [4]), -0.30, 0.45, 301, "K"),
             ((16, 16, 16, 16), _p(3, [(4, 4, 4, 4), (2, 2, 2, 2)], [4, 4]), -0.25, 0.5, 302, "V"),
             ((8, 8, 8, 16), _p(2, [(4, 4, 4, 4)], [4]), -0.35, 0.4, 303, "K")]
    out = []
    for dims, p, m0, eps, seed, cyc in specs:
        U = W.links(dims, eps, seed)
        op = WilsonClover(U, m0, 1.0)
        ctx = dd.create(dims, m0, 1.0, dev(U))
        tv = W.test_vectors(dims, 12, p["ntv"][0], seed + 1)
        H = dd.build_hierarchy(ctx, _graph_params(dd, p, cyc), dev(tv))
        zstar = W.gaussian_spinor(dims, seed + 2)
        b = op.apply(zstar)
        out.append(dict(dims=dims, op=op, ctx=ctx, H=H, b=b, zstar=zstar))
    return out


def test_batch_matches_host_driven_and_oracle(dd, systems):
    hs = [s["H"] for s in systems]
    bs = [dev(s["b"]) for s in systems]
    zs = [empty(s["b"].shape) for s in systems]
    for z in zs:
        z.zero_()
    rc, st = dd.solve_batch(hs, bs, zs)
    say(f"  solve_batch rc={rc} its={[x['outer_iters'] for x in st]} restarts={[x['restarts'] for x in st]}")
    assert rc == dd.OK
    for s, z, x in zip(systems, zs, st):
        zz = host(z)
        res = norm(s["b"] - s["op"].apply(zz)) / norm(s["b"])
        err = relerr(zz, s["zstar"])
        say(f"  {s['dims']}: oracle relres {res:.2e}, error {err:.2e}")
        assert x["status"] == dd.OK and x["true_relres"] <= 1e-10
        assert res <= 1e-10 * 1.01 and err < 1e-8
        # the host-driven solve of the same hierarchy
        z1 = empty(s["b"].shape)
        z1.zero_()
        rc1, st1 = dd.solve(s["H"], dev(s["b"]), z1)
        assert rc1 == dd.OK
        assert abs(st1[0]["outer_iters"] - x["outer_iters"]) <= 1
        assert relerr(host(z1), zz) < 1e-8
    # again with the kept graphs: the same results
    zs2 = [empty(s["b"].shape) for s in systems]
    for z in zs2:
        z.zero_()
    rc2, st2 = dd.solve_batch(hs, bs, zs2)
    assert rc2 == dd.OK
    assert [x["outer_iters"] for x in st2] == [x["outer_iters"] for x in st]
    for z, z2 in zip(zs, zs2):
        assert np.array_equal(host(z), host(z2))


def test_batch_initial_guess_and_converged_system(dd, systems):
    """A system whose initial guess already solves it stays at rest (zero
    iterations) while the others iterate."""
    hs = [s["H"] for s in systems]
    bs = [dev(s["b"]) for s in systems]
    zs = [empty(s["b"].shape) for s in systems]
    for z in zs:
        z.zero_()
    zs[1] = dev(systems[1]["zstar"])
    rc, st = dd.solve_batch(hs, bs, zs)
    assert rc == dd.OK
    assert st[1]["outer_iters"] == 0 and st[0]["outer_iters"] > 0 and st[2]["outer_iters"] > 0
    assert relerr(host(zs[1]), systems[1]["zstar"]) < 1e-12


def test_batch_validation(dd, systems):
    s = systems[0]
    H_host = dd.build_hierarchy(s["ctx"], to_params(dd, _p(2, [(4, 4, 4, 4)], [4]), dd.F32),
                                dev(W.test_vectors(s["dims"], 12, 4, 311)))
    b = dev(s["b"])
    with pytest.raises(dd.DDAMGError) as e:
        dd.solve_batch([systems[1]["H"], H_host], [dev(systems[1]["b"]), b],
                       [empty(systems[1]["b"].shape), empty(s["b"].shape)])
    assert e.value.status == dd.EINVAL and "graph" in str(e.value)
    with pytest.raises(dd.DDAMGError) as e:
        dd.solve_batch([s["H"], s["H"]], [b, b], [empty(s["b"].shape), empty(s["b"].shape)])
    assert e.value.status == dd.EINVAL and "twice" in str(e.value)
