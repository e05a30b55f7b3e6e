"""The 32^3x64 three-level workload at its full size (FP32 preconditioner
on FP16-stored operators, FP64 outer FGMRES, as the 12-source bench runs
it), on two Gaussian right-hand sides: both reach the FP64 residual bound,
and the residual recomputed by the oracle's site-by-site operator on 64
sampled sites is of the same size (the whole-lattice oracle is too slow at
2.1 M sites)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.dirac import apply_at_sites
from tests.gpu_util import dev, empty, host, say, to_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


def test_full_size_32x64_solve_sampled_residual(dd):
    cfg = W.CONFIGS["clover32x64_3lvl_12rhs"]
    dims = cfg["dims"]
    say(f"full-size solve {dims}: inputs")
    U = W.links(dims, cfg["eps"], cfg["seed_links"])
    ctx = dd.create(dims, cfg["m0"], cfg["csw"], dev(U))
    tv = torch.from_numpy(W.test_vectors(dims, 12, cfg["ntv"][0], cfg["seed_tv"])).to("cuda")
    say("  setup")
    H = dd.build_hierarchy(ctx, to_params(dd, cfg, dd.F32, half=True), tv)
    del tv
    b = W.gaussian_spinor(dims, cfg["seed_rhs"], nrhs=2)
    z = empty(b.shape)
    say("  solve")
    rc, st = dd.solve(H, dev(b), z, nrhs=2)
    say(f"  rc={rc} its {[x['outer_iters'] for x in st]} relres {[x['true_relres'] for x in st]}")
    assert rc == dd.OK
    zz = host(z)
    rng = np.random.Generator(np.random.PCG64(77))
    sites = [tuple(int(rng.integers(0, e)) for e in dims) for _ in range(64)]
    for r in range(2):
        assert st[r]["true_relres"] <= 1e-10
        dz = apply_at_sites(U, cfg["m0"], cfg["csw"], zz[r], sites)
        bs = np.array([b[r, t, zc, y, x] for (x, y, zc, t) in sites])
        res = np.sqrt(np.mean(np.abs(bs - dz) ** 2)) / np.sqrt(np.mean(np.abs(b[r]) ** 2))
        say(f"  rhs {r}: sampled residual / rms(b) = {res:.2e}")
        assert res <= 1e-9
