"""Pins of the oracle's multilevel method: two-level error propagator
(Sec. 1), cycles (Alg. 1, Alg. 2), setup invariants (Alg. 3, Alg. 4) and the
outer solve to relative residual 1e-10 (Tab. 1) against dense solves and the
known-solution error protocol of Sec. 3.4."""
import numpy as np
import pytest

import workloads as W
from oracle import multigrid as mg
from oracle.dirac import WilsonClover
from oracle.krylov import norm
from oracle.lattice import shape
from oracle.stencil import dense_matrix, gamma5_coarse


def _params(**kw):
    p = dict(W.DEFAULT_PARAMS)
    p.update(kw)
    return p


def _hier(dims, agg, ntv, levels, seed, n_inv=1, nu=2, csw=1.0, m0=-0.2, **kw):
    op = WilsonClover(W.links(dims, 0.5, seed), m0, csw)
    p = _params(levels=levels, agg=agg, ntv=ntv, n_inv=n_inv, nu=nu, **kw)
    tv = W.test_vectors(dims, 12, ntv[0], seed + 1)
    return mg.build_hierarchy(op, p, tv), op


@pytest.fixture(scope="module")
def two_level():
    return _hier((4, 4, 4, 4), [(2, 2, 2, 2)], [4], 2, 401, coarse_eps=1e-13,
                 coarse_restart=60, coarse_max_restarts=20)


def _dense_P(agg):
    from tests.test_oracle_transfer import _dense_P as dp
    return dp(agg)


def test_galerkin_orthogonality_after_exact_coarse_correction(two_level, rng):
    H, op = two_level
    H.p["nu"] = 0
    b = rng.standard_normal(shape(op.dims) + (12,)) + 0j
    z = H.cycle(0, b)
    H.p["nu"] = 2
    res = H.aggs[0].restrict(b - op.apply(z))
    assert norm(res) <= 1e-11 * norm(b)


def test_coarse_correction_is_a_projection(two_level):
    H, op = two_level
    P = _dense_P(H.aggs[0])
    D = dense_matrix(op)
    Dc = P.conj().T @ D @ P
    E = np.eye(D.shape[0]) - P @ np.linalg.solve(Dc, P.conj().T @ D)
    assert np.allclose(E @ E, E, atol=1e-10)
    assert np.allclose(dense_matrix(H.ops[1]), Dc, atol=1e-12)


def test_setup_invariants(two_level):
    H, _ = two_level
    P = _dense_P(H.aggs[0])
    assert np.allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-13)
    Dc = H.ops[1]
    g5 = gamma5_coarse(Dc.d)
    M = dense_matrix(Dc)
    G = np.kron(np.eye(int(np.prod(Dc.dims))), g5)
    assert np.allclose(M @ G, G @ M.conj().T, atol=1e-12)
    # test vectors are normalised by the iterative phase (Alg. 4)
    for v in H.tv[0]:
        assert abs(norm(v) - 1) < 1e-12


def test_two_level_solve_matches_dense(two_level, rng):
    H, op = two_level
    b = rng.standard_normal(shape(op.dims) + (12,)) + 1j * rng.standard_normal(shape(op.dims) + (12,))
    st = {}
    x = mg.solve(H, b, stats=st)
    assert st["true_relres"] <= 1e-10
    ref = np.linalg.solve(dense_matrix(op), b.reshape(-1))
    assert np.linalg.norm(x.reshape(-1) - ref) <= 1e-8 * np.linalg.norm(ref)


@pytest.fixture(scope="module")
def three_level():
    return _hier((8, 8, 8, 8), [(2, 2, 2, 2), (2, 2, 2, 2)], [4, 4], 3, 501, n_inv=1,
                 m0=-0.3)


@pytest.mark.parametrize("cycle", ["K", "V", "W"])
def test_three_level_solve_known_solution(three_level, cycle):
    """b = D z* for a Gaussian z*; report ||z - z*|| / ||z*|| (Sec. 3.4)."""
    H, op = three_level
    H.cycle_type = cycle
    zstar = W.gaussian_spinor(op.dims, 502)
    b = op.apply(zstar)
    st = {}
    z = mg.solve(H, b, stats=st)
    H.cycle_type = "K"
    assert st["true_relres"] <= 1e-10
    assert norm(z - zstar) / norm(zstar) < 1e-8
    if cycle == "K":
        assert st["kcycle_iters"] > 0
    assert st["coarsest_iters"] > 0


def test_per_level_sap_blocks(rng):
    """The per-level block shape reaches the smoother of its level and only
    that one: the level-1 smoother with 1^4 blocks is block Jacobi over
    sites (one red-black sweep of single-site MR solves), checked by hand on
    the dense coarse operator; the fine level keeps 2^4 blocks."""
    from oracle.sap import sap_sweep
    dims = (8, 8, 8, 8)
    op = WilsonClover(W.links(dims, 0.5, 77), -0.2, 1.0)
    tv = W.test_vectors(dims, 12, 4, 78)
    base = _params(levels=3, agg=[(4, 4, 4, 4), (1, 1, 1, 1)], ntv=[4, 4], n_inv=0, nu=1)
    # 2^4 blocks on the 2^4 coarse level come one per direction: rejected
    with pytest.raises(ValueError):
        mg.build_hierarchy(op, base, tv)
    H1 = mg.build_hierarchy(op, dict(base, sap_blocks=[(2, 2, 2, 2), (1, 1, 1, 1)]), tv)
    assert H1.blocks == [(2, 2, 2, 2), (1, 1, 1, 1)]
    Dc = H1.ops[1]
    shp = shape(Dc.dims) + (Dc.d,)
    b = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    z = H1.smooth(1, b, np.zeros_like(b), 1)
    assert np.allclose(z, sap_sweep(Dc, b, np.zeros_like(b), (1, 1, 1, 1), base["mr_iters"]))
    # by hand: red sites then black sites, each a 3-step MR on its self block
    M = dense_matrix(Dc)
    n, d = M.shape[0], Dc.d
    V = n // d
    coords = [np.unravel_index(s, shape(Dc.dims))[::-1] for s in range(V)]
    colour = np.array([sum(c) % 2 for c in coords])
    zz = np.zeros(n, complex)
    bb = b.reshape(-1)
    for col in (0, 1):
        r = bb - M @ zz
        for s in np.nonzero(colour == col)[0]:
            sl = slice(s * d, (s + 1) * d)
            A = M[sl, sl]
            x = np.zeros(d, complex)
            rho = r[sl].copy()
            for _ in range(base["mr_iters"]):
                q = A @ rho
                a = np.vdot(q, rho) / np.vdot(q, q)
                x += a * rho
                rho -= a * q
            zz[sl] += x
    assert np.allclose(z.reshape(-1), zz, atol=1e-12)
    # the fine level keeps its 2^4 blocks
    f = W.gaussian_spinor(dims, 79)
    assert np.array_equal(H1.smooth(0, f, np.zeros_like(f), 1),
                          sap_sweep(op, f, np.zeros_like(f), (2, 2, 2, 2), base["mr_iters"]))


def test_w_cycle_equals_v_cycle_for_exact_coarse_correction(rng):
    """Without smoothing on level 1 and with an exact coarsest solve, the
    level-1 cycle is P (P^H D_1 P)^-1 P^H, whose second application to the
    residual of the first adds nothing (Galerkin orthogonality): the W-cycle
    then equals the V-cycle.  With smoothing the two differ."""
    H, op = _hier((8, 8, 8, 8), [(2, 2, 2, 2), (2, 2, 2, 2)], [4, 4], 3, 601, n_inv=1, m0=-0.3,
                  coarse_eps=1e-14, coarse_restart=60, coarse_max_restarts=20)
    b = W.gaussian_spinor(op.dims, 602)
    H.p["mu"] = 0
    H.p["nu"] = 0
    H.cycle_type = "V"
    zv = H.cycle(0, b)
    H.cycle_type = "W"
    zw = H.cycle(0, b)
    assert norm(zw - zv) <= 1e-10 * norm(zv)
    H.p["nu"] = 2
    H.cycle_type = "V"
    zv = H.cycle(0, b)
    H.cycle_type = "W"
    zw = H.cycle(0, b)
    assert norm(zw - zv) > 1e-6 * norm(zv)
