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


@pytest.mark.parametrize("cycle", ["K", "V"])
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
