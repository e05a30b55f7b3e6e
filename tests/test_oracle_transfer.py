"""Pins of the oracle's aggregation P, Galerkin D_c = P^H D P and its
gamma5-symmetry (Sec. 1) against dense brute force."""
import numpy as np
import pytest

import workloads as W
from oracle.aggregation import Aggregation, mgs2
from oracle.dirac import WilsonClover
from oracle.galerkin import galerkin
from oracle.lattice import shape, shift
from oracle.stencil import dense_matrix, gamma5_coarse

DIMS = (4, 4, 4, 4)
AGG = (2, 2, 2, 2)


def _rand(rng, shp):
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def _setup(rng, N=4, csw=1.0):
    op = WilsonClover(W.links(DIMS, 0.5, 201), -0.3, csw)
    tv = _rand(rng, (N,) + shape(DIMS) + (12,))
    return op, Aggregation(DIMS, AGG, tv), tv


def _dense_P(agg):
    n = int(np.prod(shape(agg.dims))) * agg.d
    nc = int(np.prod(shape(agg.cdims))) * 2 * agg.N
    P = np.zeros((n, nc), complex)
    e = np.zeros(nc, complex)
    for j in range(nc):
        e[j] = 1
        P[:, j] = agg.prolong(e.reshape(shape(agg.cdims) + (2 * agg.N,))).reshape(-1)
        e[j] = 0
    return P


def test_mgs2_matches_qr(rng):
    A = _rand(rng, (3, 40, 6))
    Q = mgs2(A)
    for k in range(3):
        assert np.allclose(Q[k].conj().T @ Q[k], np.eye(6), atol=1e-14)
        Qr, _ = np.linalg.qr(A[k])
        assert np.allclose(Q[k] @ Q[k].conj().T, Qr @ Qr.conj().T, atol=1e-13)
        # index order: column k lies in the span of the first k+1 inputs
        for j in range(6):
            c = np.linalg.lstsq(A[k][:, :j + 1], Q[k][:, j], rcond=None)[0]
            assert np.allclose(A[k][:, :j + 1] @ c, Q[k][:, j], atol=1e-12)


def test_P_orthonormal_and_reproduces_test_vectors(rng):
    op, agg, tv = _setup(rng)
    P = _dense_P(agg)
    assert np.allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-13)
    for v in tv:
        assert np.allclose(agg.prolong(agg.restrict(v)), v, atol=1e-12)
    x = _rand(rng, shape(DIMS) + (12,))
    y = _rand(rng, shape(agg.cdims) + (2 * agg.N,))
    assert np.isclose(np.vdot(agg.restrict(x), y), np.vdot(x, agg.prolong(y)), atol=1e-12)


def test_P_preserves_chirality(rng):
    _, agg, _ = _setup(rng)
    P = _dense_P(agg)
    g5f = np.kron(np.eye(int(np.prod(DIMS))), np.diag([1] * 6 + [-1] * 6))
    g5c = np.kron(np.eye(int(np.prod(agg.cdims))), gamma5_coarse(2 * agg.N))
    assert np.allclose(g5f @ P, P @ g5c, atol=1e-14)


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_galerkin_equals_dense_PHDP(rng, csw):
    op, agg, _ = _setup(rng, csw=csw)
    Dc = galerkin(op, agg)
    P = _dense_P(agg)
    ref = P.conj().T @ dense_matrix(op) @ P
    assert np.allclose(dense_matrix(Dc), ref, atol=1e-12)


def test_coarse_gamma5_symmetry(rng):
    op, agg, _ = _setup(rng)
    Dc = galerkin(op, agg)
    g5 = gamma5_coarse(Dc.d)
    M = dense_matrix(Dc)
    G = np.kron(np.eye(int(np.prod(agg.cdims))), g5)
    assert np.allclose(M @ G, G @ M.conj().T, atol=1e-12)
    # blockwise: B_mu(x) = G5 F_mu(x - mu)^H G5, and the self block is G5-Hermitian
    for mu in range(4):
        Fm = shift(Dc.F[mu], mu, -1)
        assert np.allclose(Dc.B[mu], g5 @ np.conj(np.swapaxes(Fm, -1, -2)) @ g5, atol=1e-12)
    S = Dc.S
    assert np.allclose(g5 @ S @ g5, np.conj(np.swapaxes(S, -1, -2)), atol=1e-12)


def test_second_level_galerkin_dense(rng):
    """Galerkin of a coarse stencil (level 2 -> 3) against dense brute force."""
    op, agg, _ = _setup(rng)
    Dc = galerkin(op, agg)
    agg2_shape = (2, 1, 1, 2)
    tv2 = _rand(rng, (3,) + shape(agg.cdims) + (Dc.d,))
    agg2 = Aggregation(agg.cdims, agg2_shape, tv2)
    Dcc = galerkin(Dc, agg2)
    P2 = _dense_P(agg2)
    assert np.allclose(dense_matrix(Dcc), P2.conj().T @ dense_matrix(Dc) @ P2, atol=1e-12)
