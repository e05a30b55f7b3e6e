"""Pins of the oracle's FGMRES / GMRES and the odd-even coarsest solve
against numpy's dense solver."""
import numpy as np

import workloads as W
from oracle.aggregation import Aggregation
from oracle.dirac import WilsonClover
from oracle.galerkin import galerkin
from oracle.krylov import OddEvenCoarsest, cgnr, fgmres
from oracle.lattice import parity, shape
from oracle.stencil import dense_matrix


def _rand(rng, shp):
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def test_gmres_dense(rng):
    n = 60
    A = np.eye(n) * 4 + 0.3 * _rand(rng, (n, n))
    b = _rand(rng, n)
    x = fgmres(lambda v: A @ v, b, None, 10, 50, 1e-12, check_true_residual=True)
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-10)


def test_fgmres_exact_preconditioner_one_step(rng):
    n = 40
    A = np.eye(n) * 3 + _rand(rng, (n, n))
    Ainv = np.linalg.inv(A)
    b = _rand(rng, n)
    st = {}
    x = fgmres(lambda v: A @ v, b, lambda v: Ainv @ v, 5, 2, 1e-12, stats=st)
    assert st["iters"] == 1
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-11)


def test_fgmres_variable_preconditioner(rng):
    """A preconditioner that changes from call to call (the flexible case)."""
    n = 50
    A = np.eye(n) * 3 + 0.5 * _rand(rng, (n, n))
    Ainv = np.linalg.inv(A)
    b = _rand(rng, n)
    calls = [0]

    def M(v):
        calls[0] += 1
        return Ainv @ v + 1e-2 * calls[0] * v
    x = fgmres(lambda v: A @ v, b, M, 10, 20, 1e-12, check_true_residual=True)
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_gmres_tolerance_is_relative(rng):
    n = 80
    A = np.eye(n) * 2 + 0.4 / np.sqrt(n) * _rand(rng, (n, n))
    b = _rand(rng, n)
    for tol in (1e-1, 5e-2, 1e-3):
        x = fgmres(lambda v: A @ v, b, None, 30, 10, tol)
        assert np.linalg.norm(b - A @ x) <= tol * np.linalg.norm(b) * (1 + 1e-12)


def _coarse_op(rng):
    dims = (4, 4, 4, 4)
    op = WilsonClover(W.links(dims, 0.5, 301), -0.2, 1.0)
    tv = _rand(rng, (4,) + shape(dims) + (12,))
    agg = Aggregation(dims, (2, 2, 2, 2), tv)
    return galerkin(op, agg)


def test_odd_even_solution_matches_dense(rng):
    Dc = _coarse_op(rng)
    cs = OddEvenCoarsest(Dc, 1e-13, restart=40, max_restarts=20)
    b = _rand(rng, shape(Dc.dims) + (Dc.d,))
    x = cs.solve(b)
    ref = np.linalg.solve(dense_matrix(Dc), b.reshape(-1))
    assert np.allclose(x.reshape(-1), ref, atol=1e-10)


def test_odd_even_schur_identity(rng):
    """The Schur operator equals D_oo - D_oe D_ee^-1 D_eo from the dense matrix."""
    Dc = _coarse_op(rng)
    cs = OddEvenCoarsest(Dc, 5e-2)
    M = dense_matrix(Dc)
    p = np.repeat(parity(Dc.dims).reshape(-1), Dc.d)
    e, o = np.nonzero(p == 0)[0], np.nonzero(p == 1)[0]
    S = M[np.ix_(o, o)] - M[np.ix_(o, e)] @ np.linalg.solve(M[np.ix_(e, e)], M[np.ix_(e, o)])
    v = _rand(rng, shape(Dc.dims) + (Dc.d,))
    v = np.where((parity(Dc.dims) == 1)[..., None], v, 0)
    assert np.allclose(cs.schur(v).reshape(-1)[o], S @ v.reshape(-1)[o], atol=1e-12)
    # hops join even and odd sites only: D_ee couples each even site to itself
    site = np.repeat(np.arange(int(np.prod(Dc.dims))), Dc.d)
    Mee = M[np.ix_(e, e)]
    assert np.all(Mee[site[e][:, None] != site[e][None, :]] == 0)
    inv = np.linalg.inv(Dc.S)
    assert np.allclose(inv @ Dc.S, np.eye(Dc.d), atol=1e-12)


def test_odd_even_reaches_eps(rng):
    Dc = _coarse_op(rng)
    cs = OddEvenCoarsest(Dc, 5e-2)
    b = _rand(rng, shape(Dc.dims) + (Dc.d,))
    x = cs.solve(b)
    # the Schur residual reached eps; the full residual is of the same order
    assert np.linalg.norm(b - Dc.apply(x)) <= 0.5 * np.linalg.norm(b)


def test_cgnr_scaled_unitary_one_step(rng):
    """A = c Q with Q unitary: A^H A = |c|^2 I, so CG on the normal equations
    ends after one step with the exact solution."""
    n = 30
    Q, _ = np.linalg.qr(_rand(rng, (n, n)))
    A = (2.0 - 0.5j) * Q
    b = _rand(rng, n)
    st = {}
    x = cgnr(lambda v: A @ v, lambda v: A.conj().T @ v, b, 1e-12, 50, stats=st)
    assert st["iters"] == 1
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-12)


def test_cgnr_dense_and_monotone(rng):
    """CGNR minimises ||b - A x|| over the growing Krylov space of A^H A:
    the residual never increases, and the result is numpy's solution."""
    n = 50
    A = np.eye(n) * 2 + 0.4 * _rand(rng, (n, n)) / np.sqrt(n)
    b = _rand(rng, n)
    st = {}
    x = cgnr(lambda v: A @ v, lambda v: A.conj().T @ v, b, 1e-11, 500, stats=st)
    h = np.array(st["history"])
    assert st["converged"]
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-12))
    assert np.linalg.norm(b - A @ x) <= 1e-11 * np.linalg.norm(b)
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-9)


def test_cgnr_finite_termination(rng):
    """In exact arithmetic CG on an n x n system ends within n steps."""
    n = 12
    A = np.diag(np.linspace(1.0, 3.0, n)) + 0.2 * _rand(rng, (n, n))
    b = _rand(rng, n)
    st = {}
    cgnr(lambda v: A @ v, lambda v: A.conj().T @ v, b, 1e-10, 200, stats=st)
    assert st["converged"] and st["iters"] <= n + 3


def test_cgnr_wilson_clover_gamma5_adjoint(rng):
    """On a 2^4 clover lattice: D^H applied as Gamma5 D Gamma5 gives the same
    CGNR iterates as the dense conjugate transpose, and the solution of the
    dense system."""
    dims = (2, 2, 2, 2)
    op = WilsonClover(W.links(dims, 0.5, 77), -0.2, 1.0)
    M = dense_matrix(op)
    b = W.gaussian_spinor(dims, 78)
    s1, s2 = {}, {}
    x1 = cgnr(op.apply, op.apply_dagger, b, 1e-10, 2000, stats=s1)
    x2 = cgnr(lambda v: (M @ v.reshape(-1)).reshape(v.shape),
              lambda v: (M.conj().T @ v.reshape(-1)).reshape(v.shape), b, 1e-10, 2000, stats=s2)
    assert s1["iters"] == s2["iters"]
    assert np.allclose(x1, x2, atol=1e-11)
    ref = np.linalg.solve(M, b.reshape(-1)).reshape(b.shape)
    assert np.linalg.norm(x1 - ref) <= 1e-8 * np.linalg.norm(ref)
