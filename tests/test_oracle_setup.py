"""Dense brute-force pins of the oracle's setup phases (Alg. 3, Alg. 4, Fig. 1)
and of the composition of the multilevel cycles on three levels (Alg. 1 and
Alg. 2, with the W-cycle variant).

With exact block inverses in place of the MR block solves, one SAP step
z <- z + M (b - D z) is linear, with error propagator
E = (I - sum_black I_j D_j^-1 I_j^T D)(I - sum_red I_i D_i^-1 I_i^T D)
(multiplicative Schwarz over the two colours, Sec. 2), so n steps from z
give E^n z + (I - E^n) D^-1 b.  With an exact coarsest solve and a K-cycle
run to a tight tolerance, every step of the setup and of the cycles then has
a closed form in dense matrices: the coarse correction P D_c^-1 P^H, the
level solves D_l^-1, and the interpolation, rebuilt here by a QR
factorisation per (aggregate, chirality) whose Q with positive diagonal R is
the unique orthonormalisation in index order (Sec. 1: P keeps the two
chiralities apart).  None of the oracle's stencil, SAP, aggregation or
Krylov code is used for the expected values; only dense_matrix() reads the
operators, and it is pinned by the dense-operator tests of the fine stencil.

Lattice: 4^4 fine, aggregates 2^4 then 1^4 (levels 4^4 x 12, 2^4 x 8,
2^4 x 6), SAP blocks 2^4 on the fine level and 1^4 on level 1.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import multigrid as mg
from oracle.dirac import WilsonClover
from oracle.lattice import block_colour, coords, shape
from oracle.stencil import dense_matrix

DIMS = (4, 4, 4, 4)
AGG = [(2, 2, 2, 2), (1, 1, 1, 1)]
BLOCKS = [(2, 2, 2, 2), (1, 1, 1, 1)]


# ---------------------------------------------------------------------------
# dense helpers (independent of the oracle's sparse code)
# ---------------------------------------------------------------------------
def _block_ids(dims, block):
    c = coords(dims) // np.asarray(block)
    nb = [d // b for d, b in zip(dims, block)]
    return (c[..., 0] + nb[0] * (c[..., 1] + nb[1] * (c[..., 2] + nb[2] * c[..., 3]))).reshape(-1)


class DenseLevel:
    """Dense operator of one level with its exact-block SAP."""

    def __init__(self, M, dims, d, block):
        self.M = M
        self.dims = tuple(dims)
        self.d = d
        self.n = M.shape[0]
        self.lu = sla.lu_factor(M)
        bid = np.repeat(_block_ids(dims, block), d)
        self.Binv = np.zeros_like(M)
        for i in np.unique(bid):
            idx = np.nonzero(bid == i)[0]
            self.Binv[np.ix_(idx, idx)] = np.linalg.inv(M[np.ix_(idx, idx)])
        col = np.repeat(block_colour(dims, block).reshape(-1), d)
        self.red = (col == 0).astype(float)
        self.black = (col == 1).astype(float)

    def solve(self, b):
        return sla.lu_solve(self.lu, b)

    def E(self, v):
        """SAP error propagator (red blocks first, then black)."""
        v = v - self.red * (self.Binv @ (self.red * (self.M @ v)))
        return v - self.black * (self.Binv @ (self.black * (self.M @ v)))

    def smooth(self, b, z, n):
        """n SAP steps from z: E^n z + (I - E^n) D^-1 b."""
        x = self.solve(b)
        e = z - x
        for _ in range(n):
            e = self.E(e)
        return x + e


def _dense_P(dims, agg, vecs, d):
    """Interpolation from test vectors vecs (N, n) in the dense ordering:
    per (aggregate, chirality) the Q of a QR factorisation with positive
    diagonal R; coarse index = coarse site * 2N + chirality * N + k."""
    N = vecs.shape[0]
    site_agg = _block_ids(dims, agg)
    nagg = int(site_agg.max()) + 1
    V = len(site_agg)
    P = np.zeros((V * d, nagg * 2 * N), dtype=np.complex128)
    for a in range(nagg):
        sites = np.nonzero(site_agg == a)[0]
        for s in range(2):
            rows = (sites[:, None] * d + s * (d // 2) + np.arange(d // 2)[None, :]).reshape(-1)
            Q, R = np.linalg.qr(vecs[:, rows].T)
            ph = np.diag(R) / np.abs(np.diag(R))
            Q = Q * ph[None, :]
            P[np.ix_(rows, a * 2 * N + s * N + np.arange(N))] = Q
    return P


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a).reshape(-1) - np.asarray(b).reshape(-1))
                 / np.linalg.norm(np.asarray(b).reshape(-1)))


def _exact_block_factory():
    cache = {}

    def factory(l, op, block):
        key = (l, id(op))
        if key not in cache:
            dl = DenseLevel(dense_matrix(op), op.dims, op.d, block)

            def solver(rc, mask):
                return (dl.Binv @ rc.reshape(-1)).reshape(rc.shape)

            cache[key] = (op, solver)     # the op is held so that its id stays unique
        return cache[key][1]

    return factory


def _params(levels, ntv, nu, **kw):
    p = dict(W.DEFAULT_PARAMS)
    p.update(levels=levels, agg=AGG[:levels - 1], ntv=ntv, nu=nu, mu=0,
             sap_blocks=BLOCKS[:levels - 1], coarse_eps=1e-14, coarse_restart=100,
             coarse_max_restarts=10, kc_tol=1e-13, kc_restarts=60)
    p.update(kw)
    return p


@pytest.fixture(scope="module")
def fine():
    op = WilsonClover(W.links(DIMS, 0.5, 7301), -0.2, 1.0)
    return op, DenseLevel(dense_matrix(op), DIMS, 12, BLOCKS[0])


def _flat(a):
    return np.asarray(a).reshape(a.shape[0], -1)


def _hier(op, p, tv0):
    H = mg.Hierarchy(op, p)
    H.block_solver_factory = _exact_block_factory()
    return H


# ---------------------------------------------------------------------------
# Alg. 3
# ---------------------------------------------------------------------------
def test_initial_setup_matches_dense_iteration(fine):
    """Alg. 3 on three levels: for eta = 1, 2, 3 each test vector is replaced
    by eta SAP steps from zero with itself as right-hand side, i.e.
    v <- (I - E^eta) D^-1 v, unnormalised; P_0 is built from the result; the
    level-1 test vectors start as P_0^H v and take the same three rounds
    with the level-1 operator P_0^H D P_0."""
    op, d0 = fine
    p = _params(3, [4, 3], 2)
    tv0 = W.test_vectors(DIMS, 12, 4, 7302)
    H = _hier(op, p, tv0)
    mg.initial_setup(H, 0, tv0)

    v = _flat(tv0).copy()
    for eta in (1, 2, 3):
        for j in range(v.shape[0]):
            v[j] = d0.smooth(v[j], np.zeros_like(v[j]), eta)
    assert _rel(_flat(H.tv[0]), v) < 1e-11
    # a single round (eta = 3 only) or normalised vectors would be far off
    assert _rel(_flat(H.tv[0]), [d0.smooth(x, 0 * x, 3) for x in _flat(tv0)]) > 1e-3

    P0 = _dense_P(DIMS, AGG[0], v, 12)
    D1 = P0.conj().T @ d0.M @ P0
    assert _rel(dense_matrix(H.ops[1]), D1) < 1e-12
    cdims = tuple(x // a for x, a in zip(DIMS, AGG[0]))
    d1 = DenseLevel(D1, cdims, 8, BLOCKS[1])
    w = np.stack([P0.conj().T @ x for x in v])[:3]
    for eta in (1, 2, 3):
        for j in range(w.shape[0]):
            w[j] = d1.smooth(w[j], np.zeros_like(w[j]), eta)
    assert _rel(_flat(H.tv[1]), w) < 1e-10
    P1 = _dense_P(cdims, AGG[1], w, 8)
    assert _rel(dense_matrix(H.ops[2]), P1.conj().T @ D1 @ P1) < 1e-10


# ---------------------------------------------------------------------------
# Alg. 4
# ---------------------------------------------------------------------------
def test_iterative_setup_two_levels_is_normalised_coarse_correction(fine):
    """Alg. 4 on two levels without smoothing and with an exact coarsest
    solve: every test vector becomes P D_c^-1 P^H v / ||P D_c^-1 P^H v||
    (the hierarchy is fixed while the vectors are updated), then P and D_c
    are rebuilt from the new vectors."""
    op, d0 = fine
    p = _params(2, [4], 0)
    tv0 = W.test_vectors(DIMS, 12, 4, 7303)
    H = _hier(op, p, tv0)
    mg.initial_setup(H, 0, tv0)
    v = _flat(H.tv[0]).copy()
    P = _dense_P(DIMS, AGG[0], v, 12)
    Dc = P.conj().T @ d0.M @ P
    mg.iterative_setup(H, 0, 1)
    exp = []
    for x in v:
        y = P @ np.linalg.solve(Dc, P.conj().T @ x)
        exp.append(y / np.linalg.norm(y))
    exp = np.stack(exp)
    assert _rel(_flat(H.tv[0]), exp) < 1e-11
    for x in _flat(H.tv[0]):
        assert abs(np.linalg.norm(x) - 1) < 1e-13
    P2 = _dense_P(DIMS, AGG[0], exp, 12)
    assert _rel(dense_matrix(H.ops[1]), P2.conj().T @ d0.M @ P2) < 1e-10


def test_iterative_setup_three_levels_matches_dense(fine):
    """Alg. 4 on three levels, iteration i = 1, with nu = 2 exact-block SAP
    steps, an exact coarsest solve and the K-cycle run to 1e-13:

    level 0, per test vector v (hierarchy fixed):
        y1 = D_1^-1 P_0^H v                       (the K-cycle's solution)
        y0 = E_0^2 P_0 y1 + (I - E_0^2) D_0^-1 v  (post-smoothing)
        v  <- y0 / ||y0||,  level-1 vector <- y1 / ||y1||   (Fig. 1: the
        current level-k solution of the cycle becomes level k's vector)
    then P_0, D_1, P_1, D_2 are rebuilt; then the level-1 phase runs once
    (i = 1 times): for each level-1 vector w,
        y2 = D_2^-1 P_1^H w,  y1 = E_1^2 P_1 y2 + (I - E_1^2) D_1^-1 w,
        w <- y1 / ||y1||."""
    op, d0 = fine
    p = _params(3, [4, 3], 2)
    tv0 = W.test_vectors(DIMS, 12, 4, 7304)
    H = _hier(op, p, tv0)
    mg.initial_setup(H, 0, tv0)
    v0 = _flat(H.tv[0]).copy()
    v1 = _flat(H.tv[1]).copy()
    cdims = tuple(x // a for x, a in zip(DIMS, AGG[0]))
    mg.iterative_setup(H, 0, 1)

    P0 = _dense_P(DIMS, AGG[0], v0, 12)
    D1 = P0.conj().T @ d0.M @ P0
    n0, n1 = [], []
    for x in v0:
        y1 = np.linalg.solve(D1, P0.conj().T @ x)
        y0 = d0.smooth(x, P0 @ y1, 2)
        n0.append(y0 / np.linalg.norm(y0))
        n1.append(y1 / np.linalg.norm(y1))
    n0 = np.stack(n0)
    n1 = np.stack(n1)[:v1.shape[0]]
    assert _rel(_flat(H.tv[0]), n0) < 1e-9

    P0 = _dense_P(DIMS, AGG[0], n0, 12)
    D1 = P0.conj().T @ d0.M @ P0
    d1 = DenseLevel(D1, cdims, 8, BLOCKS[1])
    P1 = _dense_P(cdims, AGG[1], n1, 8)
    D2 = P1.conj().T @ D1 @ P1
    n1b = []
    for w in n1:
        y2 = np.linalg.solve(D2, P1.conj().T @ w)
        y1 = d1.smooth(w, P1 @ y2, 2)
        n1b.append(y1 / np.linalg.norm(y1))
    n1b = np.stack(n1b)
    assert _rel(_flat(H.tv[1]), n1b) < 1e-9
    # the first-phase level-1 record alone (no level-1 phase) is far off
    assert _rel(_flat(H.tv[1]), n1) > 1e-3
    assert _rel(dense_matrix(H.ops[1]), D1) < 1e-9
    P1b = _dense_P(cdims, AGG[1], n1b, 8)
    assert _rel(dense_matrix(H.ops[2]), P1b.conj().T @ D1 @ P1b) < 1e-8


def test_setup_driver_order(fine, monkeypatch):
    """Reading of the setup driver (Fig. 1): the initial phase, then for
    i = 1..n_inv the iterative phase on the finest level, each of which runs
    the next level's phase for q = 1..i."""
    op, _ = fine
    calls = []
    real_init, real_iter = mg.initial_setup, mg.iterative_setup

    def rec_init(H, l, *a):
        calls.append(("init", l))
        return real_init(H, l, *a)

    def rec_iter(H, l, i):
        if l < H.L - 1:
            calls.append(("iter", l, i))
        return real_iter(H, l, i)

    monkeypatch.setattr(mg, "initial_setup", rec_init)
    monkeypatch.setattr(mg, "iterative_setup", rec_iter)
    p = _params(3, [4, 3], 1, n_inv=2, kc_tol=1e-1, kc_restarts=2)
    tv0 = W.test_vectors(DIMS, 12, 4, 7305)
    mg.build_hierarchy(op, p, tv0)
    assert calls == [("init", 0), ("init", 1),
                     ("iter", 0, 1), ("iter", 1, 1),
                     ("iter", 0, 2), ("iter", 1, 1), ("iter", 1, 2)]


# ---------------------------------------------------------------------------
# cycles on three levels
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def three(fine):
    op, d0 = fine
    p = _params(3, [4, 3], 2, n_inv=1, kc_tol=1e-1, kc_restarts=2)
    tv0 = W.test_vectors(DIMS, 12, 4, 7306)
    H = _hier(op, p, tv0)
    mg.initial_setup(H, 0, tv0)
    mg.iterative_setup(H, 0, 1)
    P0 = _dense_P(DIMS, AGG[0], _flat(H.tv[0]), 12)
    cdims = tuple(x // a for x, a in zip(DIMS, AGG[0]))
    P1 = _dense_P(cdims, AGG[1], _flat(H.tv[1]), 8)
    D1 = P0.conj().T @ d0.M @ P0
    D2 = P1.conj().T @ D1 @ P1
    d1 = DenseLevel(D1, cdims, 8, BLOCKS[1])
    return H, d0, d1, P0, P1, D2


@pytest.mark.parametrize("cycle,nu", [("V", 0), ("V", 2), ("W", 0), ("W", 2), ("K", 2)])
def test_cycle_composition_matches_dense(three, cycle, nu):
    """One level-0 cycle on three levels (mu = 0, exact block solves, exact
    coarsest solve):
      V: z_1 = S_1(c, P_1 D_2^-1 P_1^H c) with c = P_0^H b
      W: z_1 = y + S_1(c - D_1 y, P_1 D_2^-1 P_1^H (c - D_1 y))-type second
         cycle on the residual of the first, y the first
      K: z_1 = D_1^-1 c (FGMRES on level 1 run to 1e-13)
    and z = S_0(b, P_0 z_1), S_l(b, z) = nu SAP steps from z.  With nu = 0
    the V-cycle is P_0 P_1 D_2^-1 P_1^H P_0^H b.  (The K-cycle needs nu > 0:
    without smoothing its level-1 preconditioner P_1 D_2^-1 P_1^H is
    singular and FGMRES stays in the range of P_1.)"""
    H, d0, d1, P0, P1, D2 = three
    H.p["nu"] = nu
    H.p["kc_tol"] = 1e-13
    H.p["kc_restarts"] = 60
    H.cycle_type = cycle
    b = W.gaussian_spinor(DIMS, 7307)
    try:
        z = H.cycle(0, b)
    finally:
        H.p["nu"] = 2
        H.p["kc_tol"] = 1e-1
        H.p["kc_restarts"] = 2
        H.cycle_type = "K"

    def cyc1(c):
        return d1.smooth(c, P1 @ np.linalg.solve(D2, P1.conj().T @ c), nu)

    c = P0.conj().T @ b.reshape(-1)
    if cycle == "V":
        z1 = cyc1(c)
    elif cycle == "W":
        y = cyc1(c)
        z1 = y + cyc1(c - d1.M @ y)
    else:
        z1 = d1.solve(c)
    exp = d0.smooth(b.reshape(-1), P0 @ z1, nu)
    assert _rel(z, exp) < (1e-9 if cycle == "K" else 1e-11)
    if cycle == "V" and nu == 0:
        assert _rel(z, P0 @ P1 @ np.linalg.solve(D2, P1.conj().T @ P0.conj().T @ b.reshape(-1))) < 1e-11
