"""Pins of the oracle's SAP smoother and block MR (Sec. 2, Tab. 1) against
dense brute force on a 4^4 lattice."""
import numpy as np

import workloads as W
from oracle.dirac import WilsonClover
from oracle.lattice import block_colour, coords, shape
from oracle.sap import block_apply, mr_blocks, sap_sweep
from oracle.stencil import dense_matrix

DIMS = (4, 4, 4, 4)
BLOCK = (2, 2, 2, 2)


def _op(csw=1.0):
    return WilsonClover(W.links(DIMS, 0.5, 101), -0.3, csw)


def _rand(rng, shp):
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def _block_ids():
    c = coords(DIMS) // np.asarray(BLOCK)
    nb = [d // b for d, b in zip(DIMS, BLOCK)]
    bid = c[..., 0] + nb[0] * (c[..., 1] + nb[1] * (c[..., 2] + nb[2] * c[..., 3]))
    # expand to dof index (site-major, 12 per site)
    return np.repeat(bid.reshape(-1), 12)


def test_block_apply_is_dirichlet_restriction(rng):
    op = _op()
    D = dense_matrix(op)
    bid = _block_ids()
    Dblk = np.where(bid[:, None] == bid[None, :], D, 0)
    v = _rand(rng, shape(DIMS) + (12,))
    assert np.allclose(block_apply(op, v, BLOCK).reshape(-1), Dblk @ v.reshape(-1), atol=1e-13)


def test_mr_matches_textbook_per_block(rng):
    op = _op()
    D = dense_matrix(op)
    bid = _block_ids()
    r = _rand(rng, shape(DIMS) + (12,))
    x = mr_blocks(op, r, BLOCK, 3).reshape(-1)
    rf = r.reshape(-1)
    for b in np.unique(bid):
        idx = np.nonzero(bid == b)[0]
        Di = D[np.ix_(idx, idx)]
        xi = np.zeros(len(idx), complex)
        rho = rf[idx].copy()
        prev = np.linalg.norm(rho)
        for _ in range(3):
            q = Di @ rho
            alpha = np.vdot(q, rho) / np.vdot(q, q)
            xi += alpha * rho
            rho -= alpha * q
            # the MR step leaves a residual orthogonal to q and never larger
            assert abs(np.vdot(q, rho)) < 1e-12 * np.linalg.norm(q) * np.linalg.norm(rho) + 1e-14
            assert np.linalg.norm(rho) <= prev * (1 + 1e-14)
            prev = np.linalg.norm(rho)
        assert np.allclose(x[idx], xi, atol=1e-13)


def test_zero_mr_iterations_is_identity(rng):
    op = _op()
    b = _rand(rng, shape(DIMS) + (12,))
    z = _rand(rng, shape(DIMS) + (12,))
    assert np.array_equal(sap_sweep(op, b, z, BLOCK, mr_iters=0), z)


def test_sap_exact_blocks_equals_product_formula(rng):
    """With exact block inverses, one SAP step is
    e <- (I - sum_black I_j D_j^-1 I_j^T D)(I - sum_red I_i D_i^-1 I_i^T D) e."""
    op = _op()
    D = dense_matrix(op)
    bid = _block_ids()
    n = D.shape[0]
    Dblk = np.where(bid[:, None] == bid[None, :], D, 0)
    Binv = np.linalg.inv(Dblk)                       # block-diagonal exact inverse
    colour = np.repeat(block_colour(DIMS, BLOCK).reshape(-1), 12)

    def exact(rc, mask):
        return (Binv @ rc.reshape(-1)).reshape(rc.shape)

    b = _rand(rng, shape(DIMS) + (12,))
    z = _rand(rng, shape(DIMS) + (12,))
    znew = sap_sweep(op, b, z, BLOCK, block_solver=exact)
    zstar = np.linalg.solve(D, b.reshape(-1))
    e = zstar - z.reshape(-1)
    I = np.eye(n)
    Pr = np.diag(colour == 0).astype(float)
    Pb = np.diag(colour == 1).astype(float)
    E = (I - Pb @ Binv @ Pb @ D) @ (I - Pr @ Binv @ Pr @ D)
    assert np.allclose(zstar - znew.reshape(-1), E @ e, atol=1e-11)


def test_same_colour_order_independent(rng):
    """Processing the red blocks one at a time, in shuffled order, gives the
    same step as processing them together."""
    op = _op()
    b = _rand(rng, shape(DIMS) + (12,))
    z = _rand(rng, shape(DIMS) + (12,))
    ref = sap_sweep(op, b, z, BLOCK)
    bid = _block_ids().reshape(shape(DIMS) + (12,))
    colour = block_colour(DIMS, BLOCK)
    zz = z.copy()
    for c in (0, 1):
        ids = np.unique(bid[..., 0][colour == c])
        rng.shuffle(ids)
        for i in ids:
            r = b - op.apply(zz)
            m = bid == i
            zz = zz + np.where(m, mr_blocks(op, np.where(m, r, 0), BLOCK, 3), 0)
    assert np.allclose(zz, ref, atol=1e-13)


def test_sap_reduces_error(rng):
    op = _op()
    b = _rand(rng, shape(DIMS) + (12,))
    z = np.zeros_like(b)
    r0 = np.linalg.norm(b)
    for _ in range(4):
        z = sap_sweep(op, b, z, BLOCK)
    assert np.linalg.norm(b - op.apply(z)) < 0.5 * r0
