"""Chirality-preserving aggregation interpolation P_l (Sec. 1: P groups spins
1, 2 and spins 3, 4 separately so that D_c stays gamma5-symmetric; Sec. 2.2
and Alg. 3 / Alg. 4: "construct P_l" from the test vectors; Tab. 1 gives the
aggregate sizes 4^4 on level 1 and 2^4 on coarser levels).

For every aggregate A (a lattice block) and chirality sigma (first / second
half of the site components), the restrictions of the N test vectors to
(A, sigma) are orthonormalised in index order (modified Gram-Schmidt, one
re-orthogonalisation pass) into V_{A,sigma}.  P = (+)_{A,sigma} V_{A,sigma},
so P^H P = I, and coarse component (sigma, k) has index sigma*N + k.
"""
from __future__ import annotations

import numpy as np

from .lattice import coarse_dims, from_blocks, shape, to_blocks


def split_aggregates(f, agg):
    """(T,Z,Y,X,d) -> (nT,nZ,nY,nX, 2, m) with m = |A| * d/2."""
    d = f.shape[-1]
    g = to_blocks(f, agg)                                  # (nT..nX, a3..a0, d)
    g = g.reshape(g.shape[:8] + (2, d // 2))
    g = np.moveaxis(g, 8, 4)                               # (nT..nX, 2, a3..a0, d/2)
    return g.reshape(g.shape[:5] + (-1,))


def merge_aggregates(g, agg, d):
    """Inverse of split_aggregates."""
    a0, a1, a2, a3 = agg
    h = g.reshape(g.shape[:5] + (a3, a2, a1, a0, d // 2))
    h = np.moveaxis(h, 4, 8)                               # (nT..nX, a3..a0, 2, d/2)
    h = h.reshape(h.shape[:8] + (d,))
    return from_blocks(h)


def mgs2(W):
    """Orthonormalise the columns of W (..., m, N) in index order: modified
    Gram-Schmidt with one re-orthogonalisation pass."""
    Q = np.array(W, dtype=np.complex128, copy=True)
    N = Q.shape[-1]
    for k in range(N):
        w = Q[..., :, k]
        for _ in range(2):
            for j in range(k):
                q = Q[..., :, j]
                h = np.einsum("...i,...i->...", q.conj(), w)
                w = w - h[..., None] * q
        nrm = np.sqrt(np.einsum("...i,...i->...", w.conj(), w).real)
        if np.any(nrm == 0):
            raise ValueError("test vectors are linearly dependent on an aggregate")
        Q[..., :, k] = w / nrm[..., None]
    return Q


class Aggregation:
    """P for one level: built from test vectors of shape (N, T, Z, Y, X, d)."""

    def __init__(self, dims, agg, vectors):
        self.dims = tuple(dims)
        self.agg = tuple(agg)
        self.cdims = coarse_dims(dims, agg)
        self.N = vectors.shape[0]
        self.d = vectors.shape[-1]
        for L, a in zip(dims, agg):
            if L % a:
                raise ValueError(f"aggregate {agg} does not tile {dims}")
        W = np.stack([split_aggregates(v, agg) for v in vectors], axis=-1)
        if W.shape[-2] < self.N:
            raise ValueError("more test vectors than aggregate dimension")
        self.V = mgs2(W)                                   # (nT..nX, 2, m, N)

    def restrict(self, v):
        """P^H v: fine field -> coarse field (Tc, Zc, Yc, Xc, 2N)."""
        s = split_aggregates(v, self.agg)                   # (nT..nX, 2, m)
        c = np.einsum("...smk,...sm->...sk", self.V.conj(), s)
        return c.reshape(c.shape[:4] + (2 * self.N,))

    def prolong(self, c):
        """P c: coarse field -> fine field."""
        cs = c.reshape(c.shape[:4] + (2, self.N))
        s = np.einsum("...smk,...sk->...sm", self.V, cs)
        return merge_aggregates(s, self.agg, self.d)

    def site_matrices(self):
        """P(x) per fine site: (T, Z, Y, X, d, 2N), block-diagonal in chirality."""
        h = self.d // 2
        out = np.zeros(shape(self.dims) + (self.d, 2 * self.N), dtype=np.complex128)
        for s in range(2):
            cols = np.moveaxis(self.V[..., s, :, :], -1, 0)  # (N, nT..nX, m)
            for k in range(self.N):
                g = np.zeros(self.V.shape[:4] + (2, cols.shape[-1]), dtype=np.complex128)
                g[..., s, :] = cols[k]
                f = merge_aggregates(g, self.agg, self.d)    # (T,Z,Y,X,d)
                out[..., s * h:(s + 1) * h, s * self.N + k] = f[..., s * h:(s + 1) * h]
        return out

    def columns(self):
        """The orthonormalised basis as N fields: (N, T, Z, Y, X, d); column k
        carries V_{A,sigma}[:, k] on every (A, sigma)."""
        out = []
        for k in range(self.N):
            g = self.V[..., :, :, k]                        # (nT..nX, 2, m)
            out.append(merge_aggregates(g, self.agg, self.d))
        return np.stack(out)
