"""Coarse-level operators as nearest-neighbour block stencils (Sec. 2: the
coarse operators D_{l+1} = P_l^H D_l P_l keep the lattice structure; Sec. 3
notes that the operators on all levels are applied lattice-wise).

  (D_c v)(x) = S(x) v(x) + sum_mu [ F_mu(x) v(x + mu) + B_mu(x) v(x - mu) ]

with d x d complex blocks per site.  On a coarse extent of 2 the +mu and -mu
neighbours are the same site, and the two blocks remain separate terms.
"""
from __future__ import annotations

import numpy as np

from .lattice import shift, shape


def _matvec(M, v):
    """Per-site M(x) v(x) for (..., d, d) and (..., d)."""
    return (M @ v[..., None])[..., 0]


class BlockStencil:
    """Generic stencil operator; same interface as dirac.WilsonClover."""

    def __init__(self, dims, S: np.ndarray, F: np.ndarray, B: np.ndarray):
        self.dims = tuple(dims)
        self.S = S                     # (T,Z,Y,X,d,d)
        self.F = F                     # (4,T,Z,Y,X,d,d), couples v(x+mu)
        self.B = B                     # (4,T,Z,Y,X,d,d), couples v(x-mu)
        self.d = S.shape[-1]
        assert S.shape[:4] == shape(dims)

    def self_apply(self, v):
        return _matvec(self.S, v)

    def hop(self, v, mu, sign):
        M = self.F[mu] if sign > 0 else self.B[mu]
        return _matvec(M, shift(v, mu, sign))

    def apply(self, v):
        out = self.self_apply(v)
        for mu in range(4):
            out += self.hop(v, mu, +1)
            out += self.hop(v, mu, -1)
        return out

    def self_matrix(self):
        return self.S

    def hop_matrix(self, mu, sign):
        return self.F[mu] if sign > 0 else self.B[mu]


def gamma5_coarse(d: int) -> np.ndarray:
    """Coarse Gamma5: +1 on the first d/2 components, -1 on the last d/2."""
    return np.diag(np.concatenate([np.ones(d // 2), -np.ones(d // 2)])).astype(np.complex128)


def dense_matrix(op) -> np.ndarray:
    """Dense matrix of a stencil operator (canonical site-major ordering).

    Built column by column from ``op.apply`` on unit vectors; only for tiny
    lattices (brute-force checks)."""
    lat = shape(op.dims)
    n = int(np.prod(lat)) * op.d
    M = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = op.apply(e.reshape(lat + (op.d,))).reshape(n)
        e[j] = 0.0
    return M
