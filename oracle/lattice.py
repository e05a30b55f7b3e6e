"""Lattice geometry helpers for the oracle (periodic 4D lattice).

A field has shape (T, Z, Y, X, ...); direction mu lives on axis 3 - mu.
"""
from __future__ import annotations

import numpy as np


def axis(mu: int) -> int:
    return 3 - mu


def shape(dims):
    X, Y, Z, T = dims
    return (T, Z, Y, X)


def shift(f: np.ndarray, mu: int, sign: int) -> np.ndarray:
    """g(x) = f(x + sign * mu_hat), periodic."""
    return np.roll(f, -sign, axis=axis(mu))


def coords(dims) -> np.ndarray:
    """Integer coordinates, shape (T, Z, Y, X, 4) with [..., mu] = x_mu."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X),
                             indexing="ij")
    return np.stack([x, y, z, t], axis=-1)


def parity(dims) -> np.ndarray:
    """(sum_mu x_mu) mod 2 per site."""
    return coords(dims).sum(-1) % 2


def block_colour(dims, block) -> np.ndarray:
    """Red-black colour of the lattice block that holds each site."""
    c = coords(dims) // np.asarray(block)
    return c.sum(-1) % 2


def inblock_masks(dims, block):
    """fwd[mu] is True where the hop to x + mu stays inside x's block;
    bwd[mu] is True where the hop to x - mu stays inside x's block."""
    c = coords(dims) % np.asarray(block)
    fwd = [c[..., mu] < block[mu] - 1 for mu in range(4)]
    bwd = [c[..., mu] > 0 for mu in range(4)]
    return fwd, bwd


def to_blocks(f: np.ndarray, block) -> np.ndarray:
    """Reshape (T, Z, Y, X, *rest) -> (nT, nZ, nY, nX, bT, bZ, bY, bX, *rest)."""
    T, Z, Y, X = f.shape[:4]
    b0, b1, b2, b3 = block
    rest = f.shape[4:]
    g = f.reshape((T // b3, b3, Z // b2, b2, Y // b1, b1, X // b0, b0) + rest)
    nrest = len(rest)
    perm = (0, 2, 4, 6, 1, 3, 5, 7) + tuple(range(8, 8 + nrest))
    return g.transpose(perm)


def from_blocks(g: np.ndarray) -> np.ndarray:
    """Inverse of to_blocks."""
    nT, nZ, nY, nX, b3, b2, b1, b0 = g.shape[:8]
    rest = g.shape[8:]
    nrest = len(rest)
    perm = (0, 4, 1, 5, 2, 6, 3, 7) + tuple(range(8, 8 + nrest))
    return g.transpose(perm).reshape((nT * b3, nZ * b2, nY * b1, nX * b0) + rest)


def block_sum(f: np.ndarray, block) -> np.ndarray:
    """Sum of f over the sites of each block: (T,Z,Y,X,*rest) -> (nT,nZ,nY,nX,*rest)."""
    return to_blocks(f, block).sum(axis=(4, 5, 6, 7))


def block_broadcast(c: np.ndarray, block) -> np.ndarray:
    """Per-block value (nT,nZ,nY,nX,*rest) copied to every site of the block."""
    b0, b1, b2, b3 = block
    g = c
    for ax, b in zip(range(4), (b3, b2, b1, b0)):
        g = np.repeat(g, b, axis=ax)
    return g


def coarse_dims(dims, agg):
    return tuple(d // a for d, a in zip(dims, agg))
