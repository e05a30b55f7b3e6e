"""Red-black Schwarz alternating procedure (SAP) with minimal-residual block
solves: the smoother M_l of Sec. 2 (error propagator I - M_l D_l), with the
lattice-block size and the number of MR iterations of Tab. 1.

One smoothing step z <- z + M (b - D z) is the multiplicative Schwarz method
over two colours of lattice blocks:

  for colour in (red, black):
      r = b - D z                       (full operator, current z)
      for every block i of this colour:
          z_i <- z_i + B_i r_i          (B_i ~ D_i^{-1}, D_i = D restricted to block i)

Blocks of one colour never touch (the block count per direction is even), so
they are processed together.  D_i keeps only the couplings with both ends in
block i (Dirichlet restriction).  Colour = (sum of block coordinates) mod 2,
colour 0 first.
"""
from __future__ import annotations

import numpy as np

from .lattice import block_broadcast, block_colour, block_sum, inblock_masks


def block_apply(op, v, block):
    """The block-diagonal operator (+)_i D_i applied to v (all blocks at once)."""
    fwd, bwd = inblock_masks(op.dims, block)
    out = op.self_apply(v)
    for mu in range(4):
        out += fwd[mu][..., None] * op.hop(v, mu, +1)
        out += bwd[mu][..., None] * op.hop(v, mu, -1)
    return out


def _block_dot(a, b, block):
    """<a, b> = sum conj(a) b over every block."""
    return block_sum((np.conj(a) * b).sum(-1), block)


def mr_blocks(op, r, block, n_iter):
    """Minimal residual on every block, from zero: for k < n_iter,
    q = D_i rho, alpha = <q, rho>/<q, q>, x += alpha rho, rho -= alpha q.

    alpha minimises ||rho - alpha q||.  Blocks where r is zero stay zero."""
    x = np.zeros_like(r)
    rho = r.copy()
    for _ in range(n_iter):
        q = block_apply(op, rho, block)
        qr = _block_dot(q, rho, block)
        qq = _block_dot(q, q, block).real
        alpha = np.where(qq > 0, qr / np.where(qq > 0, qq, 1.0), 0.0)
        a = block_broadcast(alpha, block)[..., None]
        x += a * rho
        rho -= a * q
    return x


def sap_sweep(op, b, z, block, mr_iters=3, block_solver=None):
    """One SAP step z <- z + M (b - D z); returns the new z.

    ``block_solver(r_masked, colour_mask)`` may replace MR (the tests use an
    exact dense block inverse)."""
    colour = block_colour(op.dims, block)
    z = z.copy()
    for c in (0, 1):
        r = b - op.apply(z)
        mask = (colour == c)[..., None]
        rc = np.where(mask, r, 0)
        if block_solver is None:
            e = mr_blocks(op, rc, block, mr_iters)
        else:
            e = block_solver(rc, mask)
        z += np.where(mask, e, 0)
    return z


def smooth(op, b, z, nsweeps, block, mr_iters=3):
    for _ in range(nsweeps):
        z = sap_sweep(op, b, z, block, mr_iters)
    return z


def validate_blocks(dims, block):
    """Blocks must tile the lattice with an even count per direction."""
    for L, s in zip(dims, block):
        if L % s != 0 or (L // s) % 2 != 0:
            raise ValueError(f"SAP block {block} does not tile {dims} with even counts")
