"""Galerkin coarse operator D_{l+1} = P_l^H D_l P_l (Sec. 1 and Sec. 2).

Blockwise: for coarse sites A (aggregates),

  S_c(A)      = sum_{x in A} P(x)^H S(x) P(x)
                + sum_{x in A, hop x->x+-mu inside A} P(x)^H H_{+-mu}(x) P(x+-mu)
  F_c,mu(A)   = sum_{x in A, x+mu outside A} P(x)^H H_{+mu}(x) P(x+mu)
  B_c,mu(A)   = sum_{x in A, x-mu outside A} P(x)^H H_{-mu}(x) P(x-mu)

i.e. the fine couplings split by the aggregate face they cross.  Backward
blocks are computed directly here; their gamma5 relation to the forward
blocks is checked by the tests, not assumed.
"""
from __future__ import annotations

import numpy as np

from .dirac import dagger
from .lattice import block_sum, inblock_masks, shift
from .stencil import BlockStencil


def galerkin(op, agg) -> BlockStencil:
    P = agg.site_matrices()                              # (T,Z,Y,X,d,2N)
    Pd = dagger(P)
    inside_f, inside_b = inblock_masks(op.dims, agg.agg)
    S_site = Pd @ op.self_matrix() @ P
    F, B = [], []
    for mu in range(4):
        for sign, inside, store in ((+1, inside_f[mu], F), (-1, inside_b[mu], B)):
            c = Pd @ op.hop_matrix(mu, sign) @ shift(P, mu, sign)
            m = inside[..., None, None]
            S_site = S_site + np.where(m, c, 0)
            store.append(block_sum(np.where(m, 0, c), agg.agg))
    S = block_sum(S_site, agg.agg)
    return BlockStencil(agg.cdims, S, np.stack(F), np.stack(B))
