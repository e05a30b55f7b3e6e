"""Krylov solvers: flexible GMRES (Sec. 2: the multilevel method preconditions
FGMRES; Sec. 2.1: the K-cycle solves each coarse system by a few FGMRES
iterations; Tab. 1: restart length 10 and tolerance 1e-10 outside, length 5,
2 restart cycles and tolerance 1e-1 in the K-cycle) and the coarsest-level
solve by odd-even preconditioned GMRES to relative accuracy eps (Sec. 3);
and CGNR, the paper's comparison method (Sec. 4).

The oracle takes the plainest route: Arnoldi with modified Gram-Schmidt and,
at every step, the small least-squares problem min || beta e1 - H y || solved
by numpy's lstsq.  Its residual is the Arnoldi residual estimate.
"""
from __future__ import annotations

import numpy as np


def vdot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def norm(a):
    return float(np.sqrt(vdot(a, a).real))


def fgmres(A, b, M, m, max_cycles, tol, x0=None, check_true_residual=False, stats=None):
    """Right-preconditioned flexible GMRES(m), at most max_cycles restart cycles.

    Stops when the Arnoldi residual estimate is <= tol * ||b||.  With
    check_true_residual, convergence is only accepted when the recomputed
    residual ||b - A x|| also is (otherwise the method restarts).
    ``M`` may be None (plain GMRES).  Returns x."""
    bnorm = norm(b)
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - A(x)
    beta = norm(r)
    target = tol * bnorm
    iters = 0
    history = [beta]
    converged = beta <= target
    for _cycle in range(max_cycles):
        if converged or beta == 0.0:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        y = None
        est = beta
        for j in range(m):
            z = V[j] if M is None else M(V[j])
            Z.append(z)
            w = A(z)
            for i in range(j + 1):
                H[i, j] = vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = norm(w)
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
            est = norm(e1 - H[:j + 2, :j + 1] @ y)
            iters += 1
            history.append(est)
            if est <= target or H[j + 1, j] == 0.0:
                break
            V.append(w / H[j + 1, j])
        for i, yi in enumerate(y):
            x = x + yi * Z[i]
        if est <= target:
            if check_true_residual:
                r = b - A(x)
                beta = norm(r)
                converged = beta <= target
            else:
                converged = True
        else:
            r = b - A(x)
            beta = norm(r)
            converged = check_true_residual and beta <= target
    if stats is not None:
        stats["iters"] = stats.get("iters", 0) + iters
        stats["converged"] = converged
        stats["history"] = history
    return x


def cgnr(A, AH, b, tol, max_iter, x0=None, stats=None):
    """CGNR, the Krylov method the paper compares against (Sec. 4, Tab. 5;
    its iteration count is the conditioning indicator of Tab. 2): conjugate
    gradients applied to A^H A x = A^H b, carried with the residual
    r = b - A x.  Textbook CG on the normal equations: search direction p,
    step alpha = ||A^H r||^2 / ||A p||^2, x += alpha p, r -= alpha A p,
    beta = ||A^H r_new||^2 / ||A^H r_old||^2, p = A^H r_new + beta p.
    Stops when ||r|| <= tol ||b|| or after max_iter iterations; ``AH``
    applies A^H.  Returns x (stats: iterations, residual history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A(x)
    target = tol * norm(b)
    z = AH(r)
    p = z.copy()
    gam = vdot(z, z).real
    history = [norm(r)]
    iters = 0
    while history[-1] > target and iters < max_iter:
        w = A(p)
        alpha = gam / vdot(w, w).real
        x = x + alpha * p
        r = r - alpha * w
        iters += 1
        history.append(norm(r))
        if history[-1] <= target:
            break
        z = AH(r)
        gam_new = vdot(z, z).real
        p = z + (gam_new / gam) * p
        gam = gam_new
    if stats is not None:
        stats["iters"] = iters
        stats["history"] = history
        stats["converged"] = history[-1] <= target
    return x


class OddEvenCoarsest:
    """Coarsest-level solve (Sec. 3): eliminate the even sites,

      S = D_oo - D_oe D_ee^{-1} D_eo,   S z_o = b_o - D_oe D_ee^{-1} b_e,
      z_e = D_ee^{-1} (b_e - D_eo z_o),

    and solve the Schur system by GMRES(restart) from zero to
    ||res|| <= eps * ||b_o - D_oe D_ee^{-1} b_e||.  D_ee is the self
    coupling of the even sites (the hops join even and odd sites only, which
    needs every extent even).  On a non-bipartite lattice the full system is
    solved by GMRES instead."""

    def __init__(self, op, eps, restart=30, max_restarts=10):
        from .lattice import parity
        self.op = op
        self.eps = eps
        self.restart = restart
        self.max_restarts = max_restarts
        self.bipartite = all(L % 2 == 0 for L in op.dims)
        p = parity(op.dims)
        self.even = (p == 0)[..., None]
        self.odd = ~self.even
        if self.bipartite:
            self.See_inv = np.linalg.inv(op.self_matrix())   # used on even sites only

    def _hops(self, v):
        out = np.zeros_like(v)
        for mu in range(4):
            out += self.op.hop(v, mu, +1)
            out += self.op.hop(v, mu, -1)
        return out

    def _Dee_inv(self, v):
        return np.where(self.even, np.einsum("...ij,...j->...i", self.See_inv, v), 0)

    def schur(self, vo):
        """S v_o on the odd sites (even components of the result are zero)."""
        t = self._Dee_inv(np.where(self.even, self._hops(vo), 0))
        out = self.op.self_apply(vo) - self._hops(t)
        return np.where(self.odd, out, 0)

    def solve(self, b, stats=None):
        if not self.bipartite:
            return fgmres(self.op.apply, b, None, self.restart, self.max_restarts,
                          self.eps, stats=stats)
        be = np.where(self.even, b, 0)
        bo = np.where(self.odd, b, 0)
        rhs = bo - np.where(self.odd, self._hops(self._Dee_inv(be)), 0)
        zo = fgmres(self.schur, rhs, None, self.restart, self.max_restarts, self.eps,
                    stats=stats)
        ze = self._Dee_inv(be - np.where(self.even, self._hops(zo), 0))
        return ze + zo
