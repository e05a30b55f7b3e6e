"""Wilson(-clover) Dirac operator D (Sec. 1, eq. (1) and the gamma5-symmetry
statement that follows it).

The paper takes the operator's definition from the preceding two-level
paper; this is the textbook Sheikholeslami-Wohlert form, written out plainly:

  (D psi)(x) = (m0 + 4) psi(x)
             - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^H psi(x-mu) ]
             - c_sw/32 sum_{mu,nu} (g_mu g_nu) (Q_mu nu(x) - Q_nu mu(x)) psi(x)

with Q_mu nu the sum of the four plaquette leaves in the (mu, nu) plane.
Spin basis: chiral, Gamma5 = g0 g1 g2 g3 = diag(1, 1, -1, -1), so Gamma5 is
+1 on spins 1, 2 and -1 on spins 3, 4 as the paper states.  A spinor site
vector has index spin*3 + colour.
"""
from __future__ import annotations

import numpy as np

from .lattice import shift

_I2 = np.eye(2, dtype=np.complex128)
_SIGMA = [np.array([[0, 1], [1, 0]], dtype=np.complex128),
          np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
          np.array([[1, 0], [0, -1]], dtype=np.complex128)]


def gammas() -> np.ndarray:
    """Euclidean chiral-basis gamma matrices g_0..g_3 (4x4, Hermitian)."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    for k in range(3):
        g[k][:2, 2:] = -1j * _SIGMA[k]
        g[k][2:, :2] = 1j * _SIGMA[k]
    g[3][:2, 2:] = _I2
    g[3][2:, :2] = _I2
    return g


GAMMA = gammas()
GAMMA5 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)
# Gamma5 on the 12 spin-colour components
GAMMA5_12 = np.kron(GAMMA5, np.eye(3))


def dagger(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def clover_leaves(U: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """Q_mu nu(x): sum of the four counter-clockwise plaquettes at x in the
    (mu, nu) plane.  U has shape (T,Z,Y,X,4,3,3)."""
    Um, Un = U[..., mu, :, :], U[..., nu, :, :]
    Um_m = shift(Um, mu, -1)          # U_mu(x - mu)
    Un_m = shift(Un, mu, -1)          # U_nu(x - mu)
    Un_n = shift(Un, nu, -1)          # U_nu(x - nu)
    # x -> x+mu -> x+mu+nu -> x+nu -> x
    q = _chain(Um, shift(Un, mu, +1), dagger(shift(Um, nu, +1)), dagger(Un))
    # x -> x+nu -> x+nu-mu -> x-mu -> x
    q = q + _chain(Un, dagger(shift(Um_m, nu, +1)), dagger(Un_m), Um_m)
    # x -> x-mu -> x-mu-nu -> x-nu -> x
    q = q + _chain(dagger(Um_m), dagger(shift(Un_m, nu, -1)), shift(Um_m, nu, -1), Un_n)
    # x -> x-nu -> x-nu+mu -> x+mu -> x
    q = q + _chain(dagger(Un_n), shift(Um, nu, -1), shift(Un_n, mu, +1), dagger(Um))
    return q


def _chain(*mats):
    out = mats[0]
    for m in mats[1:]:
        out = out @ m
    return out


def clover_term(U: np.ndarray, csw: float) -> np.ndarray:
    """-c_sw/32 sum_{mu != nu} (g_mu g_nu) (x) (Q_mu nu - Q_nu mu), shape (...,12,12)."""
    lat = U.shape[:4]
    C = np.zeros(lat + (12, 12), dtype=np.complex128)
    if csw == 0.0:
        return C
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            Q = clover_leaves(U, mu, nu)
            F = Q - dagger(Q)          # Q_nu mu = Q_mu nu^H
            s = GAMMA[mu] @ GAMMA[nu]
            C += np.einsum("st,...ab->...satb", s, F).reshape(lat + (12, 12))
    return (-csw / 32.0) * C


class WilsonClover:
    """The fine-level operator D of D z = b.

    Interface shared with the coarse stencil (oracle.stencil.BlockStencil):
    ``d``, ``dims``, ``apply``, ``self_apply``, ``hop``, ``self_matrix``,
    ``hop_matrix``.  ``hop(v, mu, +1)`` is the term coupling v(x + mu) into
    out(x); ``hop(v, mu, -1)`` couples v(x - mu).
    """

    d = 12

    def __init__(self, U: np.ndarray, m0: float, csw: float):
        self.U = U
        self.m0 = float(m0)
        self.csw = float(csw)
        T, Z, Y, X = U.shape[:4]
        self.dims = (X, Y, Z, T)
        self.A = clover_term(U, csw) + (self.m0 + 4.0) * np.eye(12)
        self._pm = [(np.eye(4) - GAMMA[mu], np.eye(4) + GAMMA[mu]) for mu in range(4)]

    def self_apply(self, v: np.ndarray) -> np.ndarray:
        return (self.A @ v[..., None])[..., 0]

    def hop(self, v: np.ndarray, mu: int, sign: int) -> np.ndarray:
        lat = v.shape[:4]
        if sign > 0:
            w = shift(v, mu, +1).reshape(lat + (4, 3))
            Uc = self.U[..., mu, :, :]                        # U_mu(x)
            s = self._pm[mu][0]
        else:
            w = shift(v, mu, -1).reshape(lat + (4, 3))
            Uc = dagger(shift(self.U[..., mu, :, :], mu, -1))  # U_mu(x-mu)^H
            s = self._pm[mu][1]
        chi = w @ np.swapaxes(Uc, -1, -2)     # chi[s, a] = sum_b U[a, b] w[s, b]
        return (-0.5 * (s @ chi)).reshape(lat + (12,))

    def apply(self, v: np.ndarray) -> np.ndarray:
        out = self.self_apply(v)
        for mu in range(4):
            out += self.hop(v, mu, +1)
            out += self.hop(v, mu, -1)
        return out

    def apply_dagger(self, v: np.ndarray) -> np.ndarray:
        """D^H v = Gamma5 D Gamma5 v (the gamma5-symmetry after eq. (1))."""
        return self.apply(v @ GAMMA5_12) @ GAMMA5_12

    def self_matrix(self) -> np.ndarray:
        return self.A

    def hop_matrix(self, mu: int, sign: int) -> np.ndarray:
        """Per-site 12x12 matrix M(x) with hop(v, mu, sign)(x) = M(x) v(x + sign mu)."""
        lat = self.U.shape[:4]
        if sign > 0:
            Uc = self.U[..., mu, :, :]
            s = self._pm[mu][0]
        else:
            Uc = dagger(shift(self.U[..., mu, :, :], mu, -1))
            s = self._pm[mu][1]
        return (-0.5 * np.einsum("st,...ab->...satb", s, Uc)).reshape(lat + (12, 12))


def apply_at_sites(U: np.ndarray, m0: float, csw: float, psi: np.ndarray, sites) -> np.ndarray:
    """(D psi)(x) at the given sites only, each written out from the
    operator's definition (Sec. 1, eq. (1)) with its own index arithmetic:
    the four leaves of every (mu, nu) plane at x, the clover term, the mass
    term and the eight hops.  For checks of large lattices on sampled sites.
    ``sites`` holds (x, y, z, t) tuples; psi has shape (T, Z, Y, X, 12);
    returns (len(sites), 12)."""
    T, Z, Y, X = U.shape[:4]
    ext = (X, Y, Z, T)

    def at(c):
        return (c[3] % T, c[2] % Z, c[1] % Y, c[0] % X)

    def link(c, mu):
        return U[at(c) + (mu,)]

    def step(c, mu, k):
        c = list(c)
        c[mu] += k
        return c

    def h(m):
        return m.conj().T

    out = np.zeros((len(sites), 12), dtype=np.complex128)
    for n, x in enumerate(sites):
        x = [int(v) % e for v, e in zip(x, ext)]
        p = psi[at(x)].reshape(4, 3)
        o = (m0 + 4.0) * p
        if csw != 0.0:
            for mu in range(4):
                for nu in range(4):
                    if mu == nu:
                        continue
                    xm, xn = step(x, mu, -1), step(x, nu, -1)
                    q = (link(x, mu) @ link(step(x, mu, 1), nu) @ h(link(step(x, nu, 1), mu)) @ h(link(x, nu))
                         + link(x, nu) @ h(link(step(xm, nu, 1), mu)) @ h(link(xm, nu)) @ link(xm, mu)
                         + h(link(xm, mu)) @ h(link(step(xm, nu, -1), nu)) @ link(step(xm, nu, -1), mu)
                         @ link(xn, nu)
                         + h(link(xn, nu)) @ link(xn, mu) @ link(step(xn, mu, 1), nu) @ h(link(x, mu)))
                    f = q - h(q)
                    o = o - (csw / 32.0) * (GAMMA[mu] @ GAMMA[nu]) @ p @ f.T
        for mu in range(4):
            fwd = psi[at(step(x, mu, 1))].reshape(4, 3)
            bwd = psi[at(step(x, mu, -1))].reshape(4, 3)
            o = o - 0.5 * ((np.eye(4) - GAMMA[mu]) @ fwd @ link(x, mu).T
                           + (np.eye(4) + GAMMA[mu]) @ bwd @ h(link(step(x, mu, -1), mu)).T)
        out[n] = o.reshape(12)
    return out
