"""Pins of the oracle's Wilson-clover operator against closed forms and
invariants (gamma5-symmetry, Sec. 1; free field; gauge covariance)."""
import numpy as np
import pytest

import workloads as W
from oracle.dirac import GAMMA, GAMMA5, GAMMA5_12, WilsonClover, clover_term, dagger
from oracle.lattice import coords, shift
from oracle.stencil import dense_matrix


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _gauge_transform(U, G):
    out = np.empty_like(U)
    for mu in range(4):
        out[..., mu, :, :] = G @ U[..., mu, :, :] @ dagger(shift(G, mu, +1))
    return out


def _apply_G(G, psi):
    """(G psi)(x) = G(x) acting on the colour index of every spin."""
    lat = psi.shape[:4]
    return np.einsum("...ab,...sb->...sa", G, psi.reshape(lat + (4, 3))).reshape(lat + (12,))


def test_clifford_algebra():
    for mu in range(4):
        assert np.allclose(GAMMA[mu], dagger(GAMMA[mu]))
        for nu in range(4):
            ac = GAMMA[mu] @ GAMMA[nu] + GAMMA[nu] @ GAMMA[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4))
    g5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
    assert np.allclose(g5, GAMMA5)           # +1 on spins 1,2 and -1 on spins 3,4


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_gamma5_hermiticity(csw, rng):
    dims = (4, 4, 2, 4)
    U = W.links(dims, 0.5, 11)
    D = WilsonClover(U, -0.3, csw)
    lat = U.shape[:4]
    phi, psi = _rand(rng, lat + (12,)), _rand(rng, lat + (12,))
    g5 = lambda v: v @ GAMMA5_12.T
    a = np.vdot(phi, g5(D.apply(psi)))
    b = np.conj(np.vdot(psi, g5(D.apply(phi))))
    assert abs(a - b) <= 1e-13 * abs(a)


def test_free_field_plane_wave():
    dims = (4, 6, 4, 8)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (8, 4, 6, 4, 4, 3, 3)).copy()
    m0 = -0.37
    D = WilsonClover(U, m0, 1.0)               # clover vanishes on U = 1
    n = (1, 2, 3, 5)
    p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
    x = coords(dims)
    phase = np.exp(1j * sum(p[mu] * x[..., mu] for mu in range(4)))
    u = np.arange(12) + 1j * np.arange(12)[::-1]
    psi = phase[..., None] * u
    K = (m0 + sum(1 - np.cos(pm) for pm in p)) * np.eye(12) + \
        1j * sum(np.sin(p[mu]) * np.kron(GAMMA[mu], np.eye(3)) for mu in range(4))
    expect = phase[..., None] * (K @ u)
    assert np.max(np.abs(D.apply(psi) - expect)) < 1e-14 * np.max(np.abs(expect))


def test_free_field_spectrum():
    dims = (4, 2, 2, 4)
    lat = (4, 2, 2, 4)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), lat + (4, 3, 3)).copy()
    m0 = 0.1
    ev = np.linalg.eigvals(dense_matrix(WilsonClover(U, m0, 0.0)))
    expect = []
    for n in np.ndindex(*dims):
        p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
        re = m0 + sum(1 - np.cos(q) for q in p)
        im = np.sqrt(sum(np.sin(q) ** 2 for q in p))
        expect += [re + 1j * im] * 6 + [re - 1j * im] * 6
    key = lambda z: (round(z.real, 8), round(z.imag, 8))
    a = np.array(sorted(ev, key=key))
    b = np.array(sorted(expect, key=key))
    assert np.max(np.abs(a - b)) < 1e-10


def test_gauge_covariance(rng):
    dims = (4, 4, 4, 4)
    U = W.links(dims, 0.6, 21)
    G = W.random_su3(dims, 22)
    psi = _rand(rng, U.shape[:4] + (12,))
    D = WilsonClover(U, -0.4, 1.0)
    DG = WilsonClover(_gauge_transform(U, G), -0.4, 1.0)
    lhs = DG.apply(_apply_G(G, psi))
    rhs = _apply_G(G, D.apply(psi))
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


def test_pure_gauge_is_free_field(rng):
    dims = (4, 2, 4, 4)
    G = W.random_su3(dims, 31)
    one = np.broadcast_to(np.eye(3, dtype=np.complex128), G.shape[:4] + (4, 3, 3)).copy()
    U = _gauge_transform(one, G)
    assert np.max(np.abs(clover_term(U, 1.0))) < 1e-13
    psi = _rand(rng, G.shape[:4] + (12,))
    D = WilsonClover(U, -0.2, 1.0)
    D0 = WilsonClover(one, -0.2, 1.0)
    Gd = dagger(G)
    assert np.allclose(D.apply(psi), _apply_G(G, D0.apply(_apply_G(Gd, psi))), atol=1e-13)


def test_clover_constant_abelian_field():
    """U_y(x) = exp(i B x_0) (colour-diagonal), all other links 1: every
    (0,1) plaquette leaf equals exp(iB), so F_01 = 8 i sin B and the clover
    term is -(i c_sw sin B / 2) g0 g1 (x) 1 at every site."""
    dims = (6, 4, 2, 2)
    B = 2 * np.pi / dims[0]
    lat = (2, 2, 4, 6)
    x = coords(dims)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), lat + (4, 3, 3)).copy()
    U[..., 1, :, :] = np.exp(1j * B * x[..., 0])[..., None, None] * np.eye(3)
    csw = 0.8
    C = clover_term(U, csw)
    expect = -(1j * csw * np.sin(B) / 2) * np.kron(GAMMA[0] @ GAMMA[1], np.eye(3))
    assert np.max(np.abs(C - expect)) < 1e-14


def test_clover_hermitian_and_chiral(rng):
    U = W.links((4, 4, 4, 4), 0.5, 41)
    C = clover_term(U, 1.0)
    assert np.max(np.abs(C - dagger(C))) < 1e-14
    assert np.max(np.abs(C[..., :6, 6:])) < 1e-14   # commutes with Gamma5
    assert np.max(np.abs(C)) > 1e-2


def test_hop_matrix_consistent(rng):
    U = W.links((4, 2, 2, 4), 0.5, 51)
    D = WilsonClover(U, -0.1, 1.0)
    v = _rand(rng, U.shape[:4] + (12,))
    for mu in range(4):
        for s in (+1, -1):
            M = D.hop_matrix(mu, s)
            ref = np.einsum("...ij,...j->...i", M, shift(v, mu, s))
            assert np.allclose(D.hop(v, mu, s), ref, atol=1e-14)


def test_links_are_su3():
    U = W.links((2, 2, 2, 4), 0.5, 3)
    I = np.eye(3)
    assert np.max(np.abs(dagger(U) @ U - I)) < 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-14


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_apply_at_sites_matches_full_apply(csw, rng):
    """The site-by-site evaluation (used on sampled sites of large lattices)
    against the whole-lattice operator, on every site of a 4x4x4x6 lattice."""
    from oracle.dirac import apply_at_sites
    dims = (4, 4, 4, 6)
    U = W.links(dims, 0.6, 97)
    psi = W.gaussian_spinor(dims, 98)
    full = WilsonClover(U, -0.3, csw).apply(psi)
    sites = [(x, y, z, t) for t in range(6) for z in range(4) for y in range(4) for x in range(4)]
    got = apply_at_sites(U, -0.3, csw, psi, sites)
    ref = np.array([full[t, z, y, x] for (x, y, z, t) in sites])
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
