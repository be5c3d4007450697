"""Pins of the clover-term oracle: the free field, the algebra of F and
sigma, gamma5-hermiticity of the full operator and gauge covariance of its
traces (a random local SU(3) rotation of the links)."""
import numpy as np
import pytest

from oracle import clover, dirac
from oracle.gamma import GAMMA5
from oracle.geometry import coords, neighbour, volume
from oracle.solve import dense_inverse
from synth.gauge import gauge_field


def test_free_field_has_no_clover_term():
    dims = (2, 2, 2, 4)
    U = gauge_field(dims, 0.0, seed=1)
    assert np.max(np.abs(clover.clover_blocks(U, dims, 1.7))) < 1e-14


def test_field_strength_algebra():
    dims = (2, 4, 2, 4)
    U = gauge_field(dims, 0.6, seed=2)
    F = clover.field_strength(U, dims)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            f = F[:, mu, nu]
            assert np.max(np.abs(f - np.conj(np.swapaxes(f, 1, 2)))) < 1e-14   # Hermitian
            assert np.max(np.abs(f + F[:, nu, mu])) < 1e-14                     # antisymmetric
    # sigma: Hermitian, commutes with gamma5 (the term keeps chirality)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            s = clover.sigma(mu, nu)
            assert np.max(np.abs(s - s.conj().T)) < 1e-15
            assert np.max(np.abs(s @ GAMMA5 - GAMMA5 @ s)) < 1e-15


def test_field_strength_abelian_closed_form():
    """Diagonal links diag(e^{i a}, e^{i b}, e^{i c}) are three independent U(1)
    fields.  Every leaf is then the phase of one plaquette with the same
    orientation, and the four leaves at x are the plaquettes based at x,
    x - mu, x - nu and x - mu - nu, so per colour
    F_{mu nu}(x) = (1/4) sum of sin(plaquette angle) over those four."""
    dims = (3, 2, 4, 2)
    V = volume(dims)
    rng = np.random.default_rng(7)
    th = rng.uniform(-np.pi, np.pi, (V, 4, 3))
    U = np.zeros((V, 4, 3, 3), dtype=complex)
    for a in range(3):
        U[:, :, a, a] = np.exp(1j * th[:, :, a])
    F = clover.field_strength(U, dims)
    C = coords(dims)

    def idx(c):
        c = np.mod(c, dims)
        return c[..., 0] + dims[0] * (c[..., 1] + dims[1] * (c[..., 2] + dims[2] * c[..., 3]))

    e = np.eye(4, dtype=int)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue

            def plaq(base):   # angle of the (mu, nu) plaquette based at coordinates base
                return (th[idx(base), mu] + th[idx(base + e[mu]), nu]
                        - th[idx(base + e[nu]), mu] - th[idx(base), nu])

            want = 0.25 * sum(np.sin(plaq(C - shift)) for shift in
                              (0 * e[mu], e[mu], e[nu], e[mu] + e[nu]))
            got = np.diagonal(F[:, mu, nu], axis1=1, axis2=2)
            assert np.max(np.abs(got - want)) < 1e-14, (mu, nu)
            off = F[:, mu, nu] - np.einsum("xa,ab->xab", got, np.eye(3))
            assert np.max(np.abs(off)) == 0


def test_clover_operator_gamma5_hermitian():
    dims, m0, csw = (2, 2, 2, 4), 0.1, 1.3
    U = gauge_field(dims, 0.5, seed=3)
    D = clover.dense_D_clover(U, m0, dims, csw)
    g5 = np.kron(np.eye(volume(dims)), np.kron(GAMMA5, np.eye(3)))
    assert np.max(np.abs(g5 @ D @ g5 - D.conj().T)) < 1e-13
    C = clover.clover_blocks(U, dims, csw)
    assert np.max(np.abs(C)) > 1e-3                   # the term is really there
    assert np.max(np.abs(C - np.conj(np.swapaxes(C, 1, 2)))) < 1e-14


def _random_su3(n, rng):
    A = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    Q, R = np.linalg.qr(A)
    d = np.diagonal(R, axis1=1, axis2=2)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    return Q / det[:, None, None] ** (1.0 / 3.0)


def test_gauge_covariance_of_clover_operator():
    """U_mu(x) -> W(x) U_mu(x) W(x + mu)^dag maps the clover blocks to
    W(x) C(x) W(x)^dag and leaves tr D^-1 unchanged."""
    dims, m0, csw = (2, 2, 2, 4), 0.2, 1.1
    U = gauge_field(dims, 0.5, seed=4)
    V = volume(dims)
    rng = np.random.default_rng(5)
    W = _random_su3(V, rng)
    U2 = np.empty_like(U)
    for mu in range(4):
        fwd = neighbour(dims, mu, +1, +1)[0]
        U2[:, mu] = W @ U[:, mu] @ np.conj(np.swapaxes(W[fwd], 1, 2))
    C, C2 = clover.clover_blocks(U, dims, csw), clover.clover_blocks(U2, dims, csw)
    Wf = np.einsum("st,xab->xsatb", np.eye(4), W).reshape(V, 12, 12)
    assert np.max(np.abs(C2 - Wf @ C @ np.conj(np.swapaxes(Wf, 1, 2)))) < 1e-13
    Di = dense_inverse(clover.dense_D_clover(U, m0, dims, csw))
    Di2 = dense_inverse(clover.dense_D_clover(U2, m0, dims, csw))
    assert abs(np.trace(Di) - np.trace(Di2)) < 1e-11 * abs(np.trace(Di))
    # and csw = 0 is the plain Wilson operator
    assert np.max(np.abs(clover.dense_D_clover(U, m0, dims, 0.0) - dirac.dense_D(U, m0, dims))) == 0


def _constant_field(dims, mu, nu, n):
    """Diagonal (abelian) links with n flux quanta spread evenly over the
    (mu, nu) plane of a torus: every plaquette of that plane has angle
    B = 2 pi n / (L_mu L_nu), the others zero."""
    V = volume(dims)
    C = coords(dims)
    B = 2 * np.pi * n / (dims[mu] * dims[nu])
    th = np.zeros((V, 4))
    th[:, nu] = B * C[:, mu]
    edge = C[:, mu] == dims[mu] - 1
    th[edge, mu] = -B * dims[mu] * C[edge, nu]
    U = np.zeros((V, 4, 3, 3), dtype=complex)
    for a in range(3):
        U[:, :, a, a] = np.exp(1j * th)
    return U, B


@pytest.mark.parametrize("dims,mu,nu", [((8, 8, 1, 1), 0, 1), ((1, 1, 8, 8), 2, 3),
                                        ((1, 8, 1, 8), 1, 3)])
def test_clover_sign_removes_wilson_shift_of_landau_modes(dims, mu, nu):
    """Tree-level O(a) improvement fixes the sign of the term.  In a constant
    field B (lattice units) the naive operator has exact zero modes (index
    theorem: n per colour and per 2-d spinor copy, 6 here).  The Wilson term
    lifts them to |lambda| = B/2 + O(B^2); the clover term at c_sw = 1 must
    cancel that shift to O(B^2), and the opposite sign doubles it.  Extents 1
    (periodic) reduce the operator to the two-dimensional one in the plane."""
    U, B = _constant_field(dims, mu, nu, 1)
    F = clover.field_strength(U, dims)
    assert np.max(np.abs(F[:, mu, nu] - np.sin(B) * np.eye(3))) < 1e-15
    low = {}
    for csw in (0.0, 1.0, -1.0):
        ev = np.abs(np.linalg.eigvals(clover.dense_D_clover(U, 0.0, dims, csw, bc_t=+1)))
        ev.sort()
        assert ev[6] > 0.4                          # a gap above the six modes
        low[csw] = ev[:6]
    assert np.all(np.abs(low[0.0] - B / 2) < 0.02 * B)
    assert np.all(low[1.0] < 0.01 * B)
    assert np.all(np.abs(low[-1.0] - B) < 0.02 * B)
