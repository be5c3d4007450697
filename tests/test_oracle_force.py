"""Pins of the oracle's derivatives of eta^dag D^-1 eta: central finite
differences, torch complex autograd through a dense solve, and the free-field
closed form of -tr D^-2."""
import numpy as np
import pytest
import torch

from oracle import dirac, force, gamma, geometry, noise, solve
from synth.gauge import gauge_field

DIMS = (2, 2, 2, 4)


def _f(U, m0, eta):
    D = dirac.dense_D(U, m0, DIMS, -1)
    return np.vdot(eta, solve.dense_solve(D, eta))


@pytest.fixture(scope="module")
def setup():
    V = geometry.volume(DIMS)
    U = gauge_field(DIMS, 0.4, seed=21)
    m0 = 0.15
    eta = noise.rademacher(3, 12 * V).astype(complex)
    D = dirac.dense_D(U, m0, DIMS, -1)
    x = solve.dense_solve(D, eta)
    y = solve.dense_solve(D.conj().T, eta)
    return U, m0, eta, x, y


def test_adjoint_solution_by_gamma5(setup):
    U, m0, eta, x, y = setup
    V = geometry.volume(DIMS)
    G5 = np.kron(np.eye(V), gamma.spin_colour(gamma.GAMMA5))
    D = dirac.dense_D(U, m0, DIMS, -1)
    assert np.allclose(y, G5 @ solve.dense_solve(D, G5 @ eta), atol=1e-13)


def test_dm0_finite_difference(setup):
    U, m0, eta, x, y = setup
    h = 1e-5
    fd = (_f(U, m0 + h, eta) - _f(U, m0 - h, eta)) / (2 * h)
    assert abs(force.dm0(x, y) - fd) < 1e-7 * abs(fd)


def test_link_derivatives_finite_difference(setup):
    U, m0, eta, x, y = setup
    A, B = force.force_terms(x, y, DIMS, -1)
    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(6):
        s, mu, a, b = rng.integers(16), rng.integers(4), rng.integers(3), rng.integers(3)
        if rng.integers(2) == 0:
            mu = 3                               # include time-boundary links
            s = 8 + rng.integers(8)
        E = np.zeros_like(U)
        E[s, mu, a, b] = 1.0
        dre = (_f(U + h * E, m0, eta) - _f(U - h * E, m0, eta)) / (2 * h)
        dim = (_f(U + 1j * h * E, m0, eta) - _f(U - 1j * h * E, m0, eta)) / (2 * h)
        # Wirtinger: df/dU = (d/dRe - i d/dIm)/2, df/dconjU = (d/dRe + i d/dIm)/2
        assert abs(A[s, mu, a, b] - 0.5 * (dre - 1j * dim)) < 1e-7
        assert abs(B[s, mu, a, b] - 0.5 * (dre + 1j * dim)) < 1e-7


def _torch_D(U, m0):
    """Dense D assembled in torch from the same definition (for autograd)."""
    V = geometry.volume(DIMS)
    n = 12 * V
    G = torch.tensor(gamma.GAMMA)
    I4 = torch.eye(4, dtype=torch.complex128)
    D = (4 + m0) * torch.eye(n, dtype=torch.complex128)
    for mu in range(4):
        fwd, phf = geometry.neighbour(DIMS, mu, +1, -1)
        for xs in range(V):
            y = int(fwd[xs])
            blk = torch.kron(I4 - G[mu], U[xs, mu]) * (-0.5 * phf[xs])
            D = D.index_put((torch.arange(12 * xs, 12 * xs + 12)[:, None],
                             torch.arange(12 * y, 12 * y + 12)[None, :]), blk, accumulate=True)
            blkb = torch.kron(I4 + G[mu], U[xs, mu].conj().T.resolve_conj().contiguous()) * (-0.5 * phf[xs])
            D = D.index_put((torch.arange(12 * y, 12 * y + 12)[:, None],
                             torch.arange(12 * xs, 12 * xs + 12)[None, :]), blkb, accumulate=True)
    return D


@pytest.mark.parametrize("g", [1.0 + 0j, 1j, 0.3 - 0.7j])
def test_torch_autograd_convention(setup, g):
    U, m0, eta, x, y = setup
    Ut = torch.tensor(U, requires_grad=True)
    mt = torch.tensor(m0, dtype=torch.float64, requires_grad=True)
    et = torch.tensor(eta)
    f = torch.vdot(et, torch.linalg.solve(_torch_D(Ut, mt), et))
    f.backward(torch.tensor(g, dtype=torch.complex128))
    gU = force.grad_links([x], [y], [g], DIMS, -1)
    assert np.max(np.abs(Ut.grad.numpy() - gU)) < 1e-12
    assert abs(mt.grad.item() - force.grad_m0([x], [y], [g])) < 1e-12


def test_free_field_mean_dm0_closed_form():
    """E[df/dm0] = -tr D^-2; for U = 1 it has a momentum-space closed form."""
    dims, m0 = (2, 2, 2, 4), 0.2
    V = geometry.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    D = dirac.dense_D(U, m0, dims, -1)
    Dinv = solve.dense_inverse(D)
    Dinvh = solve.dense_inverse(D.conj().T)
    tot = sum(force.dm0(Dinv[:, i], Dinvh[:, i]) for i in range(12 * V))
    ks = [(2 * np.pi * np.arange(L) + (np.pi if mu == 3 else 0)) / L for mu, L in enumerate(dims)]
    P = np.meshgrid(*ks, indexing="ij")
    M = m0 + sum(1 - np.cos(p) for p in P)
    s2 = sum(np.sin(p) ** 2 for p in P)
    closed = np.sum(12 * (s2 - M ** 2) / (M ** 2 + s2) ** 2)
    assert abs(tot - closed) < 1e-11 * abs(closed)
