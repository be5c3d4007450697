"""Pins of the oracle's operator, gauge links and solvers against facts fixed
by mathematics: the Dirac algebra, free-field momentum-space closed forms,
gauge covariance and gamma5-hermiticity (Hermiticity of Q = Gamma5 D, Sec. 2).
"""
import numpy as np
import pytest

from oracle import dirac, gamma, geometry, solve, estimator
from synth.gauge import gauge_field, random_su3_transform


def test_gamma_algebra():
    G = gamma.GAMMA
    for m in range(4):
        assert np.allclose(G[m], G[m].conj().T)
        for n in range(4):
            assert np.allclose(G[m] @ G[n] + G[n] @ G[m], 2 * (m == n) * np.eye(4))
    assert np.allclose(gamma.GAMMA5, np.diag([1, 1, -1, -1]))


def test_gauge_links_su3():
    U = gauge_field((4, 4, 4, 4), 0.5, seed=3)
    uu = np.einsum("xmab,xmcb->xmac", U, np.conj(U))
    assert np.allclose(uu, np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(U), 1.0, atol=1e-14)
    U0 = gauge_field((2, 2, 2, 2), 0.0, seed=3)
    assert np.array_equal(U0, np.broadcast_to(np.eye(3), U0.shape))
    # seeded: same seed, same field; different seed, different field
    assert np.array_equal(U, gauge_field((4, 4, 4, 4), 0.5, seed=3))
    assert not np.allclose(U, gauge_field((4, 4, 4, 4), 0.5, seed=4))


def _free_momenta(dims, bc_t):
    ks = []
    for mu, L in enumerate(dims):
        n = np.arange(L)
        shift = np.pi if (mu == 3 and bc_t == -1) else 0.0
        ks.append((2 * np.pi * n + shift) / L)
    return np.meshgrid(*ks, indexing="ij")


def test_free_field_trace_closed_form():
    # D(p) = M(p) + i sum gamma_mu sin p_mu, M = m0 + sum(1 - cos p_mu):
    # tr D^-1 = sum_p 12 M / (M^2 + sum sin^2 p_mu).
    dims, m0 = (4, 4, 4, 4), 0.2
    P = _free_momenta(dims, -1)
    M = m0 + sum(1 - np.cos(p) for p in P)
    s2 = sum(np.sin(p) ** 2 for p in P)
    closed = np.sum(12 * M / (M ** 2 + s2))
    U = np.broadcast_to(np.eye(3, dtype=complex), (256, 4, 3, 3)).copy()
    Dinv = solve.dense_inverse(dirac.dense_D(U, m0, dims, -1))
    assert abs(np.trace(Dinv) - closed) < 1e-11 * abs(closed)
    # -tr D^-2 (the mean of d/dm0 of eta^dag D^-1 eta) also has a closed form
    closed2 = np.sum(12 * (s2 - M ** 2) / (M ** 2 + s2) ** 2)
    assert abs(-np.trace(Dinv @ Dinv) - closed2) < 1e-11 * abs(closed2)


@pytest.mark.parametrize("bc_t", [-1, 1])
def test_free_field_point_propagator_fft(bc_t):
    """A point-source column of D^-1 equals the 4D inverse FFT of
    D(p)^-1 = (M - i sum gamma_mu sin p_mu)/(M^2 + s^2): this fixes the hopping
    sign, the (1 - gamma) forward projector, the time boundary and the
    (4 + m0) normalisation."""
    dims, m0 = (4, 2, 2, 6), 0.3
    V = geometry.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    D = dirac.dense_D(U, m0, dims, bc_t)
    src = np.zeros(12 * V, dtype=complex)
    src[3 * 1 + 0] = 1.0                      # site 0, spin 1, colour 0
    col = solve.dense_solve(D, src).reshape(dims[::-1] + (4, 3))  # [t,z,y,x,s,c]
    P = _free_momenta(dims, bc_t)            # indexed [x,y,z,t]
    M = m0 + sum(1 - np.cos(p) for p in P)
    s2 = sum(np.sin(p) ** 2 for p in P)
    Sp = (M[..., None, None] * np.eye(4)
          - 1j * sum(np.sin(P[m])[..., None, None] * gamma.GAMMA[m] for m in range(4)))
    Sp = Sp / (M ** 2 + s2)[..., None, None]
    # S(x) = (1/V) sum_p e^{i p.x} S(p); antiperiodic p_t = 2 pi n/Lt + pi/Lt
    Sx = np.fft.ifftn(Sp, axes=(0, 1, 2, 3))
    if bc_t == -1:
        t = np.arange(dims[3])
        Sx = Sx * np.exp(1j * np.pi * t / dims[3])[None, None, None, :, None, None]
    expect = Sx[..., :, 1]                     # column spin 1
    got = np.transpose(col[..., :, 0], (3, 2, 1, 0, 4))  # -> [x,y,z,t,s]
    assert np.max(np.abs(got - expect)) < 1e-13
    assert np.max(np.abs(col[..., :, 1:])) == 0.0       # colour-diagonal


def test_gamma5_hermiticity():
    dims = (4, 2, 2, 4)
    U = gauge_field(dims, 0.4, seed=11)
    D = dirac.dense_D(U, 0.1, dims, -1)
    G5 = np.kron(np.eye(geometry.volume(dims)), gamma.spin_colour(gamma.GAMMA5))
    assert np.max(np.abs(G5 @ D @ G5 - D.conj().T)) < 1e-15


def test_gauge_covariance():
    """U_mu(x) -> W(x) U_mu(x) W(x+mu)^dag maps D to W D W^dag: fixes which
    site's link each hop uses and where the dagger goes."""
    dims = (2, 4, 2, 4)
    V = geometry.volume(dims)
    U = gauge_field(dims, 0.7, seed=5)
    W = random_su3_transform(V, seed=6)
    Ug = np.empty_like(U)
    for mu in range(4):
        fwd, _ = geometry.neighbour(dims, mu, +1, 1)
        Ug[:, mu] = W @ U[:, mu] @ np.conj(np.transpose(W[fwd], (0, 2, 1)))
    D = dirac.dense_D(U, 0.05, dims, -1)
    Dg = dirac.dense_D(Ug, 0.05, dims, -1)
    Wbig = np.zeros((12 * V, 12 * V), dtype=complex)
    for x in range(V):
        Wbig[12 * x:12 * x + 12, 12 * x:12 * x + 12] = np.kron(np.eye(4), W[x])
    assert np.max(np.abs(Wbig @ D @ Wbig.conj().T - Dg)) < 1e-13


def test_apply_matches_dense_and_dagger():
    dims = (2, 2, 4, 2)
    V = geometry.volume(dims)
    U = gauge_field(dims, 0.5, seed=9)
    D = dirac.dense_D(U, 0.2, dims, -1)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal((V, 12, 3)) + 1j * rng.standard_normal((V, 12, 3))
    out = dirac.apply_D(U, 0.2, psi, dims, -1)
    assert np.allclose(out.reshape(12 * V, 3), D @ psi.reshape(12 * V, 3), atol=1e-14)
    outd = dirac.apply_D(U, 0.2, psi, dims, -1, dagger=True)
    assert np.allclose(outd.reshape(12 * V, 3), D.conj().T @ psi.reshape(12 * V, 3), atol=1e-14)


def test_bicgstab_matches_lu():
    dims = (4, 4, 4, 4)
    U = gauge_field(dims, 0.3, seed=1)
    A = dirac.sparse_D(U, 0.2, dims, -1)
    b = np.random.default_rng(2).standard_normal(A.shape[0]).astype(complex)
    x, it = solve.bicgstab(A, b, tol=1e-12)
    xd = solve.dense_solve(A.toarray(), b)
    assert it < 200
    assert np.linalg.norm(x - xd) < 1e-10 * np.linalg.norm(xd)


def test_exact_traces_real_by_gamma5_hermiticity():
    dims = (4, 4, 4, 4)
    U = gauge_field(dims, 0.3, seed=1)
    Dinv = solve.dense_inverse(dirac.dense_D(U, 0.2, dims, -1))
    tr = estimator.exact_trace(Dinv)
    assert abs(tr.imag) < 1e-10 * abs(tr)
    for t in range(4):
        o = estimator.exact_loop(Dinv, dims, t)
        assert abs(o.imag) < 1e-11


@pytest.mark.parametrize("dagger", [False, True])
def test_sampled_rows_match_sparse(dagger):
    dims = (4, 2, 2, 6)
    V = geometry.volume(dims)
    U = gauge_field(dims, 0.6, seed=12)
    rng = np.random.default_rng(1)
    psi = rng.standard_normal((V, 12, 2)) + 1j * rng.standard_normal((V, 12, 2))
    full = dirac.apply_D(U, 0.3, psi, dims, -1, dagger=dagger)
    sites = [0, 3, 17, 40, V - 1, 8, 88]
    part = dirac.apply_D_sites(U, 0.3, psi, dims, sites, -1, dagger=dagger)
    assert np.max(np.abs(part - full[sites])) < 1e-14


def test_apply_D_sites_row_function_matches_array():
    """The row-provider form of the sampled operator gives the same rows."""
    dims, N = (4, 2, 2, 4), 3
    V = int(np.prod(dims))
    U = gauge_field(dims, 0.4, seed=12)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((V, 12, N)) + 1j * rng.standard_normal((V, 12, N))
    sites = [0, 5, V - 1, 17]
    a = dirac.apply_D_sites(U, 0.1, psi, dims, sites)
    b = dirac.apply_D_sites(U, 0.1, lambda s: psi[s], dims, sites)
    assert np.array_equal(a, b)
