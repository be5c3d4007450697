"""Pins of the oracle's estimators: exact enumeration over every Rademacher
vector of tiny matrices (mean = trace, variance = the Sec. 1 formula and its
probing generalisation), exactness of full probing with dilution, and the
free-field correlator against a momentum-space FFT."""
import itertools

import numpy as np
import pytest

from oracle import colouring, dirac, estimator, gamma, geometry, noise, solve
from synth.gauge import gauge_field


def _all_signs(n):
    return np.array(list(itertools.product([1.0, -1.0], repeat=n)))


def test_variance_formula_exact_enumeration():
    rng = np.random.default_rng(3)
    n = 10
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    E = _all_signs(n)
    X = np.einsum("ki,ij,kj->k", E, A, E)
    assert abs(X.mean() - np.trace(A)) < 1e-12            # unbiased (Hutchinson identity)
    var = np.mean(np.abs(X - X.mean()) ** 2)
    assert abs(var - estimator.hutchinson_variance(A)) < 1e-10 * var


def test_probing_variance_exact_enumeration():
    rng = np.random.default_rng(4)
    n = 10
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    classes = np.array([0, 1, 2, 0, 1, 2, 0, 1, 2, 0])
    E = _all_signs(n)
    X = np.zeros(len(E), dtype=complex)
    for c in range(3):
        m = (classes == c).astype(float)
        X += np.einsum("ki,ij,kj->k", E * m, A, E * m)
    assert abs(X.mean() - np.trace(A)) < 1e-12
    var = np.mean(np.abs(X - X.mean()) ** 2)
    assert abs(var - estimator.probing_variance(A, classes)) < 1e-10 * var
    # one class reduces to the plain formula; all-distinct classes give zero
    assert np.isclose(estimator.probing_variance(A, np.zeros(n)), estimator.hutchinson_variance(A))
    assert estimator.probing_variance(A, np.arange(n)) == 0.0


@pytest.fixture(scope="module")
def small_system():
    dims = (4, 4, 4, 4)
    U = gauge_field(dims, 0.3, seed=1)
    D = dirac.dense_D(U, 0.2, dims, -1)
    Dinv = solve.dense_inverse(D)
    return dims, U, D, Dinv


def test_full_probing_with_dilution_is_exact(small_system):
    """Full colouring (n_c = V, one site per colour) x 12 spin-colour dilution:
    each vector has one nonzero, so the estimator returns the exact trace."""
    dims = (2, 2, 2, 4)
    V = geometry.volume(dims)
    U = gauge_field(dims, 0.4, seed=2)
    Dinv = solve.dense_inverse(dirac.dense_D(U, 0.1, dims, -1))
    col = colouring.colours(dims, (1, 2, 4, 8), V)
    assert len(np.unique(col)) == V
    tot = 0j
    loop = 0j
    for j in range(V):
        for k in range(12):
            v = noise.probing_vector(dims, 3, col, j, k).ravel()
            x = Dinv @ v
            tot += np.vdot(v, x)
            loop += estimator.sample_dot(v, x, dims, t=1, spin=gamma.GAMMA5)
    assert abs(tot - np.trace(Dinv)) < 1e-12 * abs(np.trace(Dinv))
    assert abs(loop - estimator.exact_loop(Dinv, dims, 1)) < 1e-12


def test_hutchinson_variance_matches_sample(small_system):
    dims, U, D, Dinv = small_system
    V = geometry.volume(dims)
    N = 1500
    Eta = np.stack([noise.rademacher(s, 12 * V) for s in range(N)], axis=1)
    X = np.einsum("ik,ik->k", Eta, Dinv @ Eta)
    vs = estimator.sample_variance(X)
    vf = estimator.hutchinson_variance(Dinv)
    assert abs(vs - vf) < 0.12 * vf
    assert abs(X.mean() - np.trace(Dinv)) < 5 * np.sqrt(vf / N)


def test_probing_reduces_variance_as_formula_says(small_system):
    dims, U, D, Dinv = small_system
    V = geometry.volume(dims)
    nc, sig = colouring.search(dims, 1)
    col = colouring.colours(dims, sig, nc)
    site_class = np.repeat(col, 12)
    dil_class = site_class * 12 + np.tile(np.arange(12), V)
    v_plain = estimator.hutchinson_variance(Dinv)
    v_prob = estimator.probing_variance(Dinv, site_class)
    v_dil = estimator.probing_variance(Dinv, dil_class)
    assert v_dil < v_prob < v_plain
    # sample check of the probed + diluted variance with the oracle's own vectors
    N = 300
    S = []
    for s in range(N):
        Vm = np.stack([noise.probing_vector(dims, s, col, j, k).ravel()
                       for j in range(nc) for k in range(12)], axis=1)
        S.append(np.sum(np.conj(Vm) * (Dinv @ Vm)))
    S = np.array(S)
    assert abs(estimator.sample_variance(S) - v_dil) < 0.25 * v_dil
    assert abs(S.mean() - np.trace(Dinv)) < 5 * np.sqrt(v_dil / N)


def test_free_field_correlator_fft():
    """||D^-1(t, 0)||_F^2 from the dense inverse against the free propagator
    S(x) = FFT^-1[(M - i gamma.sin p)/(M^2 + s^2)], colour trace 3."""
    dims, m0 = (4, 4, 2, 6), 0.25
    V = geometry.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    Dinv = solve.dense_inverse(dirac.dense_D(U, m0, dims, -1))
    ks = [(2 * np.pi * np.arange(L) + (np.pi if mu == 3 else 0)) / L for mu, L in enumerate(dims)]
    P = np.meshgrid(*ks, indexing="ij")
    M = m0 + sum(1 - np.cos(p) for p in P)
    s2 = sum(np.sin(p) ** 2 for p in P)
    Sp = (M[..., None, None] * np.eye(4)
          - 1j * sum(np.sin(P[m])[..., None, None] * gamma.GAMMA[m] for m in range(4)))
    Sp = Sp / (M ** 2 + s2)[..., None, None]
    Sx = np.fft.ifftn(Sp, axes=(0, 1, 2, 3))
    # sum over the source slice by translation invariance in space:
    # ||D^-1(t,0)||^2 = Lx Ly Lz * 3 * sum_{x in slice t} |S(x)|^2 (spin matrix)
    per_t = 3 * dims[0] * dims[1] * dims[2] * np.sum(np.abs(Sx) ** 2, axis=(0, 1, 2, 4, 5))
    for t in range(dims[3]):
        assert abs(estimator.exact_correlator(Dinv, dims, t) - per_t[t]) < 1e-11 * per_t[t]


def test_time_diluted_correlator_estimator_unbiased_exact_limit():
    """Summing sum_t ||D^-1 v|_t||^2 over a full set of point sources on slice 0
    gives ||D^-1(t, 0)||_F^2 exactly."""
    dims = (2, 2, 2, 4)
    V = geometry.volume(dims)
    U = gauge_field(dims, 0.5, seed=8)
    Dinv = solve.dense_inverse(dirac.dense_D(U, 0.1, dims, -1))
    col = colouring.colours(dims, (1, 2, 4, 8), V)
    acc = np.zeros(dims[3])
    for j in range(V):
        for k in range(12):
            v = noise.probing_vector(dims, 0, col, j, k, t0=0)
            if not v.any():
                continue
            x = (Dinv @ v.ravel()).reshape(V, 12)
            acc += estimator.sample_norm2_per_t(x, dims)
    for t in range(dims[3]):
        assert abs(acc[t] - estimator.exact_correlator(Dinv, dims, t, 0)) < 1e-12 * acc[t]


def test_connected_G_is_average_of_slice_frobenius_norms():
    """eq. connected-results-G written with Gamma5 equals (1/T) sum_t'
    ||D^-1(t+t', t')||_F^2 (gamma5-hermiticity), and is real and positive."""
    from oracle import dirac
    from oracle.solve import dense_inverse
    from synth.gauge import gauge_field
    dims, m0 = (2, 2, 2, 6), 0.1
    U = gauge_field(dims, 0.5, seed=3)
    Dinv = dense_inverse(dirac.dense_D(U, m0, dims, -1))
    T = dims[3]
    for t in range(T):
        g = estimator.exact_G(Dinv, dims, t)
        ref = sum(estimator.exact_correlator(Dinv, dims, (t + tp) % T, tp) for tp in range(T)) / T
        assert abs(g.imag) < 1e-12 * abs(g)
        assert abs(g.real - ref) < 1e-12 * ref
        assert ref > 0
