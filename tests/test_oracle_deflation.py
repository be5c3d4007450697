"""Pins of the deflation oracle (Sec. 2, eq. defl-split) against facts that do
not go through its own formulas: the dense trace of B D^-1, singular values of
D, the spectral norm of the deflated inverse, and exact unit-vector probing."""
import numpy as np
import pytest

from oracle import deflation as dfl, dirac, estimator
from oracle.gamma import GAMMA5
from oracle.solve import dense_inverse
from synth.gauge import gauge_field


@pytest.fixture(scope="module")
def small():
    dims, m0 = (2, 2, 2, 4), 0.05
    U = gauge_field(dims, 0.5, seed=11)
    D = dirac.dense_D(U, m0, dims, -1)
    return dims, D, dense_inverse(D)


def test_q_hermitian_and_spectrum_is_singular_values_of_D(small):
    dims, D, _ = small
    Q = dfl.q_matrix(D)
    assert np.max(np.abs(Q - Q.conj().T)) < 1e-13
    lam, _ = dfl.low_modes(Q, Q.shape[0])
    sv = np.linalg.svd(D, compute_uv=False)
    assert np.allclose(np.sort(np.abs(lam)), np.sort(sv), rtol=1e-10, atol=1e-12)
    # ordered by magnitude
    assert np.all(np.diff(np.abs(lam)) >= -1e-14)


@pytest.mark.parametrize("k", [1, 6, 40])
@pytest.mark.parametrize("where", ["lattice", "slice"])
def test_split_reproduces_dense_trace(small, k, where):
    """exact part + stochastic part = tr(B D^-1), B = 1 on the lattice or
    gamma5 on slice 1 (the loop O(1))."""
    dims, D, Dinv = small
    lam, Vk = dfl.low_modes(dfl.q_matrix(D), k)
    if where == "lattice":
        t, spin, ref = None, None, np.trace(Dinv)
    else:
        t, spin, ref = 1, GAMMA5, estimator.exact_loop(Dinv, dims, 1)
    tot = dfl.exact_part(lam, Vk, dims, t, spin) + dfl.stochastic_trace(Dinv, Vk, dims, t, spin)
    assert abs(tot - ref) < 1e-11 * max(1.0, abs(ref))


@pytest.mark.parametrize("where", ["lattice", "slice"])
def test_split_holds_for_any_orthonormal_basis(small, where):
    """With the low-mode part taken by solves, the split is exact for any
    orthonormal V_k (here random), and for eigenvectors the solve form
    equals the eigenvalue form."""
    dims, D, Dinv = small
    n = D.shape[0]
    rng = np.random.default_rng(5)
    Vr, _ = np.linalg.qr(rng.standard_normal((n, 7)) + 1j * rng.standard_normal((n, 7)))
    if where == "lattice":
        t, spin, ref = None, None, np.trace(Dinv)
    else:
        t, spin, ref = 3, GAMMA5, estimator.exact_loop(Dinv, dims, 3)
    tot = dfl.exact_part_solves(Dinv, Vr, dims, t, spin) + dfl.stochastic_trace(Dinv, Vr, dims, t, spin)
    assert abs(tot - ref) < 1e-11 * max(1.0, abs(ref))
    lam, Vk = dfl.low_modes(dfl.q_matrix(D), 9)
    a = dfl.exact_part_solves(Dinv, Vk, dims, t, spin)
    b = dfl.exact_part(lam, Vk, dims, t, spin)
    assert abs(a - b) < 1e-11 * max(1.0, abs(b))


def test_full_deflation_leaves_nothing_to_sample(small):
    dims, D, Dinv = small
    n = D.shape[0]
    lam, Vk = dfl.low_modes(dfl.q_matrix(D), n)
    assert np.max(np.abs(dfl.deflated_operator(Dinv, Vk))) < 1e-10
    assert abs(dfl.exact_part(lam, Vk, dims) - np.trace(Dinv)) < 1e-10 * abs(np.trace(Dinv))


@pytest.mark.parametrize("k", [0, 3, 12])
def test_deflated_inverse_norm_is_one_over_next_mode(small, k):
    """||D^-1 (I - Gamma5 Pi Gamma5)||_2 = 1 / |lambda_{k+1}|: the k modes of
    smallest |lambda| are removed and nothing else."""
    dims, D, Dinv = small
    lam_all, _ = dfl.low_modes(dfl.q_matrix(D), D.shape[0])
    lam, Vk = dfl.low_modes(dfl.q_matrix(D), k)
    nrm = np.linalg.norm(dfl.deflated_operator(Dinv, Vk), 2)
    assert abs(nrm - 1.0 / abs(lam_all[k])) < 1e-9 * nrm


def test_unit_vector_probing_of_samples_gives_stochastic_trace(small):
    """Summing the sample over the unit vectors of slice 2 (full probing x
    dilution) gives the stochastic part's trace exactly."""
    dims, D, Dinv = small
    lam, Vk = dfl.low_modes(dfl.q_matrix(D), 5)
    n = D.shape[0]
    rows = np.nonzero(estimator.slice_mask(dims, 2))[0]
    tot = 0j
    for r in rows:
        e = np.zeros(n, dtype=complex)
        e[r] = 1.0
        tot += dfl.deflated_sample(Dinv, Vk, e, dims, 2, GAMMA5)
    ref = dfl.stochastic_trace(Dinv, Vk, dims, 2, GAMMA5)
    assert abs(tot - ref) < 1e-11 * max(1.0, abs(ref))


def test_deflation_reduces_rademacher_variance(small):
    """Exact Rademacher variance of the slice-loop sample, undeflated against
    deflated with the 8 lowest modes (eq. hutchinson-variance restricted to
    the slice's components)."""
    dims, D, Dinv = small
    lam, Vk = dfl.low_modes(dfl.q_matrix(D), 8)
    rows = estimator.slice_mask(dims, 0)
    B = np.kron(np.eye(int(np.prod(dims))), np.kron(GAMMA5, np.eye(3)))
    A0 = (B @ Dinv)[np.ix_(rows, rows)]
    A1 = (B @ dfl.deflated_operator(Dinv, Vk))[np.ix_(rows, rows)]
    assert estimator.hutchinson_variance(A1) < estimator.hutchinson_variance(A0)
