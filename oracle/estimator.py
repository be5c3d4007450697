"""Trace estimators and exact traces.

- Hutchinson (Sec. 1, eq. Hutchinson-estimator): tr(D^-1) ~ (1/N) sum_i
  eta_i^dag D^-1 eta_i.
- Probing with dilution (Sec. 3, eq. Hutchinson-probing-estimator, read with
  the dagger the printed formula lacks): tr(D^-1) ~ sum_j (1/N) sum_i
  v_j^(i)dag D^-1 v_j^(i), one term per colour j and dilution component.
- Rademacher variance (Sec. 1, eq. hutchinson-variance):
  V[eta^dag A eta] = 1/2 ||offdiag(A + A^T)||_F^2, with V the complex variance
  E|X - EX|^2.
- Observables (Sec. 4): the disconnected loop O(t) = tr[Gamma5 D^-1(t,t)] and
  the slice-to-slice correlator ||D^-1(t, 0)||_F^2 (the pseudoscalar function
  of eq. connected-results-G at source slice 0, using gamma5-hermiticity).

Spin insertion B acts on the 4 spin indices of a site (12x12 = B (x) 1_colour).
"""
import numpy as np

from .gamma import GAMMA5, spin_colour


def slice_sites(dims, t):
    Lxyz = dims[0] * dims[1] * dims[2]
    return np.arange(t * Lxyz, (t + 1) * Lxyz)


def slice_mask(dims, t):
    """Boolean mask over the n = 12 V components selecting time slice t."""
    V = int(np.prod(dims))
    m = np.zeros((V, 12), dtype=bool)
    m[slice_sites(dims, t)] = True
    return m.ravel()


def exact_trace(Dinv):
    return np.trace(Dinv)


def exact_slice_trace(Dinv, dims, t, spin=None):
    """tr[B D^-1(t,t)] over the sites of slice t, B a 4x4 spin matrix (default 1)."""
    B = spin_colour(np.eye(4) if spin is None else spin)
    tot = 0j
    for s in slice_sites(dims, t):
        blk = Dinv[12 * s:12 * s + 12, 12 * s:12 * s + 12]
        tot += np.trace(B @ blk)
    return tot


def exact_loop(Dinv, dims, t):
    """O(t) = tr[Gamma5 D^-1(t,t)]."""
    return exact_slice_trace(Dinv, dims, t, GAMMA5)


def exact_correlator(Dinv, dims, t, t0=0):
    """||D^-1(t, t0)||_F^2: squared entries of the (t, t0) time-slice block."""
    rows = slice_mask(dims, t)
    cols = slice_mask(dims, t0)
    blk = Dinv[np.ix_(rows, cols)]
    return float(np.sum(np.abs(blk) ** 2))


def exact_G(Dinv, dims, t):
    """G(t) = (1/T) sum_t' tr[D^-1(t+t', t') Gamma5 D^-1(t', t+t') Gamma5] (Sec. 4,
    eq. connected-results-G), time indices mod T, written out block by block."""
    T = dims[3]
    G5 = spin_colour(GAMMA5)
    V = Dinv.shape[0] // 12
    g5 = np.kron(np.eye(V // T), G5)  # Gamma5 on one time slice
    tot = 0j
    for tp in range(T):
        a, b = slice_mask(dims, (t + tp) % T), slice_mask(dims, tp)
        A = Dinv[np.ix_(a, b)]        # D^-1(t+t', t')
        B = Dinv[np.ix_(b, a)]        # D^-1(t', t+t')
        tot += np.trace(A @ g5 @ B @ g5)
    return tot / T


def sample_dot(v, x, dims=None, t=None, spin=None):
    """One sample sum conj(v) (B x) over the whole lattice or slice t.

    v, x: [V, 12] arrays.  B a 4x4 spin matrix (default identity)."""
    B = spin_colour(np.eye(4) if spin is None else spin)
    v = np.asarray(v).reshape(-1, 12)
    x = np.asarray(x).reshape(-1, 12)
    if t is not None:
        sites = slice_sites(dims, t)
        v, x = v[sites], x[sites]
    return np.sum(np.conj(v) * (x @ B.T))


def sample_norm2_per_t(x, dims):
    """sum_{sites in t} ||x||^2 for every t = 0..Lt-1 ([V, 12] input)."""
    x = np.asarray(x).reshape(dims[3], -1)
    return np.sum(np.abs(x) ** 2, axis=1)


def hutchinson_variance(A):
    """1/2 ||offdiag(A + A^T)||_F^2 (exact variance for real Rademacher noise)."""
    S = A + A.T
    S = S - np.diag(np.diag(S))
    return 0.5 * float(np.sum(np.abs(S) ** 2))


def probing_variance(A, classes):
    """Exact variance of sum_k v_k^dag A v_k when v_k = eta restricted to class k
    and eta is one real Rademacher vector: only pairs (i, j), i != j, inside the
    same class contribute, each pair as |A_ij + A_ji|^2 (the same argument that
    gives the Rademacher formula, restricted to one class at a time)."""
    classes = np.asarray(classes)
    same = classes[:, None] == classes[None, :]
    S = A + A.T
    S = np.where(same, S, 0)
    S = S - np.diag(np.diag(S))
    return 0.5 * float(np.sum(np.abs(S) ** 2))


def sample_variance(samples):
    """Unbiased complex sample variance (N - 1 normalisation) of E|X - EX|^2."""
    s = np.asarray(samples)
    return float(np.sum(np.abs(s - s.mean()) ** 2) / (len(s) - 1))
