"""The Wilson-Dirac matrix D (Sec. 1: 12x12 spin-colour block per site,
nearest-neighbour couplings on the periodic lattice).

The paper does not print D; this oracle takes the Wilson form with r = 1, no
clover term, and the bare mass m0 in the (4 + m0) normalisation:

    (D psi)(x) = (4 + m0) psi(x)
                 - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x)        psi(x + mu)
                               + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ],

with the time-boundary factor bc_t on hops that cross t = Lt-1 <-> 0.
gamma5 D gamma5 = D^dag (the Hermiticity of Q = Gamma5 D in Sec. 2) holds for
this form and is checked by the tests.

Global index of a component: 12*site + 3*spin + colour.
"""
import numpy as np
import scipy.sparse as sp

from .gamma import GAMMA, ID4
from .geometry import volume, neighbour


def _hop_triplets(U, dims, bc_t):
    """COO rows, cols and values of the hopping part, including the -1/2."""
    V = volume(dims)
    rows, cols, vals = [], [], []
    ii, jj = np.meshgrid(np.arange(12), np.arange(12), indexing="ij")
    for mu in range(4):
        fwd, ph_f = neighbour(dims, mu, +1, bc_t)
        bwd, ph_b = neighbour(dims, mu, -1, bc_t)
        Pm = ID4 - GAMMA[mu]
        Pp = ID4 + GAMMA[mu]
        # forward: (1 - gamma_mu) (x) U_mu(x), coupling x -> x + mu
        blk = np.einsum("st,xab->xsatb", Pm, U[:, mu]).reshape(V, 12, 12)
        blk *= (-0.5 * ph_f)[:, None, None]
        rows.append((12 * np.arange(V)[:, None, None] + ii).ravel())
        cols.append((12 * fwd[:, None, None] + jj).ravel())
        vals.append(blk.ravel())
        # backward: (1 + gamma_mu) (x) U_mu(x - mu)^dag, coupling x -> x - mu
        Ub = np.conj(np.transpose(U[bwd, mu], (0, 2, 1)))
        blk = np.einsum("st,xab->xsatb", Pp, Ub).reshape(V, 12, 12)
        blk *= (-0.5 * ph_b)[:, None, None]
        rows.append((12 * np.arange(V)[:, None, None] + ii).ravel())
        cols.append((12 * bwd[:, None, None] + jj).ravel())
        vals.append(blk.ravel())
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def sparse_D(U, m0, dims, bc_t=-1):
    """D as a scipy CSR matrix (duplicate entries, e.g. for extent 2, are summed)."""
    U = np.asarray(U, dtype=np.complex128)
    n = 12 * volume(dims)
    r, c, v = _hop_triplets(U, dims, bc_t)
    H = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    return (H + (4.0 + m0) * sp.identity(n, dtype=np.complex128, format="csr")).tocsr()


def dense_D(U, m0, dims, bc_t=-1):
    """D as a dense complex128 matrix (tiny lattices only: n = 12 V)."""
    return sparse_D(U, m0, dims, bc_t).toarray()


def apply_D_sites(U, m0, psi, dims, sites, bc_t=-1, dagger=False):
    """(D psi)(x) (or D^dag) at the listed sites only, straight from the
    definition above: for lattices too large for a whole matrix.

    psi: [V, 12, N] array, or a function site -> [12, N] row (for inputs too
    large to hold); returns [len(sites), 12, N]."""
    from .geometry import coords
    U = np.asarray(U)
    if callable(psi):
        row = psi
    else:
        arr = np.asarray(psi)
        row = lambda s: arr[s]
    c = coords(dims)
    L = np.asarray(dims)
    strides = [1, dims[0], dims[0] * dims[1], dims[0] * dims[1] * dims[2]]
    out = []
    sgn = +1 if dagger else -1          # forward projector (1 + sgn gamma)
    for s in sites:
        acc = (4.0 + m0) * row(s)
        for mu in range(4):
            cm = c[s, mu]
            f = s + strides[mu] if cm < L[mu] - 1 else s - (L[mu] - 1) * strides[mu]
            b = s - strides[mu] if cm > 0 else s + (L[mu] - 1) * strides[mu]
            phf = bc_t if (mu == 3 and cm == L[mu] - 1) else 1.0
            phb = bc_t if (mu == 3 and cm == 0) else 1.0
            Pf = ID4 + sgn * GAMMA[mu]
            Pb = ID4 - sgn * GAMMA[mu]
            hf = np.einsum("st,ab,tbn->san", Pf, U[s, mu], row(f).reshape(4, 3, -1))
            hb = np.einsum("st,ba,tbn->san", Pb, np.conj(U[b, mu]), row(b).reshape(4, 3, -1))
            acc = acc - 0.5 * (phf * hf + phb * hb).reshape(12, -1)
        out.append(acc)
    return np.stack(out)


def apply_D(U, m0, psi, dims, bc_t=-1, dagger=False):
    """D psi (or D^dag psi) for psi of shape [V, 12] or [V, 12, N]."""
    A = sparse_D(U, m0, dims, bc_t)
    if dagger:
        A = A.conj().T.tocsr()
    psi = np.asarray(psi, dtype=np.complex128)
    V = volume(dims)
    flat = psi.reshape(12 * V, -1)
    return (A @ flat).reshape(psi.shape)
