"""Random SU(3) gauge links U = reunit(expm(i*eps*H)).

The paper measures on a real QCD ensemble that is not available here; these
synthetic links stand in for it.  H = sum_a g_a lambda_a / 2 is traceless
Hermitian with g_a drawn from a seeded unit Gaussian (numpy PCG64), draw order
site-lexicographic (x fastest), then direction mu = x, y, z, t, then a = 1..8.
eps = 0 gives the free field U = 1.

Layout returned: complex128 array [V, 4, 3, 3], link U_mu(x)[a, b] with the
site index x + Lx*(y + Ly*(z + Lz*t)).
"""
import numpy as np


def gell_mann():
    """The eight Gell-Mann matrices lambda_1..lambda_8 (3x3 complex)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0, 0, 1] = l[0, 1, 0] = 1
    l[1, 0, 1], l[1, 1, 0] = -1j, 1j
    l[2, 0, 0], l[2, 1, 1] = 1, -1
    l[3, 0, 2] = l[3, 2, 0] = 1
    l[4, 0, 2], l[4, 2, 0] = -1j, 1j
    l[5, 1, 2] = l[5, 2, 1] = 1
    l[6, 1, 2], l[6, 2, 1] = -1j, 1j
    l[7, 0, 0] = l[7, 1, 1] = 1 / np.sqrt(3)
    l[7, 2, 2] = -2 / np.sqrt(3)
    return l


def reunitarise(u):
    """Project [..., 3, 3] matrices back onto SU(3) row by row.

    Row 0 is normalised, row 1 is Gram-Schmidt orthogonalised against row 0
    and normalised, row 2 = conj(row0 x row1) so that det U = 1.
    """
    u = np.array(u, dtype=np.complex128, copy=True)
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def gauge_field(dims, eps, seed, chunk=1 << 18):
    """Seeded SU(3) links for a lattice of extent dims = (Lx, Ly, Lz, Lt)."""
    dims = tuple(int(d) for d in dims)
    V = int(np.prod(dims))
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = gell_mann() / 2
    out = np.empty((V, 4, 3, 3), dtype=np.complex128)
    nlinks = V * 4
    flat = out.reshape(nlinks, 3, 3)
    for lo in range(0, nlinks, chunk):
        hi = min(nlinks, lo + chunk)
        g = rng.standard_normal((hi - lo, 8))
        if eps == 0.0:
            flat[lo:hi] = np.eye(3)
            continue
        H = np.einsum("na,aij->nij", g, lam)
        w, Q = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        U = np.einsum("nij,nj,nkj->nik", Q, ph, np.conj(Q))
        flat[lo:hi] = reunitarise(U)
    return out


def random_su3_transform(V, seed):
    """Seeded SU(3) matrices Omega(x), one per site (for gauge-covariance tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((V, 3, 3)) + 1j * rng.standard_normal((V, 3, 3))
    return reunitarise(z)
