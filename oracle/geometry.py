"""Lattice geometry: site index x + Lx*(y + Ly*(z + Lz*t)), so each time slice
is a contiguous block of Lx*Ly*Lz sites.  Periodic in space; in time the hop
across the t = Lt-1 <-> 0 boundary carries the factor bc_t (+1 periodic,
-1 antiperiodic), applied to the hop and never stored in the links.
"""
import numpy as np


def volume(dims):
    return int(np.prod(dims))


def coords(dims):
    """[V, 4] integer coordinates (x, y, z, t) of every site, in index order."""
    Lx, Ly, Lz, Lt = dims
    s = np.arange(volume(dims))
    x = s % Lx
    y = (s // Lx) % Ly
    z = (s // (Lx * Ly)) % Lz
    t = s // (Lx * Ly * Lz)
    return np.stack([x, y, z, t], axis=1)


def site_index(dims, c):
    Lx, Ly, Lz, Lt = dims
    c = np.asarray(c)
    return c[..., 0] + Lx * (c[..., 1] + Ly * (c[..., 2] + Lz * c[..., 3]))


def neighbour(dims, mu, step, bc_t):
    """Index of x + step*mu_hat for every site and the boundary factor of that hop."""
    c = coords(dims)
    n = c.copy()
    n[:, mu] = (c[:, mu] + step) % dims[mu]
    phase = np.ones(len(c))
    if mu == 3:
        crossed = (c[:, 3] + step < 0) | (c[:, 3] + step >= dims[3])
        phase[crossed] = bc_t
    return site_index(dims, n), phase


def torus_distance(dims, a, b):
    """Periodic L1 (graph) distance between coordinate arrays a and b."""
    d = np.abs(np.asarray(a) - np.asarray(b))
    L = np.asarray(dims)
    return np.sum(np.minimum(d, L - d), axis=-1)
