"""Torus colouring (Sec. 3, eq. coloring-formula): c(x) = sum_j sigma_j x_j mod n_c.

`search` wraps the exhaustive search in colour_search.c (built into
oracle/_colour_search.so by the build step); `check_pairs` is an independent
brute-force verifier over all site pairs of a small lattice.
"""
import ctypes
import os
import subprocess

import numpy as np

from .geometry import coords, torus_distance

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_colour_search.so")
_SRC = os.path.join(_HERE, "colour_search.c")


def build():
    """Compile the C search with gcc (plain C, no GPU)."""
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", _SO, _SRC])


def _lib():
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_SO)
    lib.oracle_colour_search.restype = ctypes.c_int
    lib.oracle_colour_search.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]
    return lib


def search(dims, d, max_nc=4096):
    """(n_c, sigma) of the first valid linear colouring; dims lists the extents
    of the n_D coordinates being coloured (4 on the whole lattice, 3 on a slice)."""
    nD = len(dims)
    L = (ctypes.c_int32 * nD)(*dims)
    nc = ctypes.c_int32(0)
    sig = (ctypes.c_int32 * 4)()
    rc = _lib().oracle_colour_search(L, nD, d, max_nc, ctypes.byref(nc), sig)
    if rc != 0:
        raise ValueError(f"no torus colouring with n_c <= {max_nc} (rc={rc})")
    return nc.value, tuple(sig[j] for j in range(nD))


def colours(dims, sigma, n_c):
    """Per-site colour array [V] of the 4D colouring on lattice dims."""
    c = coords(dims)
    s = np.asarray(sigma, dtype=np.int64)
    return (c[:, : len(s)] @ s) % n_c


def check_pairs(dims, col, d, chunk=256):
    """True iff every pair of distinct sites at periodic L1 distance <= d has
    different colours (brute force over all pairs; small lattices only)."""
    c = coords(dims)
    col = np.asarray(col)
    V = len(c)
    for lo in range(0, V, chunk):
        hi = min(V, lo + chunk)
        dist = torus_distance(dims, c[lo:hi, None, :], c[None, :, :])
        near = dist <= d
        near[np.arange(hi - lo), np.arange(lo, hi)] = False
        same = col[lo:hi, None] == col[None, :]
        if np.any(near & same):
            return False
    return True
