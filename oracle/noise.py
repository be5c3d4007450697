"""Stochastic vectors: Rademacher noise and probing vectors with dilution.

Noise (Sec. 1): every component is +1 or -1 with probability 1/2.  The paper
does not fix a generator; this build draws the sign of component g of the
vector with seed `seed` from the counter-based SplitMix64 generator of Steele,
Lea and Flood (OOPSLA 2014):

    c     = seed * 2^40 + g                 (the counter)
    z     = (c + 1) * 0x9E3779B97F4A7C15     (mod 2^64), i.e. the (c+1)-th
            output state of SplitMix64 started from state 0
    z     = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z     = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z     =  z ^ (z >> 31)
    eta_g = +1 if the top bit of z is 0, else -1.

g = 12*site + 3*spin + colour ranges over the whole lattice; the same eta
underlies every colour and dilution mask of one seed.

Probing (Sec. 3, eq. "probing vectors"): v_j = eta restricted to the sites of
colour j.  Dilution (Sec. 3, last paragraph): the probing vector is further
restricted to one spin-colour component k (12-fold dilution) and/or one time
slice t0 (time dilution).
"""
import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1


def mix64(z):
    """SplitMix64 output function on one Python int (mod 2^64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def splitmix64_stream(state, count):
    """The first `count` outputs of SplitMix64 started from `state` (Python ints)."""
    out = []
    for _ in range(count):
        state = (state + GOLDEN) & MASK64
        out.append(mix64(state))
    return out


def noise_word(seed, g):
    """The 64-bit word behind component g of noise vector `seed` (scalar form)."""
    c = (seed << 40) + g
    return mix64(((c + 1) * GOLDEN) & MASK64)


def rademacher_scalar(seed, g):
    return 1.0 if (noise_word(seed, g) >> 63) == 0 else -1.0


def _mix64_np(z):
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(M1)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def rademacher(seed, n):
    """eta_seed as a float64 array of length n (vectorised form of the above)."""
    with np.errstate(over="ignore"):
        c = (np.uint64(seed) << np.uint64(40)) + np.arange(n, dtype=np.uint64)
        z = (c + np.uint64(1)) * np.uint64(GOLDEN)
        z = _mix64_np(z)
    return np.where((z >> np.uint64(63)) == 0, 1.0, -1.0)


def rademacher_at(seed, g):
    """eta_seed at the global indices g (an integer array): the same formula
    as rademacher(), for vectors too long to form whole."""
    with np.errstate(over="ignore"):
        c = (np.uint64(seed) << np.uint64(40)) + np.asarray(g, dtype=np.uint64)
        z = (c + np.uint64(1)) * np.uint64(GOLDEN)
        z = _mix64_np(z)
    return np.where((z >> np.uint64(63)) == 0, 1.0, -1.0)


def probing_vector(dims, seed, colours=None, colour=None, component=-1, t0=-1):
    """Source vector [V, 12] (float64 +-1 / 0).

    colours   : per-site colour array (None: no probing, all sites kept)
    colour    : which colour class j to keep
    component : spin-colour dilution component k = 3*spin + colour, or -1
    t0        : time slice kept by time dilution, or -1
    """
    V = int(np.prod(dims))
    eta = rademacher(seed, 12 * V).reshape(V, 12)
    keep = np.ones((V, 12), dtype=bool)
    if colours is not None:
        keep &= (np.asarray(colours) == colour)[:, None]
    if component >= 0:
        m = np.zeros(12, dtype=bool)
        m[component] = True
        keep &= m[None, :]
    if t0 >= 0:
        Lxyz = dims[0] * dims[1] * dims[2]
        t = np.arange(V) // Lxyz
        keep &= (t == t0)[:, None]
    return np.where(keep, eta, 0.0)
