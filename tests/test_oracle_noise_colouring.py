"""Pins of the oracle's noise generator (published SplitMix64 outputs) and of
the torus colouring (Table 1 of the paper, plus brute force on small lattices)."""
import json
import os

import numpy as np
import pytest

from oracle import colouring, geometry, noise

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    g = json.load(open(os.path.join(GOLD, "splitmix64.json")))
    s0 = g["streams"][0]
    assert noise.splitmix64_stream(0, 3) == [int(h, 16) for h in s0["outputs_hex"]]
    s1 = g["streams"][1]
    assert noise.splitmix64_stream(1234567, 3) == s1["outputs_dec"]
    # the noise word of counter c is the (c+1)-th output from state 0
    stream = noise.splitmix64_stream(0, 5)
    for g_ in range(5):
        assert noise.noise_word(0, g_) == stream[g_]


def test_rademacher_vectorised_matches_scalar():
    for seed in (0, 1, 7, 123456):
        r = noise.rademacher(seed, 4096)
        assert np.array_equal(r, [noise.rademacher_scalar(seed, g) for g in range(4096)])


def test_rademacher_statistics():
    r = np.stack([noise.rademacher(s, 1 << 16) for s in range(4)])
    assert set(np.unique(r)) == {-1.0, 1.0}
    assert abs(r.mean()) < 5 / np.sqrt(r.size)
    # E[eta_j eta_k] = delta_jk: neighbouring components and different seeds
    assert abs(np.mean(r[:, 1:] * r[:, :-1])) < 5 / np.sqrt(r[:, 1:].size)
    assert abs(np.mean(r[0] * r[1])) < 5 / np.sqrt(r.shape[1])


def test_probing_vectors_partition_the_noise():
    dims = (4, 4, 2, 4)
    V = geometry.volume(dims)
    nc, sig = colouring.search(dims, 2)
    col = colouring.colours(dims, sig, nc)
    eta = noise.rademacher(5, 12 * V).reshape(V, 12)
    tot = np.zeros((V, 12))
    for j in range(nc):
        for k in range(12):
            v = noise.probing_vector(dims, 5, col, j, k, t0=1)
            assert np.count_nonzero(tot[v != 0]) == 0       # disjoint supports
            tot += v
    keep = np.zeros((V, 12))
    keep[np.arange(V) // (dims[0] * dims[1] * dims[2]) == 1] = 1
    assert np.array_equal(tot, eta * keep)
    # one colour, no dilution, no time dilution with n_c = 1 is plain Hutchinson
    v = noise.probing_vector(dims, 5, np.zeros(V, int), 0)
    assert np.array_equal(v, eta)


def test_table1_colour_counts():
    g = json.load(open(os.path.join(GOLD, "table1_colours.json")))
    for d, nc in g["n_c_3d"].items():
        assert colouring.search(tuple(g["torus_3d"]), int(d))[0] == nc
    for d, nc in g["n_c_4d"].items():
        got = colouring.search(tuple(g["torus_4d"]), int(d))[0]
        if d == "2":
            assert got == 16 and nc == 10     # erratum: see the fixture
        else:
            assert got == nc


@pytest.mark.parametrize("dims,d", [((4, 4, 4, 4), 1), ((4, 4, 4, 4), 2),
                                    ((6, 4, 4, 8), 2), ((8, 8, 4, 4), 3),
                                    ((6, 6, 6, 6), 3), ((8, 8, 8, 8), 3),
                                    ((4, 4, 8, 8), 2), ((5, 4, 4, 4), 1)])
def test_colouring_valid_by_brute_force(dims, d):
    nc, sig = colouring.search(dims, d)
    col = colouring.colours(dims, sig, nc)
    assert colouring.check_pairs(dims, col, d)


def test_brute_force_catches_a_bad_colouring():
    dims = (4, 4, 4, 4)
    nc, sig = colouring.search(dims, 2)
    bad = colouring.colours(dims, (sig[0], sig[1], sig[2], (sig[3] + 1) % nc), nc)
    assert not colouring.check_pairs(dims, bad, 2)


def _first_valid_python(dims, d):
    """Independent tiny search: every sigma, every pair of sites."""
    V = geometry.volume(dims)
    c = geometry.coords(dims)
    close = [(i, j) for i in range(V) for j in range(i + 1, V)
             if geometry.torus_distance(dims, c[i], c[j]) <= d]
    I = np.array([p[0] for p in close])
    J = np.array([p[1] for p in close])
    for nc in range(2, V + 1):
        for s in np.ndindex(*([nc] * 4)):
            col = (c @ np.array(s)) % nc
            if np.all(col[I] != col[J]):
                return nc, tuple(int(v) for v in s)


@pytest.mark.parametrize("dims,d", [((4, 2, 2, 4), 1), ((4, 4, 2, 2), 2), ((3, 2, 2, 4), 1)])
def test_search_is_first_valid(dims, d):
    assert colouring.search(dims, d) == _first_valid_python(dims, d)


def test_rademacher_at_matches_whole_vector():
    from oracle import noise
    g = np.array([0, 1, 5, 1000, 12 * 300 - 1])
    for seed in (0, 3, 2 ** 24 - 1):
        assert np.array_equal(noise.rademacher_at(seed, g), noise.rademacher(seed, 12 * 300)[g])
