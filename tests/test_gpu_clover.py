"""GPU parity of the clover-improved operator against the oracle, through the
C interface: the packed clover blocks, the operator in every storage
precision (both kernel shapes, D and D^dag), solves against dense LU (even-odd
preconditioned with the inverse odd-site blocks, and not), the
batched solver, the estimator's samples, and a full-size solve checked by the
oracle's residual at sampled sites.  Bars as for the plain operator: FP64
operator 1e-14 relative, FP32 2e-6, FP16 4e-3, BF16 2^-8 against the
BF16-rounded input; FP64 solves 1e-10, mixed solves 1e-8 after refinement to
1e-10."""
import numpy as np
import pytest

from oracle import clover, dirac, gamma, noise, solve as osolve
from synth.gauge import gauge_field
from test_gpu_parity import bf16_batch, fp16_batch, from_bf16_words, from_fp16, rand_batch, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

W = None


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device():
    global W
    from paper_2607_05157_amd import wdt
    W = wdt
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wdt.init(0)
    yield


def unpack(P):
    """[V, 2, 36] packed -> [V, 12, 12] (zero between the chiral blocks)."""
    V = P.shape[0]
    C = np.zeros((V, 12, 12), dtype=complex)
    iu = np.triu_indices(6, 1)
    for h in range(2):
        B = np.zeros((V, 6, 6), dtype=complex)
        B[:, np.arange(6), np.arange(6)] = P[:, h, :6]
        B[:, iu[0], iu[1]] = P[:, h, 6::2] + 1j * P[:, h, 7::2]
        B[:, iu[1], iu[0]] = P[:, h, 6::2] - 1j * P[:, h, 7::2]
        C[:, 6 * h:6 * h + 6, 6 * h:6 * h + 6] = B
    return C


def clover_ref(U, m0, psi, dims, csw, dagger=False):
    return dirac.apply_D(U, m0, psi, dims, -1, dagger=dagger) + clover.apply_clover(U, dims, csw, psi)


@pytest.mark.parametrize("dims,eps,csw", [((4, 4, 2, 6), 0.5, 1.7), ((3, 2, 5, 4), 0.8, -0.9),
                                          ((2, 2, 2, 2), 0.0, 1.0)])
def test_clover_blocks_match_oracle(dims, eps, csw):
    say("clover blocks", dims, eps, csw)
    U = gauge_field(dims, eps, seed=31)
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    g.set_clover(csw)
    got = unpack(g.clover_packed())
    ref = clover.clover_blocks(U, dims, csw)
    scale = max(np.max(np.abs(ref)), 1.0)
    # the oracle's blocks vanish between the chiralities; the packed form has
    # the diagonal's real part only (the oracle's imaginary part is rounding)
    assert np.max(np.abs(got - ref)) < 1e-14 * scale
    if eps == 0.0:
        assert np.max(np.abs(got)) == 0


@pytest.mark.parametrize("dims,N,dagger", [((4, 4, 2, 6), 1, False), ((4, 4, 2, 6), 48, False),
                                           ((4, 4, 2, 6), 48, True), ((3, 2, 5, 4), 70, False),
                                           ((3, 2, 5, 4), 64, True)])
def test_clover_operator_fp64(dims, N, dagger):
    say("clover apply_D fp64", dims, N, dagger)
    V = int(np.prod(dims))
    U = gauge_field(dims, 0.6, seed=32)
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    g.set_clover(1.3)
    psi = rand_batch(V, N, 3)
    out = lat.new_batch(N)
    W.apply_D(g, 0.1, to_dev(psi), out, N, W.FP64, dagger)
    torch.cuda.synchronize()
    ref = clover_ref(U, 0.1, psi, dims, 1.3, dagger)
    err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err < 1e-14, err


@pytest.mark.parametrize("N", [20, 48])
def test_clover_operator_low_precision(N):
    dims = (4, 4, 2, 6)
    say("clover apply_D low precision", N)
    V = int(np.prod(dims))
    U = gauge_field(dims, 0.5, seed=33)
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    g.set_clover(1.1)
    psi = rand_batch(V, N, 4)
    ref = clover_ref(U, 0.05, psi, dims, 1.1)
    x = torch.from_numpy(np.ascontiguousarray(psi.astype(np.complex64))).cuda()
    out = torch.zeros_like(x)
    W.apply_D(g, 0.05, x, out, N, W.FP32)
    err = np.max(np.abs(out.cpu().numpy().astype(np.complex128) - ref)) / np.max(np.abs(ref))
    assert err < 2e-6, ("fp32", err)
    x = fp16_batch(psi)
    out = torch.zeros_like(x)
    W.apply_D(g, 0.05, x, out, N, W.FP16)
    err = np.max(np.abs(from_fp16(out, V, N) - ref)) / np.max(np.abs(ref))
    assert err < 4e-3, ("fp16", err)
    x, psi_r = bf16_batch(psi)
    psi_r = psi_r.reshape(V, 12, N)
    for dagger in (False, True):
        ref = clover_ref(U, 0.05, psi_r, dims, 1.1, dagger)
        out = torch.zeros_like(x)
        W.apply_D(g, 0.05, x, out, N, W.BF16, dagger)
        res = from_bf16_words(out.cpu().numpy().view(np.uint32)).reshape(V, 12, N)
        err = np.max(np.abs(res - ref) / (np.abs(ref) + 1e-3 * np.max(np.abs(ref))))
        assert err < 2 ** -8, ("bf16", dagger, err)


@pytest.fixture(scope="module")
def c2():
    dims, m0, csw = (4, 4, 2, 4), 0.05, 1.4
    U = gauge_field(dims, 0.4, seed=34)
    Dinv = osolve.dense_inverse(clover.dense_D_clover(U, m0, dims, csw))
    return dims, m0, csw, U, Dinv


@pytest.mark.parametrize("prec", ["fp64", "fp16", "bf16"])
def test_clover_solve_and_samples_match_dense_lu(c2, prec):
    """Solutions and Hutchinson samples against the dense inverse of the
    clover operator, even-odd preconditioned (the inverse odd-site blocks) and
    on the whole lattice; the preconditioned solve takes fewer iterations."""
    dims, m0, csw, U, Dinv = c2
    V, N = int(np.prod(dims)), 24
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    g.set_clover(csw)
    b = lat.new_batch(N)
    W.sources(lat, W.source_descs(list(range(N))), b)
    E = np.stack([noise.rademacher(s, 12 * V) for s in range(N)], axis=1).astype(complex)
    assert np.array_equal(b.cpu().numpy().reshape(-1, N), E)
    X = Dinv @ E
    p = {"fp64": W.FP64, "fp16": W.FP16, "bf16": W.BF16}[prec]
    tol, bar = (1e-12, 1e-10) if prec == "fp64" else (1e-10, 1e-8)
    kw = {"inner_tol": 0.05} if prec == "bf16" else {}
    its = {}
    try:
        for eo in (1, 0):
            say("clover solve", prec, "even-odd", eo)
            W.set_launch_shape(even_odd=eo)
            x = lat.new_batch(N)
            rc, st = W.solve(g, m0, b, x, N, tol=tol, prec=p, **kw)
            assert rc == W.OK and all(s["converged"] for s in st)
            its[eo] = max(s["iterations"] for s in st)
            xs = x.cpu().numpy().reshape(-1, N)
            assert np.max(np.linalg.norm(xs - X, axis=0) / np.linalg.norm(X, axis=0)) < bar
            full = W.contract(lat, b, x, N).sum(axis=1)
            ref = np.einsum("ik,ik->k", np.conj(E), X)
            norms = np.linalg.norm(E, axis=0) * np.linalg.norm(X, axis=0)
            assert np.all(np.abs(full - ref) <= bar * norms)
    finally:
        W.set_launch_shape()
    assert its[1] < its[0], its


def test_clover_even_odd_mass_change_and_term_change(c2):
    """The inverse blocks follow m0 and the clover coefficient: solves with a
    second mass, then a new c_sw, then the first mass again all match their
    dense inverses."""
    dims, m0, csw, U, Dinv = c2
    V, N = int(np.prod(dims)), 6
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    b = lat.new_batch(N)
    W.sources(lat, W.source_descs([50 + k for k in range(N)]), b)
    bh = b.cpu().numpy().reshape(-1, N)
    last = None
    for mass, c in ((m0, csw), (0.3, csw), (0.3, 0.7), (m0, csw)):
        say("clover even-odd", mass, c)
        if c != last:
            g.set_clover(c)
            last = c
        x = lat.new_batch(N)
        rc, st = W.solve(g, mass, b, x, N, tol=1e-12, prec=W.FP64)
        assert rc == W.OK and all(s["converged"] for s in st)
        D = clover.dense_D_clover(U, mass, dims, c)
        r = bh - D @ x.cpu().numpy().reshape(-1, N)
        assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(bh, axis=0)) <= 1.01e-12


def test_clover_batched_next_to_plain_system(c2):
    """The batched solver with one clover system (even extents: solved on the
    whole lattice) beside a plain Wilson system (even-odd)."""
    dims, m0, csw, U, Dinv = c2
    say("clover batched")
    lat = W.Lattice(dims, -1)
    g1 = W.Gauge(lat, U)
    g1.set_clover(csw)
    U2 = gauge_field((4, 4, 4, 4), 0.3, seed=35)
    lat2 = W.Lattice((4, 4, 4, 4), -1)
    g2 = W.Gauge(lat2, U2)
    N1, N2 = 8, 5
    b1, b2 = lat.new_batch(N1), lat2.new_batch(N2)
    W.sources(lat, W.source_descs(list(range(N1))), b1)
    W.sources(lat2, W.source_descs([100 + k for k in range(N2)]), b2)
    B = W.Batch([g1, g2], [m0, 0.2], [N1, N2])
    x1, x2 = lat.new_batch(N1), lat2.new_batch(N2)
    rc, st = B.solve([b1, b2], [x1, x2], tol=1e-11)
    assert rc == W.OK and all(t["converged"] for t in st)
    X = Dinv @ b1.cpu().numpy().reshape(-1, N1)
    xs = x1.cpu().numpy().reshape(-1, N1)
    assert np.max(np.linalg.norm(xs - X, axis=0) / np.linalg.norm(X, axis=0)) < 1e-9
    r2 = b2.cpu().numpy() - dirac.apply_D(U2, 0.2, x2.cpu().numpy(), (4, 4, 4, 4), -1)
    assert np.max(np.linalg.norm(r2.reshape(-1, N2), axis=0)
                  / np.linalg.norm(b2.cpu().numpy().reshape(-1, N2), axis=0)) <= 1.01e-11


def test_clover_removed_and_force_rejected():
    dims, N = (4, 4, 2, 6), 16
    say("clover on/off")
    V = int(np.prod(dims))
    U = gauge_field(dims, 0.5, seed=36)
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    psi = to_dev(rand_batch(V, N, 5))
    plain = lat.new_batch(N)
    W.apply_D(g, 0.1, psi, plain, N, W.FP64)
    with pytest.raises(RuntimeError):
        g.clover_packed()
    g.set_clover(1.5)
    with_c = lat.new_batch(N)
    W.apply_D(g, 0.1, psi, with_c, N, W.FP64)
    assert not torch.equal(with_c, plain)
    gU = torch.zeros((V, 4, 3, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError):
        W.force(g, psi, psi, N, np.ones(N, dtype=complex), gU)
    g.set_clover(0.0)
    again = lat.new_batch(N)
    W.apply_D(g, 0.1, psi, again, N, W.FP64)
    assert torch.equal(again, plain)


def test_clover_full_size_solve_sampled_residual():
    """16^3 x 32, 48 RHS, mixed FP16 solve with the clover term: the oracle's
    residual b - D_sw x at sampled sites (on the source slice, next to it,
    anywhere) is within the solve tolerance."""
    dims, m0, csw, N, t0 = (16, 16, 16, 32), -0.05, 1.0, 48, 5
    say("clover full size 16^3x32")
    V = int(np.prod(dims))
    Lxyz = dims[0] * dims[1] * dims[2]
    U = gauge_field(dims, 0.3, seed=37)
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    g.set_clover(csw)
    d = W.source_descs(list(range(N)), t0=t0)
    b = lat.new_batch(N)
    W.sources(lat, d, b)
    x = lat.new_batch(N)
    rc, st = W.solve(g, m0, b, x, N, tol=1e-10, prec=W.FP16)
    assert rc == W.OK and all(s["converged"] for s in st)
    rng = np.random.default_rng(38)
    sites = np.concatenate([t0 * Lxyz + rng.integers(0, Lxyz, 64),
                            (t0 + 1) * Lxyz + rng.integers(0, Lxyz, 32), rng.integers(0, V, 32)])
    sites = [int(s) for s in sites]
    C = clover.clover_blocks(U, dims, csw)
    xh = x.cpu().numpy()
    Dx = dirac.apply_D_sites(U, m0, lambda s: xh[s], dims, sites, -1)
    Dx += np.einsum("sij,sjn->sin", C[sites], xh[sites])
    bh = b.cpu().numpy()
    r = bh[sites] - Dx
    nb = np.linalg.norm(bh.reshape(-1, N), axis=0)
    rel = np.linalg.norm(r.transpose(2, 0, 1).reshape(N, -1), axis=1) / nb
    assert np.max(rel) <= 1.01e-10, np.max(rel)


def test_clover_low_modes_match_dense_eigensolver():
    """The deflation's low modes of Q = Gamma5 D_sw (solves and operator with
    the clover term) against a dense Hermitian eigensolver of the oracle's
    Q, with k at a gap of the spectrum."""
    from oracle import deflation as odfl
    from paper_2607_05157_amd import deflation
    dims, m0, csw = (4, 4, 2, 4), -0.6, 1.0
    U = gauge_field(dims, 0.5, seed=31)
    D = clover.dense_D_clover(U, m0, dims, csw)
    Q = odfl.q_matrix(D)
    lam_all, _ = odfl.low_modes(Q, D.shape[0])
    a = np.abs(lam_all)
    k = next(k for k in range(6, 15) if a[k] > 1.03 * a[k - 1])
    say("clover low modes k", k)
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    g.set_clover(csw)
    lam, Vk, info = deflation.low_modes(g, lat, m0, k, extra=16, tol=1e-9, prec=W.FP64,
                                        solve_tol=1e-12)
    assert np.all(info["residuals"] <= 1e-9), info
    ref_lam, ref_V = odfl.low_modes(Q, k)
    assert np.max(np.abs(lam - ref_lam) / np.abs(ref_lam)) < 1e-9
    Vg = Vk.cpu().numpy().reshape(-1, k)
    assert np.linalg.norm(Vg @ Vg.conj().T - ref_V @ ref_V.conj().T, 2) < 1e-6


@pytest.mark.parametrize("N", [1, 64])
def test_clover_even_odd_rhs_counts(c2, N):
    """A single RHS and a full 64-lane batch (one site per wavefront at
    N = 64): mixed FP16 even-odd solves with the clover term against the
    dense inverse."""
    dims, m0, csw, U, Dinv = c2
    say("clover even-odd N", N)
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    g.set_clover(csw)
    b = lat.new_batch(N)
    W.sources(lat, W.source_descs([200 + k for k in range(N)]), b)
    x = lat.new_batch(N)
    rc, st = W.solve(g, m0, b, x, N, tol=1e-10, prec=W.FP16)
    assert rc == W.OK and all(s["converged"] for s in st)
    X = Dinv @ b.cpu().numpy().reshape(-1, N)
    xs = x.cpu().numpy().reshape(-1, N)
    assert np.max(np.linalg.norm(xs - X, axis=0) / np.linalg.norm(X, axis=0)) < 1e-8


def test_clover_changed_after_batch_creation(c2):
    """A batch made before the clover term is set, then solved with it, then
    after it is removed: each solve uses the gauge's term as it is at that
    solve (checked against the dense operator of that moment)."""
    dims, m0, csw, U, Dinv = c2
    say("clover set after batch creation")
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    N = 4
    B = W.Batch([g], [m0], [N])
    b = lat.new_batch(N)
    W.sources(lat, W.source_descs([300 + k for k in range(N)]), b)
    bh = b.cpu().numpy().reshape(-1, N)
    for c in (csw, 0.0):
        g.set_clover(c)
        x = lat.new_batch(N)
        rc, st = B.solve([b], [x], tol=1e-11)
        assert rc == W.OK and all(t["converged"] for t in st)
        r = bh - clover.dense_D_clover(U, m0, dims, c) @ x.cpu().numpy().reshape(-1, N)
        assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(bh, axis=0)) <= 1.01e-11, c


def test_clover_variance_study_matches_oracle():
    """The probing-variance study on a clover gauge (mixed FP16 even-odd
    solves): every estimator's per-seed values against the oracle's estimates
    from the dense inverse of D_sw with the same noise and colouring."""
    from oracle import colouring, estimator as oest
    from paper_2607_05157_amd import study
    dims, m0, csw, t0, seeds = (4, 4, 4, 4), 0.2, 1.2, 1, [0, 1, 2]
    say("clover variance study", dims)
    U = gauge_field(dims, 0.3, seed=39)
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    g.set_clover(csw)
    rows = study.run(g, lat, m0, t0, seeds, distances=(1,), dim=3, eps=0.5, prec=W.FP16,
                     tol=1e-10)
    V = int(np.prod(dims))
    Dinv = osolve.dense_inverse(clover.dense_D_clover(U, m0, dims, csw))
    for row in rows:
        if row["distance"] == 0:
            col, comps = None, ([-1] if row["estimator"] == "hutchinson" else list(range(12)))
            classes = [0]
        else:
            col = colouring.colours(dims, row["sigma"], row["n_c"])
            comps = list(range(12))
            classes = sorted(set(col[np.arange(V) // 64 == t0].tolist()))
        ref = []
        for s in seeds:
            tot = 0j
            for j in classes:
                for k in comps:
                    v = noise.probing_vector(dims, s, col, j, k, t0)
                    if not v.any():
                        continue
                    x = (Dinv @ v.ravel()).reshape(V, 12)
                    tot += oest.sample_dot(v, x, dims, t0, gamma.GAMMA5)
            ref.append(tot)
        ref = np.array(ref)
        got = np.array(row["per_seed_re"]) + 1j * np.array(row["per_seed_im"])
        assert np.max(np.abs(got - ref)) < 1e-8 * max(1.0, np.max(np.abs(ref))), row["estimator"]


def test_clover_connected_correlator_matches_oracle():
    """G(t) averaged over source slices on a clover gauge (mixed FP16
    even-odd solves): per seed against the oracle's norms with the same noise,
    and the mean within its error of the exact G(t) of D_sw (whose trace form
    relies on gamma5-hermiticity, which the term keeps)."""
    from oracle import estimator as oest
    from paper_2607_05157_amd import estimator as E
    dims, m0, csw, seeds = (4, 4, 2, 6), 0.2, 1.3, [0, 1, 2]
    say("clover connected correlator", dims)
    U = gauge_field(dims, 0.4, seed=40)
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    g.set_clover(csw)
    out = E.connected_correlator(g, lat, m0, seeds, n_rhs=48, tol=1e-10, prec=W.FP16)
    V, T = int(np.prod(dims)), dims[3]
    Dinv = osolve.dense_inverse(clover.dense_D_clover(U, m0, dims, csw))
    ref = np.zeros((len(seeds), T))
    for a, s in enumerate(seeds):
        for tp in range(T):
            for k in range(12):
                v = noise.probing_vector(dims, s, None, None, k, tp)
                x = (Dinv @ v.ravel()).reshape(V, 12)
                ref[a] += np.roll(oest.sample_norm2_per_t(x, dims), -tp)
    ref /= T
    assert np.max(np.abs(out["per_seed"] - ref)) < 1e-8 * np.max(ref)
    exact = np.array([oest.exact_G(Dinv, dims, t).real for t in range(T)])
    err = np.sqrt(out["var"] / len(seeds))
    assert np.all(np.abs(out["G"] - exact) < 6 * err + 1e-8 * exact)
