"""GPU checks of the multi-system batched solve: every system's solution
matches its own single-system solve and the oracle, in one graph-replayed
launch sequence over uneven lattices and RHS counts."""
import numpy as np
import pytest

from oracle import dirac, noise, solve as osolve
from synth.gauge import gauge_field
from synth.workloads import batched_instances

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


def _systems(specs):
    out = []
    for i, (dims, eps, m0, N) in enumerate(specs):
        U = gauge_field(dims, eps, seed=500 + i)
        lat = W.Lattice(dims, -1)
        g = W.Gauge(lat, U)
        b = lat.new_batch(N)
        W.sources(lat, W.source_descs([1000 * i + k for k in range(N)]), b)
        out.append(dict(dims=dims, U=U, m0=m0, N=N, lat=lat, g=g, b=b))
    return out


@pytest.mark.parametrize("tune", [False, True])
def test_batched_matches_single_and_oracle(tune):
    specs = [((4, 4, 4, 4), 0.3, 0.2, 5), ((4, 4, 2, 8), 0.5, 0.1, 17), ((2, 4, 4, 6), 0.4, 0.3, 16),
             ((6, 4, 4, 4), 0.2, 0.05, 33), ((4, 4, 4, 4), 0.45, 0.25, 48)]
    say("batched solve", len(specs), "systems, tune", tune)
    sys = _systems(specs)
    B = W.Batch([s["g"] for s in sys], [s["m0"] for s in sys], [s["N"] for s in sys])
    if tune:
        ms = B.tune(iters=2)
        assert ms > 0
    xs = [s["lat"].new_batch(s["N"]) for s in sys]
    rc, st = B.solve([s["b"] for s in sys], xs, tol=1e-11)
    assert rc == W.OK and all(t["converged"] for t in st)
    assert max(t["true_residual"] for t in st) <= 1e-11
    k = 0
    for s, x in zip(sys, xs):
        xr = s["lat"].new_batch(s["N"])
        W.solve(s["g"], s["m0"], s["b"], xr, s["N"], tol=1e-11)
        a, b_ = x.cpu().numpy(), xr.cpu().numpy()
        assert np.max(np.abs(a - b_)) < 1e-9 * np.max(np.abs(b_))
        D = dirac.dense_D(s["U"], s["m0"], s["dims"], -1)
        ref = osolve.dense_solve(D, s["b"].cpu().numpy().reshape(-1, s["N"]))
        assert np.max(np.abs(a.reshape(-1, s["N"]) - ref)) < 1e-9 * np.max(np.abs(ref))
        k += s["N"]


def test_batched_workload_shapes_small():
    """The three lattice shapes of the uneven workload (8^4, 8^3x16, 12^3x24),
    one instance each with its seeded parameters, against single solves."""
    inst = batched_instances(n_per_shape=1)
    say("batched workload shapes", [i["dims"] for i in inst])
    sys = []
    for i in inst:
        U = gauge_field(i["dims"], i["eps"], seed=i["gauge_seed"])
        lat = W.Lattice(i["dims"], -1)
        g = W.Gauge(lat, U)
        b = lat.new_batch(i["n_rhs"])
        W.sources(lat, W.source_descs([i["noise_seed_base"] + k for k in range(i["n_rhs"])]), b)
        sys.append(dict(lat=lat, g=g, b=b, m0=i["m0"], N=i["n_rhs"]))
    B = W.Batch([s["g"] for s in sys], [s["m0"] for s in sys], [s["N"] for s in sys])
    xs = [s["lat"].new_batch(s["N"]) for s in sys]
    rc, st = B.solve([s["b"] for s in sys], xs, tol=1e-10)
    assert rc == W.OK
    for s, x in zip(sys, xs):
        xr = s["lat"].new_batch(s["N"])
        W.solve(s["g"], s["m0"], s["b"], xr, s["N"], tol=1e-10)
        # both meet 1e-10; the solutions agree to the tolerance times cond(D)
        assert torch.max(torch.abs(x - xr)).item() < 1e-8 * torch.max(torch.abs(xr)).item()


def test_batched_uneven_convergence_redeals_blocks():
    """Systems that converge many iterations apart (a heavy mass next to light
    ones), checked every iteration so the block budget is dealt again each
    time one finishes; two solves in a row on the same batch."""
    specs = [((4, 4, 4, 4), 0.3, 3.0, 8), ((4, 4, 2, 8), 0.5, 0.02, 24), ((2, 4, 4, 6), 0.4, 1.0, 16),
             ((6, 4, 4, 4), 0.2, 0.05, 40)]
    say("batched uneven convergence", len(specs))
    sys = _systems(specs)
    B = W.Batch([s["g"] for s in sys], [s["m0"] for s in sys], [s["N"] for s in sys])
    for rep in range(2):
        xs = [s["lat"].new_batch(s["N"]) for s in sys]
        rc, st = B.solve([s["b"] for s in sys], xs, tol=1e-11, check_every=1)
        assert rc == W.OK and all(t["converged"] for t in st)
        its = [t["iterations"] for t in st]
        assert its[0] < its[8] // 2  # the heavy system finishes far earlier
        for s, x in zip(sys, xs):
            D = dirac.dense_D(s["U"], s["m0"], s["dims"], -1)
            ref = osolve.dense_solve(D, s["b"].cpu().numpy().reshape(-1, s["N"]))
            got = x.cpu().numpy().reshape(-1, s["N"])
            assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("even_odd", [-1, 0])
def test_batched_even_odd_next_to_odd_lattices(even_odd):
    """Even-odd preconditioned systems (every extent even) and systems with an
    odd extent (full operator) in one batch, each against the dense-LU
    oracle; with even_odd=0 every system solves the full operator."""
    specs = [((3, 4, 2, 5), 0.4, 0.1, 7), ((4, 4, 4, 4), 0.3, 0.05, 20), ((2, 3, 4, 6), 0.5, 0.2, 16),
             ((4, 2, 2, 6), 0.45, 0.02, 48)]
    say("batched even-odd next to odd lattices", even_odd)
    sys = _systems(specs)
    try:
        W.set_launch_shape(even_odd=even_odd)
        B = W.Batch([s["g"] for s in sys], [s["m0"] for s in sys], [s["N"] for s in sys])
        xs = [s["lat"].new_batch(s["N"]) for s in sys]
        rc, st = B.solve([s["b"] for s in sys], xs, tol=1e-11)
        assert rc == W.OK and all(t["converged"] for t in st)
        assert max(t["true_residual"] for t in st) <= 1e-11
        for s, x in zip(sys, xs):
            D = dirac.dense_D(s["U"], s["m0"], s["dims"], -1)
            ref = osolve.dense_solve(D, s["b"].cpu().numpy().reshape(-1, s["N"]))
            got = x.cpu().numpy().reshape(-1, s["N"])
            assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref)), s["dims"]
    finally:
        W.set_launch_shape()
