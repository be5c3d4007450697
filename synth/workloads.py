"""The benchmark workloads as seeded recipes (shapes, link spread, mass, seeds).

Every workload is synthetic: links come from `synth.gauge.gauge_field`, the
noise from the counter-based Rademacher generator (implemented separately by
the oracle and by the HIP library).  Field names follow the paper's notation:
dims = (Lx, Ly, Lz, Lt), m0 the bare mass in the (4 + m0) normalisation,
eps the link spread of U = expm(i*eps*H), d the colouring distance.
"""
import numpy as np

WORKLOADS = {
    # 4^4, plain Hutchinson with 32 Rademacher vectors, BiCGStab to 1e-12.
    "hutchinson_4x4x4x4": dict(dims=(4, 4, 4, 4), bc_t=-1, eps=0.3, m0=0.2,
                               gauge_seed=1, n_rhs=32, noise_seeds=list(range(32)),
                               tol=1e-12, prec="fp64"),
    # 16^3x32, 4D torus distance-2 probing x time dilution (t0=0) x spin-colour
    # dilution x 4 seeds: 48 RHS per colour, 16 colour batches.
    "loop_16c32_d2": dict(dims=(16, 16, 16, 32), bc_t=-1, eps=0.5, m0=0.02,
                          gauge_seed=2, n_rhs=48, noise_seeds=[0, 1, 2, 3],
                          colouring_d=2, t0=0, dilution=12, tol=1e-10,
                          prec="mixed_fp16"),
    # Differentiation on 8^4 with 8 Rademacher vectors.
    "grad_8x8x8x8": dict(dims=(8, 8, 8, 8), bc_t=-1, eps=0.3, m0=0.2,
                         gauge_seed=4, n_rhs=8, noise_seeds=list(range(8)),
                         tol=1e-12, prec="fp64"),
    # 24^3x48, distance-4 torus colouring x time dilution x spin-colour
    # dilution, batches of 64, loop and connected correlator.
    "loop_24c48_d4": dict(dims=(24, 24, 24, 48), bc_t=-1, eps=0.6, m0=0.0,
                          gauge_seed=5, n_rhs=64, noise_seeds=[0],
                          colouring_d=4, t0=0, dilution=12, tol=1e-10,
                          prec="mixed_fp16"),
}


def workload(name):
    return dict(WORKLOADS[name])


def batched_instances(n_per_shape=32, seed=7):
    """Uneven batch of lattice instances: 8^4, 8^3x16 and 12^3x24.

    For instance i the link spread eps ~ U[0.2, 0.5], the mass m0 ~ U[0.05, 0.3]
    and the RHS count ~ U{16..48}, all from one seeded stream; gauge seed 1000+i.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(8, 8, 8, 8), (8, 8, 8, 16), (12, 12, 12, 24)]
    out = []
    i = 0
    for dims in shapes:
        for _ in range(n_per_shape):
            eps = float(rng.uniform(0.2, 0.5))
            m0 = float(rng.uniform(0.05, 0.3))
            n_rhs = int(rng.integers(16, 49))
            out.append(dict(dims=dims, bc_t=-1, eps=eps, m0=m0, gauge_seed=1000 + i,
                            n_rhs=n_rhs, noise_seed_base=100000 * (i + 1)))
            i += 1
    return out
