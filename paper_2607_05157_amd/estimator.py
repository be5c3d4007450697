"""Host-side estimator bookkeeping and the autograd wrapper, on top of libwdt.

Every vector operation runs in the library's HIP kernels (sources, solves,
contractions, gamma5, force); this module only decides which sources go into
which batch and adds up the per-batch pieces the library returns.

- hutchinson: tr D^-1 and tr[B D^-1(t,t)] from full-lattice Rademacher
  vectors (Sec. 1, eq. Hutchinson-estimator).
- probing_loop: the disconnected loop O(t0) = tr[Gamma5 D^-1(t0,t0)] (Sec. 4)
  from torus-coloured probing vectors (Sec. 3) with time dilution on t0 and
  spin-colour dilution, optionally with the slice correlator
  ||D^-1(t, t0)||_F^2; batches are checkpointed as JSON lines so an
  interrupted run resumes where it stopped.
- probing_loop(deflation=...): the same with low modes of Q = Gamma5 D
  deflated (Sec. 2, eq. defl-split; see deflation.py): sources deflated before
  the solve, the contraction against the original sources, and the exact
  low-mode part added to every seed's estimate.
- connected_correlator: G(t) = (1/T) sum_t' tr[D^-1(t+t',t') Gamma5
  D^-1(t',t+t') Gamma5] (Sec. 4, eq. connected-results-G) = (1/T) sum_t'
  ||D^-1(t+t', t')||_F^2 by gamma5-hermiticity, from spin-colour diluted
  noise on every source slice t' (all-source-slice time dilution).
- TraceLoss: f_k = eta_k^dag D(U, m0)^-1 eta_k as a torch.autograd.Function
  whose backward is the library's link force (d f / d U, d f / d m0).
"""
import json
import os

import numpy as np

from . import wdt

GAMMA5 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)


def _torch():
    import torch
    return torch


def hutchinson(gauge, lat, m0, seeds, n_rhs=32, tol=1e-12, prec=wdt.FP64, spin=None, t=0):
    """Plain Hutchinson samples.  Returns dict with per-seed samples of
    eta^dag D^-1 eta (whole lattice) and of eta^dag B D^-1 eta on slice t."""
    full, sl, stats = [], [], []
    for lo in range(0, len(seeds), n_rhs):
        chunk = list(seeds[lo:lo + n_rhs])
        N = len(chunk)
        b = lat.new_batch(N)
        wdt.sources(lat, wdt.source_descs(chunk), b)
        x = lat.new_batch(N)
        _, st = wdt.solve(gauge, m0, b, x, N, tol=tol, prec=prec)
        full.extend(wdt.contract(lat, b, x, N).sum(axis=1))
        sl.extend(wdt.contract(lat, b, x, N, spin=spin if spin is not None else GAMMA5)[:, t])
        stats.extend(st)
    full, sl = np.array(full), np.array(sl)
    return dict(samples_full=full, samples_slice=sl, trace=full.mean(), slice_trace=sl.mean(),
                var_full=_var(full), var_slice=_var(sl), stats=stats)


def _var(x):
    x = np.asarray(x)
    return float(np.sum(np.abs(x - x.mean()) ** 2) / (len(x) - 1)) if len(x) > 1 else 0.0


def colours_on_slice(dims, n_c, sigma, t0):
    """Colours of the 4D torus colouring present on time slice t0."""
    x = np.indices(tuple(dims[:3])).reshape(3, -1)
    c = (np.asarray(sigma[:3]) @ x + sigma[3] * t0) % n_c
    return sorted(set(int(v) for v in c))


def probing_loop(gauge, lat, m0, n_c, sigma, t0, seeds, n_rhs=48, dilution=12, tol=1e-10,
                 prec=wdt.FP16, spin=None, correlator=False, checkpoint=None, inner_tol=0.003,
                 max_batches=None, deflation=None):
    """Probing x time dilution x spin-colour dilution estimate of
    tr[B D^-1(t0, t0)] (B = gamma5 by default) and, with correlator=True, of
    ||D^-1(t, t0)||_F^2 for every t.

    Jobs are (colour j, seed, component k); with dilution=1 the component
    mask is off.  Each seed's estimate is the sum over its jobs; the result
    is the mean over seeds with the seed-to-seed sample variance.
    checkpoint: path of a JSON-lines file; batches already recorded there are
    not recomputed.
    deflation: a deflation.Deflation; each source eta is solved as
    eta - Gamma5 V V^dag Gamma5 eta and contracted against eta, and the
    low-mode part tr(B D^-1 Gamma5 V V^dag Gamma5) (k solves) is added to
    every seed."""
    spin = GAMMA5 if spin is None else spin
    if deflation is not None and correlator:
        raise ValueError("the correlator is not deflated")
    cols = colours_on_slice(lat.dims, n_c, sigma, t0)
    comps = list(range(12)) if dilution == 12 else [None]
    jobs = [(j, s, k) for j in cols for s in seeds for k in comps]
    done = {}
    if checkpoint and os.path.exists(checkpoint):
        for line in open(checkpoint):
            rec = json.loads(line)
            done[rec["batch"]] = rec
    Lt = lat.dims[3]
    per_seed = {s: 0j for s in seeds}
    corr = {s: np.zeros(Lt) for s in seeds}
    stats = []
    nb = 0
    for bi, lo in enumerate(range(0, len(jobs), n_rhs)):
        if max_batches is not None and nb >= max_batches:
            break
        batch = jobs[lo:lo + n_rhs]
        if bi in done:
            rec = done[bi]
            samples = np.array(rec["re"]) + 1j * np.array(rec["im"])
            norms = np.array(rec["norm2"]) if correlator else None
        else:
            N = len(batch)
            descs = []
            for (j, s, k) in batch:
                descs.append(dict(seed=s, colour=j, component=k))
            d = wdt.source_descs([x["seed"] for x in descs], n_c=n_c,
                                 colour=[x["colour"] for x in descs], sigma=sigma,
                                 component=[x["component"] for x in descs], t0=t0)
            b = lat.new_batch(N)
            wdt.sources(lat, d, b)
            rhs = b
            if deflation is not None:
                rhs = b.clone()
                deflation.deflate(rhs, N)
            x = lat.new_batch(N)
            _, st = wdt.solve(gauge, m0, rhs, x, N, tol=tol, prec=prec, inner_tol=inner_tol,
                              max_iter=20000, max_outer=60, check_every=10)
            stats.extend(st)
            samples = wdt.contract(lat, b, x, N, spin=spin)[:, t0]
            norms = wdt.contract(lat, None, x, N, mode=wdt.CONTRACT_NORM2) if correlator else None
            if checkpoint:
                rec = dict(batch=bi, jobs=batch, re=samples.real.tolist(), im=samples.imag.tolist())
                if correlator:
                    rec["norm2"] = norms.tolist()
                with open(checkpoint, "a") as f:
                    f.write(json.dumps(rec) + "\n")
            nb += 1
        for i, (j, s, k) in enumerate(batch):
            per_seed[s] += samples[i]
            if correlator:
                corr[s] += norms[i]
    est = np.array([per_seed[s] for s in seeds])
    exact = 0j
    if deflation is not None:
        exact = deflation.exact_part(gauge, m0, t0, spin, tol=tol, prec=prec)
        est = est + exact
    out = dict(per_seed=est, estimate=est.mean(), var_seeds=_var(est), colours=cols,
               n_jobs=len(jobs), stats=stats, exact_part=exact)
    if correlator:
        C = np.array([corr[s] for s in seeds])
        out["correlator"] = C.mean(axis=0)
        out["correlator_per_seed"] = C
    return out


def connected_correlator(gauge, lat, m0, seeds, t_sources=None, n_rhs=48, tol=1e-10,
                         prec=wdt.FP16, inner_tol=0.003):
    """G(t) of eq. connected-results-G with the (1/T) sum over source slices.

    For every source slice t' and seed, the 12 spin-colour components of a
    Rademacher vector on t' are solved; sum_k ||x_k(t)||^2 estimates
    ||D^-1(t, t')||_F^2 (unbiased: the noise has unit variance and the
    dilution removes the cross terms inside a site), and G(t) averages
    t -> t + t' over the source slices.  t_sources defaults to every slice.
    Returns dict(G=[T] mean over seeds, per_seed=[S, T], var=[T], stats)."""
    T = lat.dims[3]
    ts = list(range(T)) if t_sources is None else list(t_sources)
    jobs = [(tp, s, k) for tp in ts for s in seeds for k in range(12)]
    acc = {s: np.zeros(T) for s in seeds}
    stats = []
    for lo in range(0, len(jobs), n_rhs):
        batch = jobs[lo:lo + n_rhs]
        N = len(batch)
        d = wdt.source_descs([s for (_, s, _) in batch], n_c=0,
                             component=[k for (_, _, k) in batch],
                             t0=[tp for (tp, _, _) in batch])
        b = lat.new_batch(N)
        wdt.sources(lat, d, b)
        x = lat.new_batch(N)
        _, st = wdt.solve(gauge, m0, b, x, N, tol=tol, prec=prec, inner_tol=inner_tol,
                          max_iter=20000, max_outer=60)
        stats.extend(st)
        norms = wdt.contract(lat, None, x, N, mode=wdt.CONTRACT_NORM2)   # [N, T]
        for i, (tp, s, _) in enumerate(batch):
            acc[s] += np.roll(norms[i], -tp)          # entry t: ||x(t + t')||^2
    per = np.array([acc[s] / len(ts) for s in seeds])
    var = (np.sum((per - per.mean(axis=0)) ** 2, axis=0) / (len(seeds) - 1)
           if len(seeds) > 1 else np.zeros(T))
    return dict(G=per.mean(axis=0), per_seed=per, var=var, stats=stats, t_sources=ts)


class TraceLoss:
    """f = TraceLoss.apply(U, m0, lat, eta, tol): f_k = eta_k^dag D(U, m0)^-1 eta_k.

    U: complex128 tensor [V, 4, 3, 3] (links U_mu(x)[a, b]); m0: float64 0-d
    tensor; eta: device FP64 batch [V, 12, N].  The forward solves the 2N
    batch [eta, gamma5 eta] once (x = D^-1 eta, y = gamma5 D^-1 gamma5 eta =
    D^-dag eta); the backward is the library's force kernel.  Gradients follow
    torch's complex convention (dL/dconj(z)); m0 is a real leaf."""

    _fn = None

    @classmethod
    def _impl(cls):
        if cls._fn is not None:
            return cls._fn
        torch = _torch()

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, U, m0, lat, eta, tol):
                N = eta.shape[2]
                g = wdt.Gauge(lat, U.detach().cpu().numpy())
                g5eta = torch.empty_like(eta)
                wdt.gamma5(lat, eta, g5eta, N)
                b = torch.cat([eta, g5eta], dim=2).contiguous()
                x2 = torch.zeros_like(b)
                wdt.solve(g, float(m0), b, x2, 2 * N, tol=tol, prec=wdt.FP64)
                x = x2[:, :, :N].contiguous()
                y = x2[:, :, N:].contiguous()
                wdt.gamma5(lat, y, y, N)
                f = wdt.contract(lat, eta, x, N).sum(axis=1)
                ctx.save_for_backward(x, y)
                ctx.g, ctx.lat, ctx.N, ctx.U_device = g, lat, N, U.device
                return torch.tensor(f, dtype=torch.complex128)

            @staticmethod
            def backward(ctx, grad_f):
                x, y = ctx.saved_tensors
                gU = torch.zeros((ctx.lat.V, 4, 3, 3), dtype=torch.complex128, device=x.device)
                gm = wdt.force(ctx.g, x, y, ctx.N, grad_f.detach().cpu().numpy(), gU)
                return (gU.to(ctx.U_device), torch.tensor(gm, dtype=torch.float64), None, None,
                        None)

        cls._fn = _F
        return _F

    @classmethod
    def apply(cls, U, m0, lat, eta, tol=1e-12):
        return cls._impl().apply(U, m0, lat, eta, tol)
