// Device bodies of the solver's kernels, shared by the single-system launches
// (solver.hip, dslash.hip) and the multi-system launches (batch.hip).  Each
// body takes its tile, logical block and block count explicitly.
#pragma once
#include "internal.h"

namespace wdt {

struct RhsState {
    double2 rho, alpha, omega, beta;
    double rr, bb, tol2;
    int active;  // 1 while the RHS is iterating
    int flag;    // 0 running, 1 converged, 2 breakdown
    int iters;
    int pad;
};

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 cmuld(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Sum partials[(d*G + i)*N + r] over i in a fixed order (one block per RHS).
__device__ __forceinline__ double2 block_sum(const double2 *__restrict__ partials, int d, int G, int N, int r) {
    __shared__ double2 sm[256];
    double2 acc = make_double2(0, 0);
    for (int i = threadIdx.x; i < G; i += blockDim.x) {
        const double2 p = partials[((size_t)d * G + i) * N + r];
        acc.x += p.x;
        acc.y += p.y;
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sm[threadIdx.x].x += sm[threadIdx.x + w].x;
            sm[threadIdx.x].y += sm[threadIdx.x + w].y;
        }
        __syncthreads();
    }
    const double2 out = sm[0];
    __syncthreads();
    return out;
}

// After r = b - D x: rr = ||r||^2, bb = ||b||^2; start the recurrence with
// rhat = r.  `bb_ref` (optional) supplies the norm the tolerance refers to.
__device__ __forceinline__ void init_state_body(RhsState *st, const double2 *partials, int G,
                                                int N, double tol, const int *mask, int r) {
    const double2 rr = block_sum(partials, 0, G, N, r);
    const double2 bb = block_sum(partials, 1, G, N, r);
    if (threadIdx.x == 0) {
        RhsState s = st[r];
        s.rr = rr.x;
        s.bb = bb.x;
        s.tol2 = tol * tol;
        s.rho = make_double2(rr.x, 0.0);
        s.alpha = make_double2(0, 0);
        s.omega = make_double2(0, 0);
        s.beta = make_double2(0, 0);
        const bool want = (mask == nullptr) || mask[r];
        const bool done = !(rr.x > s.tol2 * bb.x);
        s.active = (want && !done) ? 1 : 0;
        s.flag = done ? 1 : 0;
        st[r] = s;
    }
}

__device__ __forceinline__ void scalar_alpha_body(RhsState *st, const double2 *partials, int G,
                                                  int N, int r) {
    const double2 rv = block_sum(partials, 0, G, N, r);
    if (threadIdx.x == 0) {
        RhsState s = st[r];
        if (s.active) {
            if (rv.x == 0.0 && rv.y == 0.0) {
                s.active = 0;
                s.flag = 2;
                s.alpha = make_double2(0, 0);
            } else {
                s.alpha = cdiv(s.rho, rv);
            }
        } else {
            s.alpha = make_double2(0, 0);
        }
        st[r] = s;
    }
}

__device__ __forceinline__ void scalar_omega_body(RhsState *st, const double2 *partials, int G,
                                                  int N, int r) {
    const double2 ts = block_sum(partials, 0, G, N, r);
    const double2 tt = block_sum(partials, 1, G, N, r);
    if (threadIdx.x == 0) {
        RhsState s = st[r];
        if (s.active && tt.x > 0.0) {
            s.omega = make_double2(ts.x / tt.x, ts.y / tt.x);
        } else {
            s.omega = make_double2(0, 0);
        }
        st[r] = s;
    }
}

__device__ __forceinline__ void scalar_beta_body(RhsState *st, const double2 *partials, int G,
                                                 int N, int r) {
    const double2 rho_new = block_sum(partials, 0, G, N, r);
    const double2 rr = block_sum(partials, 1, G, N, r);
    if (threadIdx.x == 0) {
        RhsState s = st[r];
        if (s.active) {
            s.iters += 1;
            s.rr = rr.x;
            if (!(rr.x > s.tol2 * s.bb)) {
                s.active = 0;
                s.flag = 1;
                s.beta = make_double2(0, 0);
            } else if ((rho_new.x == 0.0 && rho_new.y == 0.0) ||
                       (s.omega.x == 0.0 && s.omega.y == 0.0) || !isfinite(rr.x)) {
                s.active = 0;
                s.flag = 2;
                s.beta = make_double2(0, 0);
            } else {
                s.beta = cmuld(cdiv(rho_new, s.rho), cdiv(s.alpha, s.omega));
                s.rho = rho_new;
            }
        } else {
            s.beta = make_double2(0, 0);
        }
        st[r] = s;
    }
}

// ---------------------------------------------------------------------------
// Vector kernels over (site, rhs) with the operator's block shape.

template <class S> using Rl = typename S::real;

template <class S>
__device__ __forceinline__ cplx<Rl<S>> to_c(double2 a) {
    return {(Rl<S>)a.x, (Rl<S>)a.y};
}



// s = r - alpha v
template <class S>
__device__ __forceinline__ void update_s_body(const Geom &g, int N, int NT, int SB,
                                              const RhsState *__restrict__ st, SpinorPtr<S> rv,
                                              SpinorPtr<S> vv, SpinorPtr<S> sv, int tile, int lb,
                                              int gb) {
    using R = Rl<S>;
    SITE_LOOP_BEGIN_AT(tile, lb, gb)
    const cplx<R> a = to_c<S>(st[r].alpha);
    cplx<R> x[12], y[12];
    load_site<S>(rv, s, r, x);
    load_site<S>(vv, s, r, y);
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = csub(x[k], cmul(a, y[k]));
    store_site<S>(sv, s, r, x);
    SITE_LOOP_END
}

// x += alpha p + omega s;  r = s - omega t;  partials: rhat^dag r, ||r||^2
template <class S>
__device__ __forceinline__ void update_xr_body(const Geom &g, int N, int NT, int SB,
                                               const RhsState *__restrict__ st, SpinorPtr<S> xv,
                                               SpinorPtr<S> pv, SpinorPtr<S> sv, SpinorPtr<S> tv,
                                               SpinorPtr<S> rv, SpinorPtr<S> rhat,
                                               double2 *partials, int tile, int lb, int gb) {
    using R = Rl<S>;
    __shared__ double2 red[2][256];
    double d0r = 0, d0i = 0, d1r = 0;
    SITE_LOOP_BEGIN_AT(tile, lb, gb)
    const cplx<R> a = to_c<S>(st[r].alpha);
    const cplx<R> w = to_c<S>(st[r].omega);
    cplx<R> x[12], p[12], sv_[12], t[12], h[12];
    load_site<S>(xv, s, r, x);
    load_site<S>(pv, s, r, p);
    load_site<S>(sv, s, r, sv_);
    load_site<S>(tv, s, r, t);
    load_site<S>(rhat, s, r, h);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        x[k] = cadd(x[k], cadd(cmul(a, p[k]), cmul(w, sv_[k])));
        p[k] = csub(sv_[k], cmul(w, t[k]));  // new r
        d0r += (double)h[k].re * p[k].re + (double)h[k].im * p[k].im;
        d0i += (double)h[k].re * p[k].im - (double)h[k].im * p[k].re;
        d1r += (double)p[k].re * p[k].re + (double)p[k].im * p[k].im;
    }
    store_site<S>(xv, s, r, x);
    store_site<S>(rv, s, r, p);
    SITE_LOOP_END
    red[0][tid] = make_double2(d0r, d0i);
    red[1][tid] = make_double2(d1r, 0.0);
    __syncthreads();
    if (ry == 0 && r < N) {
        double2 s0 = red[0][rl], s1 = red[1][rl];
        for (int y = 1; y < SB; ++y) {
            s0.x += red[0][y * NT + rl].x;
            s0.y += red[0][y * NT + rl].y;
            s1.x += red[1][y * NT + rl].x;
        }
        partials[((size_t)0 * Gb + Lb) * N + r] = s0;
        partials[((size_t)1 * Gb + Lb) * N + r] = s1;
    }
}

// p = r + beta (p - omega v)
template <class S>
__device__ __forceinline__ void update_p_body(const Geom &g, int N, int NT, int SB,
                                              const RhsState *__restrict__ st, SpinorPtr<S> rv,
                                              SpinorPtr<S> pv, SpinorPtr<S> vv, int tile, int lb,
                                              int gb) {
    using R = Rl<S>;
    SITE_LOOP_BEGIN_AT(tile, lb, gb)
    const cplx<R> b = to_c<S>(st[r].beta);
    const cplx<R> w = to_c<S>(st[r].omega);
    cplx<R> x[12], p[12], v[12];
    load_site<S>(rv, s, r, x);
    load_site<S>(pv, s, r, p);
    load_site<S>(vv, s, r, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = cadd(x[k], cmul(b, csub(p[k], cmul(w, v[k]))));
    store_site<S>(pv, s, r, p);
    SITE_LOOP_END
}

// dst(T) = src(S) converted (and optionally dst += src when ADD)
template <class SS, class SD, bool ADD>
__device__ __forceinline__ void convert_body(const Geom &g, int N, int NT, int SB,
                                             SpinorPtr<SS> src, SpinorPtr<SD> dst, int tile,
                                             int lb, int gb) {
    SITE_LOOP_BEGIN_AT(tile, lb, gb)
    cplx<Rl<SS>> a[12];
    load_site<SS>(src, s, r, a);
    cplx<Rl<SD>> b[12];
    if constexpr (ADD) {
        load_site<SD>(dst, s, r, b);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            b[k].re += (Rl<SD>)a[k].re;
            b[k].im += (Rl<SD>)a[k].im;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) b[k] = {(Rl<SD>)a[k].re, (Rl<SD>)a[k].im};
    }
    store_site<SD>(dst, s, r, b);
    SITE_LOOP_END
}


// Empty asm that claims to modify the accumulator: it makes the hops before
// it complete before later hops start.  Without it the compiler sinks all
// accumulation to the end of the site and keeps every neighbour's spinor and
// link live at once (hundreds of VGPRs, spills); with one after every hop it
// serialises the loads.  PIN = 1 places it after each direction (two hops
// whose loads are issued together), PIN = 2 after each hop.
template <class T>
__device__ __forceinline__ void pin(cplx<T> (&a)[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) asm volatile("" : "+v"(a[k].re), "+v"(a[k].im));
}

// Schedule per precision: one direction (two spinors, two links) in flight.
template <class S> struct OpPin { static constexpr int value = 1; };

// Non-temporal output stores keep the operator's output from evicting input
// lines that neighbouring sites still have to re-read from L2.
#ifndef WDT_OP_STREAM_STORES
#define WDT_OP_STREAM_STORES 1
#endif

template <int MU, bool DAG, int PIN, int NC, class S>
__device__ __forceinline__ void hop_pair(const Geom &g, const typename S::link *__restrict__ U,
                                         const SpinorPtr<S> &in, int s, const SiteNbr &nb, int r,
                                         cplx<typename S::real> (&acc)[12]) {
    using R = typename S::real;
    constexpr int SF = DAG ? +1 : -1;  // forward projector (1 + SF gamma_mu)
    const int b = nb.bwd[MU];
    cplx<R> pf[12], pb[12], uf[9], ub[9];
    R sf = load_site_raw<S, NC>(in, nb.fwd[MU], r, pf);
    load_link<S, R>(U, s, MU, uf);
    R sb = R(1);
    if constexpr (PIN != 2) {
        sb = load_site_raw<S, NC>(in, b, r, pb);
        load_link<S, R>(U, b, MU, ub);
    }
    {
        // the FP16 scale and the time-boundary sign act on the half spinor
        if (MU == 3 && nb.fwd_wrap_t && g.bc_t < 0) sf = -sf;
        cplx<R> h[6];
        project<MU, SF>(pf, h);
        if constexpr (S::scaled || MU == 3) {
#pragma unroll
            for (int k = 0; k < 6; ++k) h[k] = {h[k].re * sf, h[k].im * sf};
        }
        cplx<R> w[6];
        su3_mul(uf, h, w);
        reconstruct_add<MU, SF>(acc, w);
    }
    if constexpr (PIN == 2) {
        pin(acc);
        sb = load_site_raw<S, NC>(in, b, r, pb);
        load_link<S, R>(U, b, MU, ub);
    }
    {
        if (MU == 3 && nb.bwd_wrap_t && g.bc_t < 0) sb = -sb;
        cplx<R> h[6];
        project<MU, -SF>(pb, h);
        if constexpr (S::scaled || MU == 3) {
#pragma unroll
            for (int k = 0; k < 6; ++k) h[k] = {h[k].re * sb, h[k].im * sb};
        }
        cplx<R> w[6];
        su3_adj_mul(ub, h, w);
        reconstruct_add<MU, -SF>(acc, w);
    }
    if constexpr (PIN != 0) pin(acc);
}

template <class S, int NC, bool DAG, int EPI>
__device__ __forceinline__ void dslash_body(const Geom &g, const typename S::link *__restrict__ U,
                                            typename S::real diag, SpinorPtr<S> in,
                                            SpinorPtr<S> out, SpinorPtr<S> aux, int N, int NT,
                                            int SB, double2 *__restrict__ partials, int tile0,
                                            int tile1, int Lb, int Gb) {
    using R = typename S::real;
    constexpr int PIN = OpPin<S>::value;
    __shared__ double2 red[2][256];
    const int tid = threadIdx.x;
    const int rl = tid % NT;
    const int ry = tid / NT;
    const Sweep sw = sweep((g.V + SB - 1) / SB, Lb, Gb);
    // RHS tiles [tile0, tile1) one after the other: the XCD's L2 then holds
    // one tile's worth of each site instead of the whole batch
    for (int tile = tile0; tile < tile1; ++tile) {
    const int r = tile * NT + rl;
    const bool live = (ry < SB) && (r < N);
    double d0r = 0, d0i = 0, d1r = 0, d1i = 0;
    if (live) {
        for (int grp = sw.first; grp < sw.end; grp += sw.step) {
            const int p = grp * SB + ry;
            if (p >= g.V) break;
            const int s = site_of(g, p);
            const SiteNbr nb = neighbours(g, s);
            cplx<R> acc[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
            hop_pair<0, DAG, PIN, NC, S>(g, U, in, s, nb, r, acc);
            hop_pair<1, DAG, PIN, NC, S>(g, U, in, s, nb, r, acc);
            hop_pair<2, DAG, PIN, NC, S>(g, U, in, s, nb, r, acc);
            hop_pair<3, DAG, PIN, NC, S>(g, U, in, s, nb, r, acc);
            cplx<R> c[12];
            load_site<S, NC>(in, s, r, c);
            cplx<R> o[12];
#pragma unroll
            for (int k = 0; k < 12; ++k)
                o[k] = {diag * c[k].re - R(0.5) * acc[k].re, diag * c[k].im - R(0.5) * acc[k].im};
            if constexpr (EPI == EPI_RESID) {
                cplx<R> b[12];
                load_site<S, NC>(aux, s, r, b);
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    o[k] = csub(b[k], o[k]);
                    d0r += (double)o[k].re * o[k].re + (double)o[k].im * o[k].im;
                    d1r += (double)b[k].re * b[k].re + (double)b[k].im * b[k].im;
                }
            } else if constexpr (EPI == EPI_DOT_AUX) {
                cplx<R> a[12];
                load_site<S, NC>(aux, s, r, a);
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    d0r += (double)a[k].re * o[k].re + (double)a[k].im * o[k].im;
                    d0i += (double)a[k].re * o[k].im - (double)a[k].im * o[k].re;
                }
            } else if constexpr (EPI == EPI_DOT_TS) {
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    d0r += (double)o[k].re * c[k].re + (double)o[k].im * c[k].im;
                    d0i += (double)o[k].re * c[k].im - (double)o[k].im * c[k].re;
                    d1r += (double)o[k].re * o[k].re + (double)o[k].im * o[k].im;
                }
            }
            store_site<S, WDT_OP_STREAM_STORES != 0, NC>(out, s, r, o);
        }
    }
    if constexpr (EPI != EPI_NONE) {
        red[0][tid] = make_double2(d0r, d0i);
        red[1][tid] = make_double2(d1r, d1i);
        __syncthreads();
        if (ry == 0 && r < N) {
            double2 s0 = red[0][rl], s1 = red[1][rl];
            for (int y = 1; y < SB; ++y) {
                const double2 a0 = red[0][y * NT + rl], a1 = red[1][y * NT + rl];
                s0.x += a0.x;
                s0.y += a0.y;
                s1.x += a1.x;
                s1.y += a1.y;
            }
            partials[((size_t)0 * Gb + Lb) * N + r] = s0;
            if (EPI != EPI_DOT_AUX) partials[((size_t)1 * Gb + Lb) * N + r] = s1;
        }
        if (tile + 1 < tile1) __syncthreads();  // red[] is reused by the next tile
    }
    }
}

}  // namespace wdt
