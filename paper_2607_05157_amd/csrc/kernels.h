// Device bodies of the solver's kernels, shared by the single-system launches
// (solver.hip, dslash.hip) and the multi-system launches (batch.hip).  Each
// body takes its tile, logical block and block count explicitly.
#pragma once
#include "internal.h"

#include <type_traits>

namespace wdt {

struct RhsState {
    double2 rho, alpha, omega, beta;
    double2 rv;  // rhat^dag v of the current iteration (fused updates)
    double rr, bb, tol2;
    int active;  // 1 while the RHS is iterating
    int flag;    // 0 running, 1 converged, 2 breakdown, 3 diverged (inner solves)
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
// tolr (may be null): per-RHS tolerances in place of tol; bbv (may be null):
// per-RHS ||b||^2 in place of partials slot 1.
__device__ __forceinline__ void init_state_body(RhsState *st, const double2 *partials, int G,
                                                int N, double tol, const int *mask,
                                                const double *tolr, const double *bbv, int r) {
    const double2 rr = block_sum(partials, 0, G, N, r);
    const double2 bb = bbv ? make_double2(bbv[r], 0.0) : block_sum(partials, 1, G, N, r);
    if (threadIdx.x == 0) {
        RhsState s = st[r];
        s.rr = rr.x;
        s.bb = bb.x;
        const double tl = tolr ? tolr[r] : tol;
        s.tol2 = tl * tl;
        s.rho = make_double2(rr.x, 0.0);
        s.alpha = make_double2(0, 0);
        s.omega = make_double2(0, 0);
        s.beta = make_double2(0, 0);
        const bool want = (mask == nullptr) || mask[r];
        const bool finite = isfinite(rr.x) && isfinite(bb.x);
        const bool done = finite && !(rr.x > s.tol2 * bb.x);
        s.active = (want && finite && !done) ? 1 : 0;
        s.flag = !finite ? 2 : done ? 1 : 0;
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
                s.rv = rv;
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

// Cache policy of the streaming vector kernels: STREAMV loads and stores the
// vectors non-temporally.  The launches choose it for FP64 vectors larger than
// the last-level cache (update passes 4.6 -> 5.1-5.2 TB/s on 16^3 x 32,
// 48 RHS); smaller ones, and the 32-bit-element formats, stay cached (their
// next pass finds them there: non-temporal, the FP16 passes fell from 4.7 to
// 4.1-4.2 TB/s).
template <class S, bool STREAMV>
__device__ __forceinline__ void vec_load(const SpinorPtr<S> &sp, int site, int r,
                                         cplx<Rl<S>> (&v)[12]) {
    if constexpr (STREAMV) load_site_once<S>(sp, site, r, v);
    else load_site<S>(sp, site, r, v);
}
template <class S, bool STREAMV>
__device__ __forceinline__ void vec_store(const SpinorPtr<S> &sp, int site, int r,
                                          const cplx<Rl<S>> (&v)[12]) {
    store_site<S, STREAMV>(sp, site, r, v);
}

template <class S>
__device__ __forceinline__ cplx<Rl<S>> to_c(double2 a) {
    return {(Rl<S>)a.x, (Rl<S>)a.y};
}



// s = r - alpha v
template <class S, bool STREAMV = false>
__device__ __forceinline__ void update_s_body(const Geom &g, int N, int NT, int SB,
                                              const RhsState *__restrict__ st, SpinorPtr<S> rv,
                                              SpinorPtr<S> vv, SpinorPtr<S> sv, int tile, int lb,
                                              int gb) {
    using R = Rl<S>;
    SITE_LOOP_BEGIN_AT(tile, lb, gb)
    const cplx<R> a = to_c<S>(st[r].alpha);
    cplx<R> x[12], y[12];
    vec_load<S, STREAMV>(rv, s, r, x);
    vec_load<S, STREAMV>(vv, s, r, y);
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = csub(x[k], cmul(a, y[k]));
    vec_store<S, STREAMV>(sv, s, r, x);
    SITE_LOOP_END
}

// x += alpha p + omega s;  r = s - omega t;  partials: rhat^dag r, ||r||^2
template <class S, bool STREAMV = false>
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
    vec_load<S, STREAMV>(xv, s, r, x);
    vec_load<S, STREAMV>(pv, s, r, p);
    vec_load<S, STREAMV>(sv, s, r, sv_);
    vec_load<S, STREAMV>(tv, s, r, t);
    vec_load<S, STREAMV>(rhat, s, r, h);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        x[k] = cadd(x[k], cadd(cmul(a, p[k]), cmul(w, sv_[k])));
        p[k] = csub(sv_[k], cmul(w, t[k]));  // new r
        d0r += (double)h[k].re * p[k].re + (double)h[k].im * p[k].im;
        d0i += (double)h[k].re * p[k].im - (double)h[k].im * p[k].re;
        d1r += (double)p[k].re * p[k].re + (double)p[k].im * p[k].im;
    }
    vec_store<S, STREAMV>(xv, s, r, x);
    vec_store<S, STREAMV>(rv, s, r, p);
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
template <class S, bool STREAMV = false>
__device__ __forceinline__ void update_p_body(const Geom &g, int N, int NT, int SB,
                                              const RhsState *__restrict__ st, SpinorPtr<S> rv,
                                              SpinorPtr<S> pv, SpinorPtr<S> vv, int tile, int lb,
                                              int gb) {
    using R = Rl<S>;
    SITE_LOOP_BEGIN_AT(tile, lb, gb)
    const cplx<R> b = to_c<S>(st[r].beta);
    const cplx<R> w = to_c<S>(st[r].omega);
    cplx<R> x[12], p[12], v[12];
    vec_load<S, STREAMV>(rv, s, r, x);
    vec_load<S, STREAMV>(pv, s, r, p);
    vec_load<S, STREAMV>(vv, s, r, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = cadd(x[k], cmul(b, csub(p[k], cmul(w, v[k]))));
    vec_store<S, STREAMV>(pv, s, r, p);
    SITE_LOOP_END
}

// Fused form of the end of an iteration, for the inner solves of the mixed
// solver: the new shadow product comes from the recurrence
//   rhat^dag r_new = rhat^dag s - omega rhat^dag t = rho - alpha rhat^dag v - omega rhat^dag t
// (rhat^dag v from the first operator's epilogue, rhat^dag t from the
// second's), so beta is known before the vector updates and x, r and p are
// updated in one pass (8 vector passes instead of 11).  The recurrence loses
// digits as |r| falls, which an inner solve to a few per cent does not feel;
// the FP64 solver keeps the direct product.
__device__ __forceinline__ void scalar_omega_beta_body(RhsState *st, const double2 *partials, int G,
                                                       int N, int r) {
    const double2 ts = block_sum(partials, 0, G, N, r);
    const double2 tt = block_sum(partials, 1, G, N, r);
    const double2 rt = block_sum(partials, 2, G, N, r);
    if (threadIdx.x == 0) {
        RhsState s = st[r];
        if (!s.active) {
            s.omega = make_double2(0, 0);
            s.beta = make_double2(0, 0);
        } else if (!(tt.x > 0.0)) {
            // t = 0: s is the residual; take x += alpha p and stop
            s.omega = make_double2(0, 0);
            s.beta = make_double2(0, 0);
            s.active = 0;
            s.flag = 2;
        } else {
            s.omega = make_double2(ts.x / tt.x, ts.y / tt.x);
            const double2 a_rv = cmuld(s.alpha, s.rv), w_rt = cmuld(s.omega, rt);
            const double2 rho_new = make_double2(s.rho.x - a_rv.x - w_rt.x, s.rho.y - a_rv.y - w_rt.y);
            if ((rho_new.x == 0.0 && rho_new.y == 0.0) || (s.omega.x == 0.0 && s.omega.y == 0.0)) {
                s.beta = make_double2(0, 0);
                s.active = 0;
                s.flag = 2;
            } else {
                s.beta = cmuld(cdiv(rho_new, s.rho), cdiv(s.alpha, s.omega));
                s.rho = rho_new;
            }
        }
        st[r] = s;
    }
}

// Whether any RHS is still iterating (one block): *live in device memory, for
// the kernels of the next iteration, and *host in host-mapped memory, for the
// host loop; both 1 or 0.
__device__ __forceinline__ void live_body(const RhsState *st, int N, int *live, int *host) {
    int a = 0;
    for (int r = threadIdx.x; r < N; r += blockDim.x) a |= st[r].active;
    const int any = __syncthreads_or(a) ? 1 : 0;
    if (threadIdx.x == 0) {
        *live = any;
        if (host) *host = any;
    }
}

// rho = the squared norm in partials slot 0 (the start of an iteration whose
// shadow vector is the current residual).
__device__ __forceinline__ void scalar_rho_body(RhsState *st, const double2 *partials, int G,
                                                int N, int r) {
    const double2 nn = block_sum(partials, 0, G, N, r);
    if (threadIdx.x == 0) {
        RhsState s = st[r];
        s.rho = make_double2(nn.x, 0.0);
        st[r] = s;
    }
}

// After the fused update: ||r||^2, convergence and the iteration count.
__device__ __forceinline__ void scalar_check_body(RhsState *st, const double2 *partials, int G,
                                                  int N, int r) {
    const double2 rr = block_sum(partials, 0, G, N, r);
    if (threadIdx.x == 0) {
        RhsState s = st[r];
        if (s.active || s.flag == 2) {
            if (s.active) s.iters += 1;
            s.rr = rr.x;
            if (s.active && !(rr.x > s.tol2 * s.bb)) {
                s.active = 0;
                s.flag = 1;
            } else if (!isfinite(rr.x)) {
                s.active = 0;
                s.flag = 2;
            } else if (s.active && rr.x > 1e8 * s.bb) {
                // the low-precision recurrence has run away (its residual is
                // 1e4 times the start): stop, the outer correction takes over
                s.active = 0;
                s.flag = 3;
            }
        }
        st[r] = s;
    }
}

// x += alpha p + omega s;  r = s - omega t;  p = r + beta (p - omega v);
// partials: ||r||^2
template <class S, bool STREAMV = false>
__device__ __forceinline__ void update_xrp_body(const Geom &g, int N, int NT, int SB,
                                                const RhsState *__restrict__ st, SpinorPtr<S> xv,
                                                SpinorPtr<S> pv, SpinorPtr<S> sv, SpinorPtr<S> tv,
                                                SpinorPtr<S> rv, SpinorPtr<S> vv,
                                                double2 *partials, int tile, int lb, int gb) {
    using R = Rl<S>;
    __shared__ double2 red[256];
    double d0 = 0;
    SITE_LOOP_BEGIN_AT(tile, lb, gb)
    const cplx<R> a = to_c<S>(st[r].alpha);
    const cplx<R> w = to_c<S>(st[r].omega);
    const cplx<R> b = to_c<S>(st[r].beta);
    cplx<R> x[12], p[12], sv_[12], t[12], v[12];
    vec_load<S, STREAMV>(xv, s, r, x);
    vec_load<S, STREAMV>(pv, s, r, p);
    vec_load<S, STREAMV>(sv, s, r, sv_);
    vec_load<S, STREAMV>(tv, s, r, t);
    vec_load<S, STREAMV>(vv, s, r, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        x[k] = cadd(x[k], cadd(cmul(a, p[k]), cmul(w, sv_[k])));
        const cplx<R> rn = csub(sv_[k], cmul(w, t[k]));
        p[k] = cadd(rn, cmul(b, csub(p[k], cmul(w, v[k]))));
        sv_[k] = rn;
        d0 += (double)rn.re * rn.re + (double)rn.im * rn.im;
    }
    vec_store<S, STREAMV>(xv, s, r, x);
    vec_store<S, STREAMV>(rv, s, r, sv_);
    vec_store<S, STREAMV>(pv, s, r, p);
    SITE_LOOP_END
    red[tid] = make_double2(d0, 0.0);
    __syncthreads();
    if (ry == 0 && r < N) {
        double2 s0 = red[rl];
        for (int y = 1; y < SB; ++y) s0.x += red[y * NT + rl].x;
        partials[(size_t)Lb * N + r] = s0;
    }
}

// partials slot 0 of block Lb: the block's ||src||^2 per RHS.
template <class S>
__device__ __forceinline__ void norm_body(const Geom &g, int N, int NT, int SB, SpinorPtr<S> src,
                                          double2 *__restrict__ partials, int tile, int lb,
                                          int gb) {
    __shared__ double red[256];
    double d0 = 0;
    SITE_LOOP_BEGIN_AT(tile, lb, gb)
    cplx<Rl<S>> a[12];
    load_site<S>(src, s, r, a);
#pragma unroll
    for (int k = 0; k < 12; ++k)
        d0 += (double)a[k].re * (double)a[k].re + (double)a[k].im * (double)a[k].im;
    SITE_LOOP_END
    red[tid] = d0;
    __syncthreads();
    if (ry == 0 && r < N) {
        double s0 = red[rl];
        for (int y = 1; y < SB; ++y) s0 += red[y * NT + rl];
        partials[(size_t)Lb * N + r] = make_double2(s0, 0.0);
    }
}

// dst = f[r] * src converted (dst += f[r] * src when ADD); f = nullptr: 1.
// The product is formed in FP64 before the conversion, so a residual can be
// brought to unit norm on its way into low precision and the correction
// scaled back on its way out.  partials (may be null): slots 0 and 1 of
// block Lb both get the block's ||dst||^2 (of the value before rounding to
// the storage precision).
template <class SS, class SD, bool ADD>
__device__ __forceinline__ void convert_body(const Geom &g, int N, int NT, int SB,
                                             SpinorPtr<SS> src, SpinorPtr<SD> dst,
                                             SpinorPtr<SD> dst2,
                                             const double *__restrict__ f,
                                             double2 *__restrict__ partials, int tile, int lb,
                                             int gb) {
    __shared__ double red[256];
    double d0 = 0;
    SITE_LOOP_BEGIN_AT(tile, lb, gb)
    const double fr = f ? f[r] : 1.0;
    cplx<Rl<SS>> a[12];
    load_site<SS>(src, s, r, a);
    cplx<Rl<SD>> b[12];
    if constexpr (ADD) {
        load_site<SD>(dst, s, r, b);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            b[k].re += (Rl<SD>)(fr * (double)a[k].re);
            b[k].im += (Rl<SD>)(fr * (double)a[k].im);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k)
            b[k] = {(Rl<SD>)(fr * (double)a[k].re), (Rl<SD>)(fr * (double)a[k].im)};
    }
    if (partials) {
#pragma unroll
        for (int k = 0; k < 12; ++k)
            d0 += (double)b[k].re * (double)b[k].re + (double)b[k].im * (double)b[k].im;
    }
    store_site<SD>(dst, s, r, b);
    if (dst2.p) store_site<SD>(dst2, s, r, b);
    SITE_LOOP_END
    if (partials) {
        red[tid] = d0;
        __syncthreads();
        if (ry == 0 && r < N) {
            double s0 = red[rl];
            for (int y = 1; y < SB; ++y) s0 += red[y * NT + rl];
            partials[(size_t)Lb * N + r] = make_double2(s0, 0.0);
            partials[((size_t)Gb + Lb) * N + r] = make_double2(s0, 0.0);
        }
    }
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

// Keeps loaded elements in registers from this point on: the inputs are
// read-only, so the compiler may otherwise load a carried value again at
// the end of a loop body, and the next iteration then waits for that load
// behind the stores issued after it.
template <class E>
__device__ __forceinline__ void pin_elems(E (&e)[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        if constexpr (sizeof(E) == 4) {
            unsigned u;
            __builtin_memcpy(&u, &e[k], 4);
            asm volatile("" : "+v"(u));
            __builtin_memcpy(&e[k], &u, 4);
        } else {
            asm volatile("" : "+v"(e[k].x), "+v"(e[k].y));
        }
    }
}

// Schedule per precision: one direction (two spinors, two links) in flight.
template <class S> struct OpPin { static constexpr int value = 1; };
#ifdef WDT_OP_PIN_F16
template <> struct OpPin<F16> { static constexpr int value = WDT_OP_PIN_F16; };
#endif

// Non-temporal output stores keep the operator's output from evicting input
// lines that neighbouring sites still have to re-read from L2.
#ifndef WDT_OP_STREAM_STORES
#define WDT_OP_STREAM_STORES 1
#endif
// The epilogue's extra vector (rhat, or b for the residual) is read once.
#ifndef WDT_AUX_LOAD
#define WDT_AUX_LOAD load_site_once
#endif

// ---------------------------------------------------------------------------
// FP16 operator arithmetic.  The half spinor is formed in packed half
// precision (one packed add per colour component, the unit factor folded into
// the add's operand modifiers), and each part of a link-times-half-spinor
// product is a chain of three two-term half dot products accumulated in FP32
// (v_dot2), with the link element stored as the pairs (ur, -ui) and (ui, ur).
// A hop then costs 36 dot products instead of 72 FP32 multiply-adds and the
// 24 conversions of the neighbour spinor.
typedef _Float16 hv2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ hv2 as_hv2(__half2 a) {
    hv2 r;
    __builtin_memcpy(&r, &a, 4);
    return r;
}

// i^K z for z = (re, im)
template <int K>
__device__ __forceinline__ hv2 hunit(hv2 z) {
    if constexpr ((K & 3) == 0) return z;
    else if constexpr ((K & 3) == 1) return hv2{-z.y, z.x};
    else if constexpr ((K & 3) == 2) return hv2{-z.x, -z.y};
    else return hv2{z.y, -z.x};
}

// rows 0, 1 of (1 + SGN gamma_mu) psi (the same tables as project())
template <int MU, int SGN>
__device__ __forceinline__ void hproject(const __half2 (&psi)[12], hv2 (&h)[6]) {
    using P = Proj<MU>;
    constexpr int sh = (SGN < 0) ? 0 : 2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h[c] = as_hv2(psi[c]) + hunit<P::a0 + sh>(as_hv2(psi[3 * P::p0 + c]));
        h[3 + c] = as_hv2(psi[3 + c]) + hunit<P::a1 + sh>(as_hv2(psi[3 * P::p1 + c]));
    }
}

// w = U h (ADJ = false) or U^dag h (ADJ = true); u in the paired form
template <bool ADJ>
__device__ __forceinline__ void hsu3(const __half2 (&u)[18], const hv2 (&h)[6],
                                     cplx<float> (&w)[6]) {
    hv2 hs[6];
    if constexpr (ADJ) {
#pragma unroll
        for (int k = 0; k < 6; ++k) hs[k] = hv2{h[k].y, h[k].x};
    }
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if constexpr (!ADJ) {
                    // (ur, -ui).(hr, hi) and (ui, ur).(hr, hi)
                    re = __builtin_amdgcn_fdot2(as_hv2(u[2 * (3 * a + b)]), h[3 * hh + b], re, false);
                    im = __builtin_amdgcn_fdot2(as_hv2(u[2 * (3 * a + b) + 1]), h[3 * hh + b], im, false);
                } else {
                    // conj(u_ba) h_b: (ui, ur).(hi, hr) and (ur, -ui).(hi, hr)
                    re = __builtin_amdgcn_fdot2(as_hv2(u[2 * (3 * b + a) + 1]), hs[3 * hh + b], re, false);
                    im = __builtin_amdgcn_fdot2(as_hv2(u[2 * (3 * b + a)]), hs[3 * hh + b], im, false);
                }
            }
            w[3 * hh + a] = {re, im};
        }
}

// acc += s * (full spinor of (1 + SGN gamma_mu) reconstructed from w), the
// scale folded into the multiply-adds
template <int MU, int SGN>
__device__ __forceinline__ void reconstruct_add_scaled(cplx<float> (&acc)[12], const cplx<float> (&w)[6],
                                                       float s) {
    using P = Proj<MU>;
    constexpr int sh = (SGN < 0) ? 0 : 2;
    auto fma_s = [s](cplx<float> &a, cplx<float> z) {
        a.re = fmaf(s, z.re, a.re);
        a.im = fmaf(s, z.im, a.im);
    };
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        fma_s(acc[c], w[c]);
        fma_s(acc[3 + c], w[3 + c]);
        fma_s(acc[6 + c], cunit<P::b2 + sh>(w[3 * P::q2 + c]));
        fma_s(acc[9 + c], cunit<P::b3 + sh>(w[3 * P::q3 + c]));
    }
}

// w = scale * U_mu(link_site) P psi (ADJ = false) or scale * U_mu(link_site)^dag
// P psi (ADJ = true), P = rows 0, 1 of (1 + SGN gamma_mu); psi given as its
// stored elements.
template <class S, int MU, int SGN, bool ADJ>
__device__ __forceinline__ void hop_w(const typename S::link *__restrict__ U, int link_site,
                                      const typename S::elem (&e)[12], typename S::real scale,
                                      cplx<typename S::real> (&w)[6]) {
    using R = typename S::real;
    if constexpr (S::scaled) {
        __half2 u[18];
        const __half2 *q = U + ((size_t)link_site * 4 + MU) * 18;
#pragma unroll
        for (int k = 0; k < 18; ++k) u[k] = q[k];
        hv2 h[6];
        hproject<MU, SGN>(e, h);
        hsu3<ADJ>(u, h, w);
#pragma unroll
        for (int k = 0; k < 6; ++k) w[k] = {w[k].re * scale, w[k].im * scale};
    } else {
        cplx<R> p[12], u[9], h[6];
        elems_to_cplx<S>(e, p);
        load_link<S, R>(U, link_site, MU, u);
        project<MU, SGN>(p, h);
        if (MU == 3) {  // the boundary sign rides on the scale
#pragma unroll
            for (int k = 0; k < 6; ++k) h[k] = {h[k].re * scale, h[k].im * scale};
        }
        if constexpr (ADJ) su3_adj_mul(u, h, w);
        else su3_mul(u, h, w);
    }
}

// acc += the reconstructed hop of hop_w (FP16: the scale folded into the adds)
template <class S, int MU, int SGN, bool ADJ>
__device__ __forceinline__ void hop_acc(const typename S::link *__restrict__ U, int link_site,
                                        const typename S::elem (&e)[12], typename S::real scale,
                                        cplx<typename S::real> (&acc)[12]) {
    if constexpr (S::scaled) {
        __half2 u[18];
        const __half2 *q = U + ((size_t)link_site * 4 + MU) * 18;
#pragma unroll
        for (int k = 0; k < 18; ++k) u[k] = q[k];
        hv2 h[6];
        hproject<MU, SGN>(e, h);
        cplx<float> w[6];
        hsu3<ADJ>(u, h, w);
        reconstruct_add_scaled<MU, SGN>(acc, w, scale);
    } else {
        cplx<typename S::real> w[6];
        hop_w<S, MU, SGN, ADJ>(U, link_site, e, scale, w);
        reconstruct_add<MU, SGN>(acc, w);
    }
}

template <int MU, bool DAG, int PIN, int NC, class S>
__device__ __forceinline__ void hop_pair(const Geom &g, const typename S::link *__restrict__ U,
                                         const SpinorPtr<S> &in, int s, const SiteNbr &nb, int r,
                                         cplx<typename S::real> (&acc)[12]) {
    using R = typename S::real;
    using E = typename S::elem;
    constexpr int SF = DAG ? +1 : -1;  // forward projector (1 + SF gamma_mu)
    const int b = nb.bwd[MU];
    E pf[12], pb[12];
    R sf = load_site_elems<S, NC>(in, nb.fwd[MU], r, pf);
    R sb = R(1);
    if constexpr (PIN != 2) sb = load_site_elems<S, NC>(in, b, r, pb);
    {
        // the FP16 scale and the time-boundary sign act on the hop
        if (MU == 3 && nb.fwd_wrap_t && g.bc_t < 0) sf = -sf;
        hop_acc<S, MU, SF, false>(U, s, pf, sf, acc);
    }
    if constexpr (PIN == 2) {
        pin(acc);
        sb = load_site_elems<S, NC>(in, b, r, pb);
    }
    {
        if (MU == 3 && nb.bwd_wrap_t && g.bc_t < 0) sb = -sb;
        hop_acc<S, MU, -SF, true>(U, b, pb, sb, acc);
    }
    if constexpr (PIN != 0) pin(acc);
}

// Dot-product partials of the operator epilogues (per thread, then per block)
struct EpiAcc {
    double d0r = 0, d0i = 0, d1r = 0, d2r = 0, d2i = 0;
};

// Reduces the epilogue partials over the block and writes
// partials[(d * Gb + Lb) * N + r] for the slots the epilogue fills:
// d = 0 (complex), d = 1 (real part), d = 2 (complex, EPI_DOT_TSR only).
template <int EPI>
__device__ __forceinline__ void epi_reduce(double2 (&red)[3][256], int tid, int rl, int ry, int r,
                                           int N, int NT, int SB, const EpiAcc &e,
                                           double2 *__restrict__ partials, int Lb, int Gb) {
    red[0][tid] = make_double2(e.d0r, e.d0i);
    red[1][tid] = make_double2(e.d1r, 0.0);
    red[2][tid] = make_double2(e.d2r, e.d2i);
    __syncthreads();
    if (ry == 0 && r < N) {
        double2 s0 = red[0][rl], s1 = red[1][rl], s2 = red[2][rl];
        for (int y = 1; y < SB; ++y) {
            const double2 a0 = red[0][y * NT + rl], a1 = red[1][y * NT + rl],
                          a2 = red[2][y * NT + rl];
            s0.x += a0.x;
            s0.y += a0.y;
            s1.x += a1.x;
            s2.x += a2.x;
            s2.y += a2.y;
        }
        partials[((size_t)0 * Gb + Lb) * N + r] = s0;
        if (EPI != EPI_DOT_AUX) partials[((size_t)1 * Gb + Lb) * N + r] = s1;
        if (EPI == EPI_DOT_TSR) partials[((size_t)2 * Gb + Lb) * N + r] = s2;
    }
}

// acc += k C c for one site: C the packed clover term, block-diagonal in
// the two chiralities (spins 0-1 and 2-3, since it commutes with gamma5).
// Each 6 x 6 Hermitian block is 36 reals: its real diagonal, then the 15
// elements above it row by row as (re, im).  With k = 1/ch the output
// cs c + ch acc gains C c.
template <class R>
__device__ __forceinline__ void clover_add(const R *__restrict__ C, const cplx<R> (&c)[12], R k,
                                           cplx<R> (&acc)[12]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const R *A = C + 36 * h;
        cplx<R> y[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) y[i] = cscale(c[6 * h + i], A[i]);
        int q = 6;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
#pragma unroll
            for (int j = i + 1; j < 6; ++j, q += 2) {
                const cplx<R> a = {A[q], A[q + 1]};
                y[i] = cfma(y[i], a, c[6 * h + j]);
                y[j] = cfmaconj(y[j], a, c[6 * h + i]);
            }
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            acc[6 * h + i].re += k * y[i].re;
            acc[6 * h + i].im += k * y[i].im;
        }
    }
}

// Output of one site, out = cs * c + ch * acc (c: the site's spinor of the
// self vector, acc: the hop sum), with the epilogue's dot contributions;
// stores the result.  The operator itself is cs = 4 + m0, ch = -1/2.
//  EPI_DOT_AUX: d0 += aux^dag out
//  EPI_DOT_TS:  d0 += out^dag in, d1 += ||out||^2
//  EPI_DOT_TSR: as EPI_DOT_TS, and d2 += aux^dag out
//  EPI_RESID:   out = aux - D in; d0 += ||out||^2, d1 += ||aux||^2
//  EPI_NORM:    d0 += ||out||^2, d1 += ||out||^2
template <class S, int NC, int EPI>
__device__ __forceinline__ void finish_site(typename S::real cs, typename S::real ch,
                                            const cplx<typename S::real> (&c)[12],
                                            const cplx<typename S::real> (&acc)[12], SpinorPtr<S> out,
                                            SpinorPtr<S> aux, int s, int r, EpiAcc &e) {
    using R = typename S::real;
    cplx<R> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
        o[k] = {cs * c[k].re + ch * acc[k].re, cs * c[k].im + ch * acc[k].im};
    if constexpr (EPI == EPI_RESID) {
        cplx<R> b[12];
        WDT_AUX_LOAD<S, NC>(aux, s, r, b);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            o[k] = csub(b[k], o[k]);
            e.d0r += (double)o[k].re * o[k].re + (double)o[k].im * o[k].im;
            e.d1r += (double)b[k].re * b[k].re + (double)b[k].im * b[k].im;
        }
    } else if constexpr (EPI == EPI_DOT_AUX) {
        cplx<R> a[12];
        WDT_AUX_LOAD<S, NC>(aux, s, r, a);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            e.d0r += (double)a[k].re * o[k].re + (double)a[k].im * o[k].im;
            e.d0i += (double)a[k].re * o[k].im - (double)a[k].im * o[k].re;
        }
    } else if constexpr (EPI == EPI_NORM) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double n = (double)o[k].re * o[k].re + (double)o[k].im * o[k].im;
            e.d0r += n;
            e.d1r += n;
        }
    } else if constexpr (EPI == EPI_DOT_TS || EPI == EPI_DOT_TSR) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            e.d0r += (double)o[k].re * c[k].re + (double)o[k].im * c[k].im;
            e.d0i += (double)o[k].re * c[k].im - (double)o[k].im * c[k].re;
            e.d1r += (double)o[k].re * o[k].re + (double)o[k].im * o[k].im;
        }
        if constexpr (EPI == EPI_DOT_TSR) {
            cplx<R> a[12];
            WDT_AUX_LOAD<S, NC>(aux, s, r, a);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                e.d2r += (double)a[k].re * o[k].re + (double)a[k].im * o[k].im;
                e.d2i += (double)a[k].re * o[k].im - (double)a[k].im * o[k].re;
            }
        }
    }
    store_site<S, WDT_OP_STREAM_STORES != 0, NC>(out, s, r, o);
}

// WPS (one site per wavefront): NT = 64, the lanes are the RHS of one site,
// so the site, its neighbours and the link addresses are wave-uniform; the
// links then come through the scalar cache into SGPRs instead of occupying
// the vector memory pipeline with 64 copies of the same address.
//
// General form: out(s) = cs * self(s) + ch * H(in)(s), H the hop sum, over
// the sites of g (one parity when g.parity >= 0); the operator D is
// self = in, cs = 4 + m0, ch = -1/2.  cs = 0 skips the self load.  CLOV
// (compile-time, so that the plain operator's registers are unaffected):
// 1, the clover term Cl, out(s) += C(s) self(s) (needs cs != 0); 2, Cl holds
// the inverse blocks (a + C)^-1 and out(s) = Cl(s) (cs self(s) + ch H(in)(s))
// (EPI_NONE only).
template <class S, int NC, bool DAG, int EPI, bool WPS = false, int CLOV = 0>
__device__ __forceinline__ void dslash_body(const Geom &g, const typename S::link *__restrict__ U,
                                            const typename S::real *__restrict__ Cl,
                                            SpinorPtr<S> self, typename S::real cs,
                                            typename S::real ch, SpinorPtr<S> in,
                                            SpinorPtr<S> out, SpinorPtr<S> aux, int N, int NT,
                                            int SB, double2 *__restrict__ partials, int tile0,
                                            int tile1, int Lb, int Gb) {
    using R = typename S::real;
    constexpr int PIN = OpPin<S>::value;
    __shared__ double2 red[3][256];
    const int tid = threadIdx.x;
    const int rl = WPS ? (tid & 63) : tid % NT;
    const int ry = WPS ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid / NT;
    const Sweep sw = sweep((g.nsites + SB - 1) / SB, Lb, Gb);
    // RHS tiles [tile0, tile1) one after the other: the XCD's L2 then holds
    // one tile's worth of each site instead of the whole batch
    for (int tile = tile0; tile < tile1; ++tile) {
    const int r = tile * NT + rl;
    const bool live = (ry < SB) && (r < N);
    EpiAcc e;
    if (live) {
        for (int grp = sw.first; grp < sw.end; grp += sw.step) {
            const int p = grp * SB + ry;
            if (p >= g.nsites) break;
            const int s = site_of(g, p);
            const SiteNbr nb = neighbours(g, s);
            cplx<R> acc[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
            // PIN 3: the accumulator is pinned after every second direction
            constexpr int PA = PIN == 3 ? 0 : PIN, PB = PIN == 3 ? 1 : PIN;
            hop_pair<0, DAG, PA, NC, S>(g, U, in, s, nb, r, acc);
            hop_pair<1, DAG, PB, NC, S>(g, U, in, s, nb, r, acc);
            hop_pair<2, DAG, PA, NC, S>(g, U, in, s, nb, r, acc);
            hop_pair<3, DAG, PB, NC, S>(g, U, in, s, nb, r, acc);
            cplx<R> c[12];
            if (cs != R(0)) {
                // a separate own-term vector is read once: keep it out of the
                // L2 lines the neighbour gathers reuse
                if (self.p != in.p) WDT_AUX_LOAD<S, NC>(self, s, r, c);
                else load_site<S, NC>(self, s, r, c);
                if constexpr (CLOV == 1)
                    clover_add<R>(Cl + (size_t)s * CLOVER_REALS, c, R(1) / ch, acc);
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) c[k] = {R(0), R(0)};
            }
            if constexpr (CLOV == 2) {
                static_assert(EPI == EPI_NONE, "inverse blocks: no epilogue");
                cplx<R> o[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    o[k] = {cs * c[k].re + ch * acc[k].re, cs * c[k].im + ch * acc[k].im};
                    acc[k] = {R(0), R(0)};
                }
                clover_add<R>(Cl + (size_t)s * CLOVER_REALS, o, R(1), acc);
                finish_site<S, NC, EPI>(R(0), R(1), c, acc, out, aux, s, r, e);
            } else {
                finish_site<S, NC, EPI>(cs, ch, c, acc, out, aux, s, r, e);
            }
        }
    }
    if constexpr (EPI != EPI_NONE) {
        epi_reduce<EPI>(red, tid, rl, ry, r, N, NT, SB, e, partials, Lb, Gb);
        if (tile + 1 < tile1) __syncthreads();  // red[] is reused by the next tile
    }
    }
}

// The same operator with every thread marching along t through one spatial
// column for one RHS.  The t-neighbours come from registers: the forward one
// is the next step's own site, and the backward hop into (x, t+1) is formed
// at step t from the own spinor and the link U_t(x, t) that the forward hop
// loads anyway.  A site then costs six spatial neighbour reads and one new
// spinor instead of nine reads, and seven links instead of eight; the
// column's spatial neighbours are computed once per column.  The columns
// are cut into bricks of B[0] x B[1] x B[2] (B[0] a multiple of CB); a work
// unit is CB consecutive columns of one brick row over TC consecutive time
// slices, numbered chunk-major, then brick, then within the brick.  Each XCD
// takes a contiguous range of units and its resident blocks take consecutive
// units, so what an XCD marches through at once is a whole brick: the six
// spatial reads of a site find the slice its neighbours loaded one step
// earlier in that XCD's L2, except across the brick's faces.
template <class S, int NC, bool DAG, int EPI, bool WPS = false>
__device__ __forceinline__ void dslash_march_body(const Geom &g, const typename S::link *__restrict__ U,
                                                  typename S::real diag, SpinorPtr<S> in,
                                                  SpinorPtr<S> out, SpinorPtr<S> aux, int N,
                                                  int NT, int CB, int TC, int4 B,
                                                  double2 *__restrict__ partials, int tile, int Lb,
                                                  int Gb) {
    using R = typename S::real;
    using E = typename S::elem;
    constexpr int PIN = OpPin<S>::value;
    constexpr int SF = DAG ? +1 : -1;
    __shared__ double2 red[3][256];
    const int tid = threadIdx.x;
    const int rl = WPS ? (tid & 63) : tid % NT;
    const int ry = WPS ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid / NT;
    const int r = tile * NT + rl;
    const bool live = (ry < CB) && (r < N);
    const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], Lt = g.L[3];
    const int Lxyz = g.Lxyz;
    const int gx = B.x / CB;                              // column groups per brick row
    const int upb = gx * B.y * B.z;                       // units per brick and chunk
    const int nbx = L0 / B.x, nby = L1 / B.y, nbz = L2 / B.z;
    const int ncg = upb * nbx * nby * nbz;                // units per chunk
    const Sweep sw = sweep(ncg * (Lt / TC), Lb, Gb);
    EpiAcc e;
    if (live) {
        for (int u = sw.first; u < sw.end; u += sw.step) {
            const int chunk = u / ncg;
            int c, x, y, z;
            {
                int q = u - chunk * ncg;
                const int brick = q / upb;
                q -= brick * upb;
                const int bxi = brick % nbx, byi = (brick / nbx) % nby, bzi = brick / (nbx * nby);
                x = bxi * B.x + (q % gx) * CB + ry;
                q /= gx;
                y = byi * B.y + q % B.y;
                z = bzi * B.z + q / B.y;
                c = x + L0 * (y + L1 * z);
            }
            int cf[3], cb[3];
            {
                const int sxy = L0 * L1;
                cf[0] = (x == L0 - 1) ? c - (L0 - 1) : c + 1;
                cb[0] = (x == 0) ? c + (L0 - 1) : c - 1;
                cf[1] = (y == L1 - 1) ? c - (L1 - 1) * L0 : c + L0;
                cb[1] = (y == 0) ? c + (L1 - 1) * L0 : c - L0;
                cf[2] = (z == L2 - 1) ? c - (L2 - 1) * sxy : c + sxy;
                cb[2] = (z == 0) ? c + (L2 - 1) * sxy : c - sxy;
            }
            const int t0 = chunk * TC;
            E ec[12];
            R sc = load_site_elems<S, NC>(in, c + Lxyz * t0, r, ec);
            // backward t-hop into (c, t0)
            cplx<R> wb[6];
            {
                const int sbk = c + Lxyz * (t0 == 0 ? Lt - 1 : t0 - 1);
                E pb[12];
                R sb = load_site_elems<S, NC>(in, sbk, r, pb);
                if (t0 == 0 && g.bc_t < 0) sb = -sb;
                hop_w<S, 3, -SF, true>(U, sbk, pb, sb, wb);
            }
            for (int t = t0; t < t0 + TC; ++t) {
                const int s = c + Lxyz * t;
                const bool wrap = (t == Lt - 1);
                E en[12];
                R sn = load_site_elems<S, NC>(in, wrap ? c : s + Lxyz, r, en);
                SiteNbr nb;
#pragma unroll
                for (int mu = 0; mu < 3; ++mu) {
                    nb.fwd[mu] = cf[mu] + Lxyz * t;
                    nb.bwd[mu] = cb[mu] + Lxyz * t;
                }
                nb.fwd[3] = nb.bwd[3] = s;
                nb.fwd_wrap_t = nb.bwd_wrap_t = false;
                cplx<R> acc[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
                hop_pair<0, DAG, PIN, NC, S>(g, U, in, s, nb, r, acc);
                hop_pair<1, DAG, PIN, NC, S>(g, U, in, s, nb, r, acc);
                hop_pair<2, DAG, PIN, NC, S>(g, U, in, s, nb, r, acc);
                {
                    const R sf = (wrap && g.bc_t < 0) ? -sn : sn;
                    hop_acc<S, 3, SF, false>(U, s, en, sf, acc);
                    pin_elems(en);
                    asm volatile("" : "+v"(sn));
                }
                reconstruct_add<3, -SF>(acc, wb);
                // the backward hop of the next step: U_t(s)^dag P psi(s)
                hop_w<S, 3, -SF, true>(U, s, ec, sc, wb);
                cplx<R> cc[12];
                elems_to_cplx<S>(ec, cc);
                if constexpr (S::scaled) {
#pragma unroll
                    for (int k = 0; k < 12; ++k) cc[k] = {cc[k].re * sc, cc[k].im * sc};
                }
                finish_site<S, NC, EPI>(diag, R(-0.5), cc, acc, out, aux, s, r, e);
#pragma unroll
                for (int k = 0; k < 12; ++k) ec[k] = en[k];
                sc = sn;
            }
        }
    }
    if constexpr (EPI != EPI_NONE)
        epi_reduce<EPI>(red, tid, rl, ry, r, N, NT, CB, e, partials, Lb, Gb);
}

}  // namespace wdt
