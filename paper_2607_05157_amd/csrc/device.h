// Device-side building blocks shared by the gfx950 kernels: complex
// arithmetic, the spinor batch formats, lattice neighbours and the
// DeGrand-Rossi spin projectors (1 -/+ gamma_mu).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace wdt {

template <class T> struct cplx { T re, im; };

template <class T> __device__ __forceinline__ cplx<T> cmake(T r, T i) { return {r, i}; }
template <class T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.re * s, a.im * s}; }
template <class T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <class T> __device__ __forceinline__ cplx<T> cconjmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// a + b * c
template <class T> __device__ __forceinline__ cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> c) {
    return {a.re + b.re * c.re - b.im * c.im, a.im + b.re * c.im + b.im * c.re};
}
// a + conj(b) * c
template <class T> __device__ __forceinline__ cplx<T> cfmaconj(cplx<T> a, cplx<T> b, cplx<T> c) {
    return {a.re + b.re * c.re + b.im * c.im, a.im + b.re * c.im - b.im * c.re};
}
// z * unit, unit index k: 0 -> +1, 1 -> +i, 2 -> -1, 3 -> -i (compile-time)
template <int K, class T> __device__ __forceinline__ cplx<T> cunit(cplx<T> z) {
    if constexpr ((K & 3) == 0) return z;
    else if constexpr ((K & 3) == 1) return {-z.im, z.re};
    else if constexpr ((K & 3) == 2) return {-z.re, -z.im};
    else return {z.im, -z.re};
}

// ---------------------------------------------------------------------------
// Lattice geometry: site = x + Lx*(y + Ly*(z + Lz*t)).
struct Geom {
    int L[4];
    int stride[4];
    int V;
    int Lxyz;
    int bc_t;
    // Processing order of the sites (see site_of): tiles of Lx*Ly*bz*bt sites,
    // or, when bx > 0, bricks of bx*by*bz columns marched through all of t.
    int bz, bt;
    int bx, by;
    // parity >= 0: kernels visit only the sites with (x+y+z+t) % 2 == parity
    // (all extents even), nsites = V/2; parity < 0: all sites, nsites = V.
    int parity;
    int nsites;
};

// Site index of processing position p.  The lattice is cut into tiles of
// Lx*Ly*bz*bt sites, z-tiles fastest, then t-tiles; inside a tile x runs
// fastest, then y, z, t.  Consecutive positions are then close in all four
// directions (a t-neighbour is Lx*Ly*bz positions away instead of Lx*Ly*Lz),
// which lets an XCD's L2 serve the neighbour re-reads of the operator.
__device__ __forceinline__ int site_of(const Geom &g, int p) {
    if (g.parity >= 0 && g.bx > 0) {
        // one parity in brick order (bx even): positions 2p and 2p + 1 of the
        // full brick order are x-neighbours in one brick row, x of 2p even
        const int q0 = 2 * p;
        const int bvol = g.bx * g.by * g.bz;
        const int per_brick = bvol * g.L[3];
        const int brick = q0 / per_brick;
        int q = q0 - brick * per_brick;
        const int t = q / bvol;
        q -= t * bvol;
        const int nbx = g.L[0] / g.bx, nby = g.L[1] / g.by;
        const int bxi = brick % nbx, byi = (brick / nbx) % nby, bzi = brick / (nbx * nby);
        int x = bxi * g.bx + q % g.bx;
        q /= g.bx;
        const int y = byi * g.by + q % g.by;
        const int z = bzi * g.bz + q / g.by;
        x += ((y + z + t) & 1) ^ g.parity;
        return x + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
    }
    if (g.parity >= 0) {
        // the p-th site of the parity: sites 2p and 2p+1 lie in one x-row
        // (Lx even) and have opposite parities; the row's (y, z, t) decide
        const int s0 = 2 * p;
        const int q = s0 / g.L[0];
        const int rowpar = (q ^ (q / g.L[1]) ^ (q / (g.L[1] * g.L[2]))) & 1;
        return s0 + (rowpar != g.parity ? 1 : 0);
    }
    if (g.bx > 0) {
        // brick order: brick by brick, each brick one time slice after the
        // other, x fastest inside a slice of the brick
        const int bvol = g.bx * g.by * g.bz;
        const int per_brick = bvol * g.L[3];
        const int brick = p / per_brick;
        int q = p - brick * per_brick;
        const int t = q / bvol;
        q -= t * bvol;
        const int nbx = g.L[0] / g.bx, nby = g.L[1] / g.by;
        const int bxi = brick % nbx, byi = (brick / nbx) % nby, bzi = brick / (nbx * nby);
        const int x = bxi * g.bx + q % g.bx;
        q /= g.bx;
        const int y = byi * g.by + q % g.by;
        const int z = bzi * g.bz + q / g.by;
        return x + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
    }
    if (g.bz == g.L[2] && g.bt == g.L[3]) return p;
    const int tvol = g.Lxyz / g.L[2] * g.bz * g.bt;
    const int tile = p / tvol;
    int q = p - tile * tvol;
    const int nzt = g.L[2] / g.bz;
    const int zt = tile % nzt, tt = tile / nzt;
    const int xy = q % (g.L[0] * g.L[1]);
    q /= g.L[0] * g.L[1];
    const int z = zt * g.bz + q % g.bz;
    const int t = tt * g.bt + q / g.bz;
    return xy + g.L[0] * g.L[1] * (z + g.L[2] * t);
}

// Work split of a (site, rhs) kernel: with a grid of G blocks (G a multiple
// of 8), the blocks on XCD k sweep the k-th eighth of the processing order
// in steps of G/8 groups, so each XCD streams through one contiguous region.
struct Sweep {
    int first, end, step;
};
__device__ __forceinline__ Sweep sweep(int ngroups, int Lb, int G) {
    const int nx = (G % 8 == 0) ? 8 : 1;
    const int Gx = G / nx;
    const int xcd = Lb / Gx, j = Lb - xcd * Gx;
    const int gpx = (ngroups + nx - 1) / nx;
    Sweep w;
    w.first = xcd * gpx + j;
    w.end = min(ngroups, (xcd + 1) * gpx);
    w.step = Gx;
    return w;
}

struct SiteNbr {
    int fwd[4], bwd[4];
    bool fwd_wrap_t, bwd_wrap_t;
};

__device__ __forceinline__ SiteNbr neighbours(const Geom &g, int s) {
    SiteNbr n;
    int c[4];
    c[0] = s % g.L[0];
    int q = s / g.L[0];
    c[1] = q % g.L[1];
    q /= g.L[1];
    c[2] = q % g.L[2];
    c[3] = q / g.L[2];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        n.fwd[mu] = (c[mu] == g.L[mu] - 1) ? s - (g.L[mu] - 1) * g.stride[mu] : s + g.stride[mu];
        n.bwd[mu] = (c[mu] == 0) ? s + (g.L[mu] - 1) * g.stride[mu] : s - g.stride[mu];
    }
    n.fwd_wrap_t = (c[3] == g.L[3] - 1);
    n.bwd_wrap_t = (c[3] == 0);
    return n;
}

// ---------------------------------------------------------------------------
// Spinor batch formats: [V][12][N] with the RHS index innermost.
//  F64: double2; F32: float2; F16: __half2 plus a float scale per (site, rhs)
//  stored after the V*12*N half2 values; B16: a bfloat16 pair, no scale.
//  `link` is the element type of the links the operator reads; the FP16
//  operator reads half links in a paired form made for half dot products.

// bfloat16 pair (re in the low half, im in the high half of one 32-bit word):
// the top 16 bits of an IEEE binary32, so decoding is a shift and encoding a
// rounding of the low 16 bits (to nearest, ties to even; NaN stays NaN).
struct bf16x2 {
    unsigned int v;
};
__device__ __forceinline__ float bf16_lo(bf16x2 e) { return __uint_as_float(e.v << 16); }
__device__ __forceinline__ float bf16_hi(bf16x2 e) { return __uint_as_float(e.v & 0xffff0000u); }
__device__ __forceinline__ unsigned int bf16_bits(float f) {
    const unsigned int u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (u >> 16) | 0x0040u;
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ bf16x2 bf16_pack(float re, float im) {
    return bf16x2{bf16_bits(re) | (bf16_bits(im) << 16)};
}

struct F64 {
    using real = double;
    using elem = double2;
    using link = double2;
    static constexpr bool scaled = false;
    static constexpr bool bf16 = false;
};
struct F32 {
    using real = float;
    using elem = float2;
    using link = float2;
    static constexpr bool scaled = false;
    static constexpr bool bf16 = false;
};
struct F16 {
    using real = float;
    using elem = __half2;
    using link = __half2;  // two per link element: (ur, -ui), (ui, ur)
    static constexpr bool scaled = true;
    static constexpr bool bf16 = false;
};
// bfloat16 storage (FP32's exponent range, so no scale), FP32 arithmetic and
// the FP32 links
struct B16 {
    using real = float;
    using elem = bf16x2;
    using link = float2;
    static constexpr bool scaled = false;
    static constexpr bool bf16 = true;
};

template <class S> struct SpinorPtr {
    typename S::elem *p;
    float *scale;  // F16 only
    int N;
};

template <class S> __host__ __device__ inline SpinorPtr<S> make_spinor(void *base, int V, int N) {
    SpinorPtr<S> s;
    s.p = reinterpret_cast<typename S::elem *>(base);
    s.scale = S::scaled ? reinterpret_cast<float *>(s.p + (size_t)V * 12 * N) : nullptr;
    s.N = N;
    return s;
}

// NC > 0: the batch size is the compile-time constant NC, so the 12 component
// offsets of a site become immediate offsets of one address.
template <class S, int NC = 0>
__device__ __forceinline__ int batch_n(const SpinorPtr<S> &sp) {
    return NC > 0 ? NC : sp.N;
}

// The 12 components of (site, r) without the FP16 scale applied; returns the
// scale (1 for unscaled formats).
template <class S, int NC = 0>
__device__ __forceinline__ typename S::real load_site_raw(const SpinorPtr<S> &sp, int site, int r,
                                                          cplx<typename S::real> (&v)[12]) {
    const int N = batch_n<S, NC>(sp);
    const typename S::elem *q = sp.p + (size_t)site * 12 * N + r;
    if constexpr (S::scaled) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const float2 f = __half22float2(q[k * N]);
            v[k] = {f.x, f.y};
        }
        return sp.scale[(size_t)site * N + r];
    } else if constexpr (S::bf16) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const bf16x2 e = q[k * N];
            v[k] = {bf16_lo(e), bf16_hi(e)};
        }
        return typename S::real(1);
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const auto e = q[k * N];
            v[k] = {e.x, e.y};
        }
        return typename S::real(1);
    }
}

// The 12 stored elements of (site, r) as they are in memory (no conversion);
// returns the scale (1 for unscaled formats).
template <class S, int NC = 0>
__device__ __forceinline__ typename S::real load_site_elems(const SpinorPtr<S> &sp, int site, int r,
                                                            typename S::elem (&e)[12]) {
    const int N = batch_n<S, NC>(sp);
    const typename S::elem *q = sp.p + (size_t)site * 12 * N + r;
#pragma unroll
    for (int k = 0; k < 12; ++k) e[k] = q[k * N];
    if constexpr (S::scaled) return sp.scale[(size_t)site * N + r];
    else return typename S::real(1);
}

template <class S>
__device__ __forceinline__ void elems_to_cplx(const typename S::elem (&e)[12],
                                              cplx<typename S::real> (&v)[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        if constexpr (S::scaled) {
            const float2 f = __half22float2(e[k]);
            v[k] = {f.x, f.y};
        } else if constexpr (S::bf16) {
            v[k] = {bf16_lo(e[k]), bf16_hi(e[k])};
        } else {
            v[k] = {e[k].x, e[k].y};
        }
    }
}

// load_site for data read once (non-temporal loads: the lines are marked
// for early eviction and do not push out neighbour lines still to be re-read)
template <class S, int NC = 0>
__device__ __forceinline__ void load_site_once(const SpinorPtr<S> &sp, int site, int r,
                                               cplx<typename S::real> (&v)[12]) {
    const int N = batch_n<S, NC>(sp);
    const typename S::elem *q = sp.p + (size_t)site * 12 * N + r;
    using R = typename S::real;
    if constexpr (S::scaled) {
        const float sc = __builtin_nontemporal_load(sp.scale + (size_t)site * N + r);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            unsigned u = __builtin_nontemporal_load(reinterpret_cast<const unsigned *>(q + k * N));
            __half2 h;
            __builtin_memcpy(&h, &u, 4);
            const float2 f = __half22float2(h);
            v[k] = {f.x * sc, f.y * sc};
        }
    } else if constexpr (S::bf16) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const bf16x2 e{__builtin_nontemporal_load(&q[k * N].v)};
            v[k] = {bf16_lo(e), bf16_hi(e)};
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k)
            v[k] = {__builtin_nontemporal_load(&q[k * N].x), __builtin_nontemporal_load(&q[k * N].y)};
    }
    (void)sizeof(R);
}

template <class S, int NC = 0>
__device__ __forceinline__ void load_site(const SpinorPtr<S> &sp, int site, int r,
                                          cplx<typename S::real> (&v)[12]) {
    const typename S::real sc = load_site_raw<S, NC>(sp, site, r, v);
    if constexpr (S::scaled) {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = {v[k].re * sc, v[k].im * sc};
    }
}

// STREAM = true marks the stores non-temporal, so a kernel's output does not
// displace the input lines its neighbours still have to re-read from L2.
template <class S, bool STREAM = false, int NC = 0>
__device__ __forceinline__ void store_site(const SpinorPtr<S> &sp, int site, int r,
                                           const cplx<typename S::real> (&v)[12]) {
    const int N = batch_n<S, NC>(sp);
    const size_t base = (size_t)site * 12 * N + r;
    if constexpr (S::scaled) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        // a site-RHS whose largest part is below the FP32 normal range is
        // stored as zero (its reciprocal would overflow)
        if (!(m >= 1.17549435e-38f)) m = 0.f;
        const float inv = (m > 0.f) ? 1.0f / m : 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const __half2 h = __floats2half2_rn(v[k].re * inv, v[k].im * inv);
            if constexpr (STREAM) {
                unsigned u;
                __builtin_memcpy(&u, &h, 4);
                __builtin_nontemporal_store(u, reinterpret_cast<unsigned *>(sp.p + base + k * N));
            } else {
                sp.p[base + k * N] = h;
            }
        }
        if constexpr (STREAM)
            __builtin_nontemporal_store(m, sp.scale + (size_t)site * N + r);
        else
            sp.scale[(size_t)site * N + r] = m;
    } else if constexpr (S::bf16) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const bf16x2 e = bf16_pack(v[k].re, v[k].im);
            if constexpr (STREAM) __builtin_nontemporal_store(e.v, &sp.p[base + k * N].v);
            else sp.p[base + k * N] = e;
        }
    } else {
        using E = typename S::elem;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            E *q = sp.p + base + k * N;
            if constexpr (STREAM) {
                __builtin_nontemporal_store(v[k].re, &q->x);
                __builtin_nontemporal_store(v[k].im, &q->y);
            } else {
                E e;
                e.x = v[k].re;
                e.y = v[k].im;
                *q = e;
            }
        }
    }
}

// Gauge links [V][4][9] in the link type of the precision.
template <class S, class R>
__device__ __forceinline__ void load_link(const typename S::link *U, int site, int mu,
                                          cplx<R> (&u)[9]) {
    const typename S::link *q = U + ((size_t)site * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = {(R)q[k].x, (R)q[k].y};
}

// ---------------------------------------------------------------------------
// Spin projection (1 + sgn*gamma_mu) in the DeGrand-Rossi basis.  Rows 0 and 1
// give the half spinor h0 = psi0 + a0 psi_p0, h1 = psi1 + a1 psi_p1; rows 2
// and 3 are b2 h_q2 and b3 h_q3.  The unit factors below are those of
// (1 - gamma_mu); (1 + gamma_mu) negates all four (k -> k + 2).
template <int MU> struct Proj;
template <> struct Proj<0> { static constexpr int p0 = 3, a0 = 3, p1 = 2, a1 = 3, q2 = 1, b2 = 1, q3 = 0, b3 = 1; };
template <> struct Proj<1> { static constexpr int p0 = 3, a0 = 0, p1 = 2, a1 = 2, q2 = 1, b2 = 2, q3 = 0, b3 = 0; };
template <> struct Proj<2> { static constexpr int p0 = 2, a0 = 3, p1 = 3, a1 = 1, q2 = 0, b2 = 1, q3 = 1, b3 = 3; };
template <> struct Proj<3> { static constexpr int p0 = 2, a0 = 2, p1 = 3, a1 = 2, q2 = 0, b2 = 2, q3 = 1, b3 = 2; };

// h = rows 0,1 of (1 + SGN gamma_mu) psi; SGN = -1 or +1.
template <int MU, int SGN, class T>
__device__ __forceinline__ void project(const cplx<T> (&psi)[12], cplx<T> (&h)[6]) {
    using P = Proj<MU>;
    constexpr int sh = (SGN < 0) ? 0 : 2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h[c] = cadd(psi[c], cunit<P::a0 + sh>(psi[3 * P::p0 + c]));
        h[3 + c] = cadd(psi[3 + c], cunit<P::a1 + sh>(psi[3 * P::p1 + c]));
    }
}

// acc += full spinor of (1 + SGN gamma_mu) reconstructed from w = U h.
template <int MU, int SGN, class T>
__device__ __forceinline__ void reconstruct_add(cplx<T> (&acc)[12], const cplx<T> (&w)[6]) {
    using P = Proj<MU>;
    constexpr int sh = (SGN < 0) ? 0 : 2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = cadd(acc[c], w[c]);
        acc[3 + c] = cadd(acc[3 + c], w[3 + c]);
        acc[6 + c] = cadd(acc[6 + c], cunit<P::b2 + sh>(w[3 * P::q2 + c]));
        acc[9 + c] = cadd(acc[9 + c], cunit<P::b3 + sh>(w[3 * P::q3 + c]));
    }
}

// w = U h (both colour halves)
template <class T>
__device__ __forceinline__ void su3_mul(const cplx<T> (&u)[9], const cplx<T> (&h)[6], cplx<T> (&w)[6]) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cplx<T> s = cmul(u[3 * a + 0], h[3 * hh + 0]);
            s = cfma(s, u[3 * a + 1], h[3 * hh + 1]);
            s = cfma(s, u[3 * a + 2], h[3 * hh + 2]);
            w[3 * hh + a] = s;
        }
}

// w = U^dag h
template <class T>
__device__ __forceinline__ void su3_adj_mul(const cplx<T> (&u)[9], const cplx<T> (&h)[6], cplx<T> (&w)[6]) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cplx<T> s = cconjmul(u[0 + a], h[3 * hh + 0]);
            s = cfmaconj(s, u[3 + a], h[3 * hh + 1]);
            s = cfmaconj(s, u[6 + a], h[3 * hh + 2]);
            w[3 * hh + a] = s;
        }
}

// XCD-aware logical block index: the scheduler deals workgroups round-robin
// over the 8 XCDs, so block b runs on XCD b % 8.  Renumbering gives each XCD
// one contiguous range of logical blocks (and therefore of lattice sites).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// Loop of a (site, rhs) kernel body: thread (rl, ry) of a block of NT*SB
// threads handles RHS TILE*NT + rl and position ry of each group of SB
// consecutive processing positions that logical block LB of GB visits.
// Expects a Geom g and N, NT, SB in scope.
#define SITE_LOOP_BEGIN_AT(TILE, LB, GB)                                   \
    const int tid = threadIdx.x;                                           \
    const int rl = tid % NT;                                               \
    const int ry = tid / NT;                                               \
    const int r = (TILE) * NT + rl;                                        \
    const bool live = (ry < SB) && (r < N);                                \
    const int Lb = (LB);                                                   \
    const int Gb = (GB);                                                   \
    const Sweep sw_ = sweep((g.nsites + SB - 1) / SB, Lb, Gb);             \
    if (live)                                                              \
        for (int grp = sw_.first; grp < sw_.end; grp += sw_.step) {        \
            const int p_ = grp * SB + ry;                                  \
            if (p_ >= g.nsites) break;                                     \
            const int s = site_of(g, p_);

#define SITE_LOOP_BEGIN SITE_LOOP_BEGIN_AT(blockIdx.y, xcd_block(blockIdx.x, gridDim.x), gridDim.x)

#define SITE_LOOP_END }

}  // namespace wdt
