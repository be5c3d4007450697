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
};

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
//  stored after the V*12*N half2 values.
struct F64 {
    using real = double;
    using elem = double2;
    static constexpr bool scaled = false;
};
struct F32 {
    using real = float;
    using elem = float2;
    static constexpr bool scaled = false;
};
struct F16 {
    using real = float;
    using elem = __half2;
    static constexpr bool scaled = true;
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

template <class S>
__device__ __forceinline__ void load_site(const SpinorPtr<S> &sp, int site, int r,
                                          cplx<typename S::real> (&v)[12]) {
    const size_t base = (size_t)site * 12 * sp.N + r;
    if constexpr (S::scaled) {
        const float sc = sp.scale[(size_t)site * sp.N + r];
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            float2 f = __half22float2(sp.p[base + (size_t)k * sp.N]);
            v[k] = {f.x * sc, f.y * sc};
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            auto e = sp.p[base + (size_t)k * sp.N];
            v[k] = {e.x, e.y};
        }
    }
}

template <class S>
__device__ __forceinline__ void store_site(const SpinorPtr<S> &sp, int site, int r,
                                           const cplx<typename S::real> (&v)[12]) {
    const size_t base = (size_t)site * 12 * sp.N + r;
    if constexpr (S::scaled) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        const float inv = (m > 0.f) ? 1.0f / m : 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            sp.p[base + (size_t)k * sp.N] = __floats2half2_rn(v[k].re * inv, v[k].im * inv);
        sp.scale[(size_t)site * sp.N + r] = m;
    } else {
        using E = typename S::elem;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            E e;
            e.x = v[k].re;
            e.y = v[k].im;
            sp.p[base + (size_t)k * sp.N] = e;
        }
    }
}

// Gauge links [V][4][9] in the element type of the precision.
template <class S> struct LinkElem { using type = typename S::elem; };

template <class S, class R>
__device__ __forceinline__ void load_link(const typename S::elem *U, int site, int mu,
                                          cplx<R> (&u)[9]) {
    const typename S::elem *q = U + ((size_t)site * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if constexpr (S::scaled) {
            float2 f = __half22float2(q[k]);
            u[k] = {f.x, f.y};
        } else {
            u[k] = {(R)q[k].x, (R)q[k].y};
        }
    }
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

// Loop of a (site, rhs) kernel: thread (rl, ry) of a block of NT*SB threads
// handles RHS blockIdx.y*NT + rl and site ry of each group of SB sites in the
// block's chunk.  Expects V, N, NT, SB, chunk in scope.
#define SITE_LOOP_BEGIN                                              \
    const int tid = threadIdx.x;                                     \
    const int rl = tid % NT;                                         \
    const int ry = tid / NT;                                         \
    const int r = blockIdx.y * NT + rl;                              \
    const bool live = (ry < SB) && (r < N);                          \
    const int Lb = xcd_block(blockIdx.x, gridDim.x);                 \
    const int ngroups = (V + SB - 1) / SB;                           \
    const int g0 = Lb * chunk;                                       \
    const int g1 = min(ngroups, g0 + chunk);                         \
    if (live)                                                        \
        for (int grp = g0; grp < g1; ++grp) {                        \
            const int s = grp * SB + ry;                             \
            if (s >= V) break;

#define SITE_LOOP_END }

}  // namespace wdt
