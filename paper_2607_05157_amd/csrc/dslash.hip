// Multi-RHS Wilson-Dirac operator for gfx950.
//
// (D psi)(x) = (4 + m0) psi(x) - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
//                                          + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
// (the 12x12-block nearest-neighbour operator of Sec. 1 in Wilson form), and
// D^dag = gamma5 D gamma5, which swaps the two projectors.
//
// Work decomposition: one thread per (site, right-hand side).  The RHS index
// is innermost in memory, so the lanes of a wavefront read contiguous runs of
// one spin-colour component across the batch (coalesced), and all lanes of a
// site read the same SU(3) link, which the memory pipeline fetches once per
// wavefront: the link bytes are amortised over the batch.  Each thread
// projects every neighbour to a half spinor (6 complex), applies the FP16
// scale and the link to the half spinor only, and reconstructs.
//
// Blocks handle SB sites x NT right-hand sides per step and sweep the lattice
// in a cache-blocked order, each XCD through one contiguous region, with
// about as many blocks as the GPU keeps resident, so neighbour re-reads find
// their lines in the XCD's L2.  For the common batch sizes the kernel is
// compiled with the batch size as a constant, which turns the component
// strides into immediate load offsets (no per-load address arithmetic).
//
// Optional epilogues fuse the per-RHS dot products BiCGStab needs right after
// an operator application, so the output is not read back from memory.
#include "internal.h"

#include <map>
#include <type_traits>

namespace wdt {

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
__global__ __launch_bounds__(256) void k_dslash(Geom g, const typename S::link *__restrict__ U,
                                                typename S::real diag, SpinorPtr<S> in,
                                                SpinorPtr<S> out, SpinorPtr<S> aux, int N, int NT,
                                                int SB, double2 *__restrict__ partials) {
    using R = typename S::real;
    constexpr int PIN = OpPin<S>::value;
    __shared__ double2 red[2][256];
    const int tid = threadIdx.x;
    const int rl = tid % NT;
    const int ry = tid / NT;
    const int r = blockIdx.y * NT + rl;
    const bool live = (ry < SB) && (r < N);
    const int Lb = xcd_block(blockIdx.x, gridDim.x);
    const Sweep sw = sweep((g.V + SB - 1) / SB, Lb, gridDim.x);
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
            const int Gt = gridDim.x;
            partials[((size_t)0 * Gt + Lb) * N + r] = s0;
            if (EPI != EPI_DOT_AUX) partials[((size_t)1 * Gt + Lb) * N + r] = s1;
        }
    }
}

// Batch sizes with a compiled-in constant (other sizes use the runtime path).
static int nc_of(int N) { return (N == 48 || N == 64 || N == 16) ? N : 0; }

template <class S> static int prec_of() {
    return std::is_same<S, F64>::value ? WDT_FP64 : std::is_same<S, F32>::value ? WDT_FP32 : WDT_FP16;
}

template <class S, int NC, bool DAG, int EPI>
static void launch_k(dim3 grid, int threads, hipStream_t stream, const Geom &g,
                     const typename S::link *U, typename S::real diag, SpinorPtr<S> pin_,
                     SpinorPtr<S> pout, SpinorPtr<S> paux, int N, int NT, int SB, double2 *part) {
    hipLaunchKernelGGL((k_dslash<S, NC, DAG, EPI>), grid, dim3(threads), 0, stream, g, U, diag,
                       pin_, pout, paux, N, NT, SB, part);
}

template <class S, bool DAG, int EPI>
static int launch_t(const wdt_gauge_s *gf, double m0, const void *in, void *out, const void *aux,
                    int N, double2 *partials, const Shape &sh, hipStream_t stream,
                    const typename S::link *U) {
    const Geom g = shaped_geom(gf->lat, sh);
    const int V = g.V;
    const dim3 grid(sh.G, sh.tiles);
    SpinorPtr<S> pin_ = make_spinor<S>(const_cast<void *>(in), V, N);
    SpinorPtr<S> pout = make_spinor<S>(out, V, N);
    SpinorPtr<S> paux = make_spinor<S>(const_cast<void *>(aux), V, N);
    const int prec = prec_of<S>();
    static const char *names[3] = {"dslash_fp64", "dslash_fp32", "dslash_fp16"};
    const int nvec = (EPI == EPI_DOT_AUX || EPI == EPI_RESID) ? 3 : 2;
    ProfScope prof(names[prec],
                   (double)V * ((double)N * nvec * site_bytes(prec) + 4.0 * link_bytes(prec)),
                   stream);
    const typename S::real diag = (typename S::real)(4.0 + m0);
    switch (nc_of(N)) {
        case 16:
            launch_k<S, 16, DAG, EPI>(grid, sh.threads, stream, g, U, diag, pin_, pout, paux, N,
                                     sh.NT, sh.SB, partials);
            break;
        case 48:
            launch_k<S, 48, DAG, EPI>(grid, sh.threads, stream, g, U, diag, pin_, pout, paux, N,
                                     sh.NT, sh.SB, partials);
            break;
        case 64:
            launch_k<S, 64, DAG, EPI>(grid, sh.threads, stream, g, U, diag, pin_, pout, paux, N,
                                     sh.NT, sh.SB, partials);
            break;
        default:
            launch_k<S, 0, DAG, EPI>(grid, sh.threads, stream, g, U, diag, pin_, pout, paux, N,
                                    sh.NT, sh.SB, partials);
            break;
    }
    WDT_HIP(hipGetLastError());
    return WDT_OK;
}

template <class S>
static int launch_p(const wdt_gauge_s *gf, double m0, int dagger, int epi, const void *in,
                    void *out, const void *aux, int N, double2 *partials, const Shape &sh,
                    hipStream_t stream, const typename S::link *U) {
#define WDT_EPI_CASE(E)                                                                      \
    case E:                                                                                  \
        return dagger ? launch_t<S, true, E>(gf, m0, in, out, aux, N, partials, sh, stream, U) \
                      : launch_t<S, false, E>(gf, m0, in, out, aux, N, partials, sh, stream, U);
    switch (epi) {
        WDT_EPI_CASE(EPI_NONE)
        WDT_EPI_CASE(EPI_DOT_AUX)
        WDT_EPI_CASE(EPI_DOT_TS)
        WDT_EPI_CASE(EPI_RESID)
        default:
            return set_error(WDT_EINVAL, "bad operator epilogue %d", epi);
    }
#undef WDT_EPI_CASE
}

int launch_dslash(const wdt_gauge_s *g, double m0, int prec, int dagger, int epi, const void *in,
                  void *out, const void *aux, int N, double2 *partials, const Shape &sh,
                  hipStream_t stream) {
    switch (prec) {
        case WDT_FP64:
            return launch_p<F64>(g, m0, dagger, epi, in, out, aux, N, partials, sh, stream, g->U64);
        case WDT_FP32:
            return launch_p<F32>(g, m0, dagger, epi, in, out, aux, N, partials, sh, stream, g->U32);
        case WDT_FP16:
            return launch_p<F16>(g, m0, dagger, epi, in, out, aux, N, partials, sh, stream, g->U32);
        default:
            return set_error(WDT_EINVAL, "bad precision %d", prec);
    }
}

// Resident blocks per CU of the operator kernel (the solve-time variant),
// used to size grids so that every block of a sweep is on the GPU at once.
template <class S, int NC>
static int occ_t(int threads) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dslash<S, NC, false, EPI_DOT_AUX>,
                                                     threads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

int op_blocks_per_cu(int prec, int N, int threads) {
    static std::map<long, int> cache;
    const long key = ((long)prec << 40) | ((long)N << 16) | threads;
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int nb = 0;
    const int nc = nc_of(N);
    switch (prec) {
        case WDT_FP64:
            nb = nc == 16 ? occ_t<F64, 16>(threads) : nc == 48 ? occ_t<F64, 48>(threads)
               : nc == 64 ? occ_t<F64, 64>(threads) : occ_t<F64, 0>(threads);
            break;
        case WDT_FP32:
            nb = nc == 16 ? occ_t<F32, 16>(threads) : nc == 48 ? occ_t<F32, 48>(threads)
               : nc == 64 ? occ_t<F32, 64>(threads) : occ_t<F32, 0>(threads);
            break;
        default:
            nb = nc == 16 ? occ_t<F16, 16>(threads) : nc == 48 ? occ_t<F16, 48>(threads)
               : nc == 64 ? occ_t<F16, 64>(threads) : occ_t<F16, 0>(threads);
            break;
    }
    cache[key] = nb;
    return nb;
}

}  // namespace wdt

extern "C" int wdt_apply_D(wdt_gauge g, double m0, const void *dev_in, void *dev_out,
                           int32_t n_rhs, int32_t prec, int32_t dagger, void *stream) {
    using namespace wdt;
    WDT_CHECK(g != nullptr, "wdt_apply_D: null gauge handle");
    WDT_CHECK(dev_in != nullptr && dev_out != nullptr, "wdt_apply_D: null vector");
    WDT_CHECK(dev_in != dev_out, "wdt_apply_D: input and output must not overlap");
    WDT_CHECK(n_rhs >= 1, "wdt_apply_D: n_rhs must be >= 1 (got %d)", n_rhs);
    WDT_CHECK(prec >= WDT_FP64 && prec <= WDT_FP16, "wdt_apply_D: bad precision %d", prec);
    WDT_CHECK(dagger == 0 || dagger == 1, "wdt_apply_D: dagger must be 0 or 1");
    const Shape sh = site_shape(g->lat, n_rhs, prec);
    return launch_dslash(g, m0, prec, dagger, EPI_NONE, dev_in, dev_out, nullptr, n_rhs, nullptr,
                         sh, (hipStream_t)stream);
}
