// Multi-RHS Wilson-Dirac operator for gfx950.
//
// (D psi)(x) = (4 + m0) psi(x) - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
//                                          + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
// (the 12x12-block nearest-neighbour operator of Sec. 1 in Wilson form), and
// D^dag = gamma5 D gamma5, which swaps the two projectors.  A gauge with a
// clover term adds C(x) psi(x) (C Hermitian and gamma5-even, so the same
// term serves D and D^dag).
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
#include "kernels.h"

#include <map>
#include <type_traits>

namespace wdt {

template <class S, int NC, bool DAG, int EPI, bool WPS = false, int CLOV = 0>
__global__ __launch_bounds__(256) void k_dslash(Geom g, const typename S::link *__restrict__ U,
                                                const typename S::real *__restrict__ Cl,
                                                SpinorPtr<S> self, typename S::real cs,
                                                typename S::real ch, SpinorPtr<S> in,
                                                SpinorPtr<S> out, SpinorPtr<S> aux, int N, int NT,
                                                int SB, double2 *__restrict__ partials,
                                                int serial_tiles, const int *live) {
    // solver iterations: nothing to do once no RHS is iterating
    if (live && *live == 0) return;
    const int t0 = serial_tiles > 0 ? 0 : (int)blockIdx.y;
    const int t1 = serial_tiles > 0 ? serial_tiles : t0 + 1;
    dslash_body<S, NC, DAG, EPI, WPS, CLOV>(g, U, Cl, self, cs, ch, in, out, aux, N, NT, SB, partials, t0,
                                      t1, xcd_block(blockIdx.x, gridDim.x), gridDim.x);
}

template <class S, int NC, bool DAG, int EPI, bool WPS = false>
__global__ __launch_bounds__(256) void k_dslash_march(Geom g, const typename S::link *__restrict__ U,
                                                      typename S::real diag, SpinorPtr<S> in,
                                                      SpinorPtr<S> out, SpinorPtr<S> aux, int N,
                                                      int NT, int CB, int TC, int4 B,
                                                      double2 *__restrict__ partials,
                                                      const int *live) {
    if (live && *live == 0) return;
    dslash_march_body<S, NC, DAG, EPI, WPS>(g, U, diag, in, out, aux, N, NT, CB, TC, B, partials,
                                       blockIdx.y, xcd_block(blockIdx.x, gridDim.x), gridDim.x);
}

// Batch sizes with a compiled-in constant (other sizes use the runtime path).
static int nc_of(int N) { return (N == 48 || N == 64 || N == 16) ? N : 0; }

template <class S> static int prec_of() {
    return std::is_same<S, F64>::value   ? WDT_FP64
           : std::is_same<S, F32>::value ? WDT_FP32
           : std::is_same<S, B16>::value ? WDT_BF16
                                         : WDT_FP16;
}

template <class S>
struct HopPtrs {
    SpinorPtr<S> self, in, out, aux;
    typename S::real cs, ch;
    const int *live;
    const typename S::real *clov;  // the clover term, its inverse blocks, or null
    int cmode;                     // 1: add the clover term; 2: multiply by the inverse blocks
};

template <class S, int NC, bool DAG, int EPI>
static void launch_k(dim3 grid, int threads, hipStream_t stream, const Geom &g,
                     const typename S::link *U, const HopPtrs<S> &h, int N, int NT, int SB,
                     double2 *part, int serial_tiles, int tc, int4 brick, bool wps) {
    // the clover operator and the inverse-block launches: their own
    // instantiations (no t-march; D^dag only without an epilogue, the inverse
    // blocks only for D without one, which launch_t checks)
    if constexpr (!DAG || EPI == EPI_NONE) {
        if (h.clov && h.cmode == 1) {
            if constexpr (NC == 48 || NC == 64) {
                if (wps) {
                    hipLaunchKernelGGL((k_dslash<S, NC, DAG, EPI, true, 1>), grid,
                                       dim3(threads), 0, stream, g, U, h.clov, h.self, h.cs, h.ch,
                                       h.in, h.out, h.aux, N, NT, SB, part, serial_tiles, h.live);
                    return;
                }
            }
            hipLaunchKernelGGL((k_dslash<S, NC, DAG, EPI, false, 1>), grid, dim3(threads), 0,
                               stream, g, U, h.clov, h.self, h.cs, h.ch, h.in, h.out, h.aux, N,
                               NT, SB, part, serial_tiles, h.live);
            return;
        }
    }
    if constexpr (!DAG && EPI == EPI_NONE) {
        if (h.clov && h.cmode == 2) {
            if constexpr (NC == 48 || NC == 64) {
                if (wps) {
                    hipLaunchKernelGGL((k_dslash<S, NC, DAG, EPI, true, 2>), grid,
                                       dim3(threads), 0, stream, g, U, h.clov, h.self, h.cs, h.ch,
                                       h.in, h.out, h.aux, N, NT, SB, part, serial_tiles, h.live);
                    return;
                }
            }
            hipLaunchKernelGGL((k_dslash<S, NC, DAG, EPI, false, 2>), grid, dim3(threads), 0,
                               stream, g, U, h.clov, h.self, h.cs, h.ch, h.in, h.out, h.aux, N,
                               NT, SB, part, serial_tiles, h.live);
            return;
        }
    }
    // the t-march covers the whole lattice with the operator's own form
    const bool march = tc > 0 && g.parity < 0 && h.self.p == h.in.p && h.ch == (typename S::real)(-0.5);
    if constexpr (NC == 48 || NC == 64) {
        if (wps && !march) {
            hipLaunchKernelGGL((k_dslash<S, NC, DAG, EPI, true>), grid, dim3(threads), 0, stream,
                               g, U, h.clov, h.self, h.cs, h.ch, h.in, h.out, h.aux, N, NT, SB,
                               part, serial_tiles, h.live);
            return;
        }
        if (wps && march) {
            hipLaunchKernelGGL((k_dslash_march<S, NC, DAG, EPI, true>), grid, dim3(threads), 0,
                               stream, g, U, h.cs, h.in, h.out, h.aux, N, NT, SB, tc, brick,
                               part, h.live);
            return;
        }
    }
    if (march)
        hipLaunchKernelGGL((k_dslash_march<S, NC, DAG, EPI>), grid, dim3(threads), 0, stream, g,
                           U, h.cs, h.in, h.out, h.aux, N, NT, SB, tc, brick, part, h.live);
    else
        hipLaunchKernelGGL((k_dslash<S, NC, DAG, EPI>), grid, dim3(threads), 0, stream, g, U,
                           h.clov, h.self, h.cs, h.ch, h.in, h.out, h.aux, N, NT, SB, part, serial_tiles,
                           h.live);
}

template <class S, bool DAG, int EPI>
static int launch_t(const wdt_gauge_s *gf, const HopSpec &hs, const void *in, void *out,
                    const void *aux, int N, double2 *partials, const Shape &sh0,
                    hipStream_t stream, const typename S::link *U) {
    Shape sh = sh0;
    Geom g = shaped_geom(gf->lat, sh);
    const int V = g.V;
    if (hs.parity >= 0) {
        // one parity: plain or brick order, no t-march
        g = gf->lat.geom();
        g.parity = hs.parity;
        g.nsites = V / 2;
        if (sh.parity_brick.x > 0) {
            g.bx = sh.parity_brick.x;
            g.by = sh.parity_brick.y;
            g.bz = sh.parity_brick.z;
        }
        sh.tc = 0;
    }
    // one site per wavefront: 64 lanes per site, four sites per block
    const bool wps = sh.wps && (nc_of(N) == 48 || nc_of(N) == 64);
    const int NT = wps ? 64 : sh.NT, SB = wps ? 4 : sh.SB, threads = wps ? 256 : sh.threads;
    const int tiles = (N + NT - 1) / NT;
    dim3 grid(sh.G, (sh.serial && sh.tc == 0) ? 1 : tiles);
    // One-parity pure hops need fewer registers than the other operator
    // launches (no own term, no epilogue: six waves per SIMD fit), and with a
    // gather-latency-bound kernel the extra resident waves pay: six blocks per
    // CU instead of four (measured 166 -> 155 us per FP16 launch on 16^3 x 32,
    // 48 RHS; eight: 162 us, three: 182 us).
    if (wps && hs.parity >= 0 && hs.cs == 0.0 && tuning().gmax == 0 && sh.G % 32 == 0)
        grid.x = sh.G / 4 * 6;
    const int serial_tiles = sh.serial ? tiles : 0;
    HopPtrs<S> h;
    h.in = make_spinor<S>(const_cast<void *>(in), V, N);
    h.self = make_spinor<S>(const_cast<void *>(hs.self ? hs.self : in), V, N);
    h.out = make_spinor<S>(out, V, N);
    h.aux = make_spinor<S>(const_cast<void *>(aux), V, N);
    h.cs = (typename S::real)hs.cs;
    h.ch = (typename S::real)hs.ch;
    h.live = hs.live;
    h.clov = nullptr;
    h.cmode = 0;
    if (hs.clover) {
        if (DAG && EPI != EPI_NONE)
            return set_error(WDT_EINVAL, "clover operator: D^dag with an epilogue is not built");
        if constexpr (std::is_same<typename S::real, double>::value) h.clov = gf->C64;
        else h.clov = gf->C32;
        h.cmode = 1;
    } else if (hs.clover_inv) {
        if (DAG || EPI != EPI_NONE)
            return set_error(WDT_EINVAL, "clover inverse blocks: D without an epilogue only");
        if constexpr (std::is_same<typename S::real, double>::value) h.clov = gf->Ci64;
        else h.clov = gf->Ci32;
        h.cmode = 2;
    }
    const int prec = prec_of<S>();
    // timing classes: the whole-lattice operator, one-parity pure hops, and
    // one-parity launches with the site's own term (the even-odd operator's
    // second half, residuals, reconstruction)
    static const char *names[3][4] = {
        {"dslash_fp64", "dslash_fp32", "dslash_fp16", "dslash_bf16"},
        {"dslash_hop_fp64", "dslash_hop_fp32", "dslash_hop_fp16", "dslash_hop_bf16"},
        {"dslash_eo_fp64", "dslash_eo_fp32", "dslash_eo_fp16", "dslash_eo_bf16"}};
    const int kind = hs.parity < 0 ? 0 : hs.cs == 0.0 ? 1 : 2;
    // algorithmic bytes: in, out, a separate self, the epilogue's vector, links once
    const int nvec = 2 + ((hs.cs != 0.0 && hs.self && hs.self != in) ? 1 : 0) +
                     ((EPI == EPI_DOT_AUX || EPI == EPI_RESID || EPI == EPI_DOT_TSR) ? 1 : 0);
    const double clov_bytes =
        h.clov ? (double)g.nsites * CLOVER_REALS * sizeof(typename S::real) : 0.0;
    ProfScope prof(names[kind][prec],
                   (double)g.nsites * N * nvec * site_bytes(prec) + 4.0 * V * link_bytes(prec) +
                       clov_bytes,
                   stream);
    switch (nc_of(N)) {
        case 16:
            launch_k<S, 16, DAG, EPI>(grid, threads, stream, g, U, h, N, NT, SB, partials,
                                     serial_tiles, sh.tc, sh.brick, sh.wps);
            break;
        case 48:
            launch_k<S, 48, DAG, EPI>(grid, threads, stream, g, U, h, N, NT, SB, partials,
                                     serial_tiles, sh.tc, sh.brick, sh.wps);
            break;
        case 64:
            launch_k<S, 64, DAG, EPI>(grid, threads, stream, g, U, h, N, NT, SB, partials,
                                     serial_tiles, sh.tc, sh.brick, sh.wps);
            break;
        default:
            launch_k<S, 0, DAG, EPI>(grid, threads, stream, g, U, h, N, NT, SB, partials,
                                    serial_tiles, sh.tc, sh.brick, sh.wps);
            break;
    }
    WDT_HIP(hipGetLastError());
    return WDT_OK;
}

template <class S>
static int launch_p(const wdt_gauge_s *gf, const HopSpec &hs, int dagger, int epi,
                    const void *in, void *out, const void *aux, int N, double2 *partials,
                    const Shape &sh, hipStream_t stream, const typename S::link *U) {
#define WDT_EPI_CASE(E)                                                                          \
    case E:                                                                                      \
        return dagger ? launch_t<S, true, E>(gf, hs, in, out, aux, N, partials, sh, stream, U)   \
                      : launch_t<S, false, E>(gf, hs, in, out, aux, N, partials, sh, stream, U);
    switch (epi) {
        WDT_EPI_CASE(EPI_NONE)
        WDT_EPI_CASE(EPI_DOT_AUX)
        WDT_EPI_CASE(EPI_DOT_TS)
        WDT_EPI_CASE(EPI_RESID)
        WDT_EPI_CASE(EPI_DOT_TSR)
        WDT_EPI_CASE(EPI_NORM)
        default:
            return set_error(WDT_EINVAL, "bad operator epilogue %d", epi);
    }
#undef WDT_EPI_CASE
}

int launch_hop(const wdt_gauge_s *g, int prec, int dagger, int epi, const HopSpec &hs,
               const void *in, void *out, const void *aux, int N, double2 *partials,
               const Shape &sh, hipStream_t stream) {
    if (hs.parity >= 0 && !g->lat.even_odd_ok())
        return set_error(WDT_EINVAL, "one-parity operator on a lattice with an odd extent");
    if (hs.clover && (hs.cs == 0.0 || hs.clover_inv || !g->C64))
        return set_error(WDT_EINVAL, "clover term: needs the site's own term and a clover gauge");
    if (hs.clover_inv && !g->Ci64)
        return set_error(WDT_EINVAL, "clover inverse blocks not computed");
    switch (prec) {
        case WDT_FP64:
            return launch_p<F64>(g, hs, dagger, epi, in, out, aux, N, partials, sh, stream, g->U64);
        case WDT_FP32:
            return launch_p<F32>(g, hs, dagger, epi, in, out, aux, N, partials, sh, stream, g->U32);
        case WDT_FP16:
            return launch_p<F16>(g, hs, dagger, epi, in, out, aux, N, partials, sh, stream, g->U16);
        case WDT_BF16:
            return launch_p<B16>(g, hs, dagger, epi, in, out, aux, N, partials, sh, stream, g->U32);
        default:
            return set_error(WDT_EINVAL, "bad precision %d", prec);
    }
}

int launch_dslash(const wdt_gauge_s *g, double m0, int prec, int dagger, int epi, const void *in,
                  void *out, const void *aux, int N, double2 *partials, const Shape &sh,
                  hipStream_t stream) {
    HopSpec hs;
    hs.parity = -1;
    hs.self = in;
    hs.cs = 4.0 + m0;
    hs.ch = -0.5;
    hs.clover = g->C64 != nullptr;
    return launch_hop(g, prec, dagger, epi, hs, in, out, aux, N, partials, sh, stream);
}

// Resident blocks per CU of the operator kernel (the solve-time variant),
// used to size grids so that every block of a sweep is on the GPU at once.
template <class S, int NC>
static int occ_t(int threads, int mode) {
    int nb = 0;
    hipError_t e;
    if (mode == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, k_dslash_march<S, NC, false, EPI_DOT_AUX>, threads, 0);
    else if (mode == 2 && (NC == 48 || NC == 64))
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, k_dslash<S, NC, false, EPI_DOT_AUX, (NC == 48 || NC == 64)>, threads, 0);
    else if (mode == 3 && (NC == 48 || NC == 64))
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, k_dslash_march<S, NC, false, EPI_DOT_AUX, (NC == 48 || NC == 64)>, threads, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, k_dslash<S, NC, false, EPI_DOT_AUX>, threads, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

template <class S>
static int occ_p(int N, int threads, int mode) {
    switch (nc_of(N)) {
        case 16: return occ_t<S, 16>(threads, mode);
        case 48: return occ_t<S, 48>(threads, mode);
        case 64: return occ_t<S, 64>(threads, mode);
        default: return occ_t<S, 0>(threads, mode);
    }
}

int op_blocks_per_cu(int prec, int N, int threads, int mode) {
    static std::map<long, int> cache;
    const long key = ((long)prec << 42) | ((long)mode << 40) | ((long)N << 16) | threads;
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const int nb = prec == WDT_FP64   ? occ_p<F64>(N, threads, mode)
                   : prec == WDT_FP32 ? occ_p<F32>(N, threads, mode)
                   : prec == WDT_BF16 ? occ_p<B16>(N, threads, mode)
                                      : occ_p<F16>(N, threads, mode);
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
    WDT_CHECK(prec >= WDT_FP64 && prec <= WDT_BF16, "wdt_apply_D: bad precision %d", prec);
    WDT_CHECK(dagger == 0 || dagger == 1, "wdt_apply_D: dagger must be 0 or 1");
    const Shape sh = site_shape(g->lat, n_rhs, prec);
    return launch_dslash(g, m0, prec, dagger, EPI_NONE, dev_in, dev_out, nullptr, n_rhs, nullptr,
                         sh, (hipStream_t)stream);
}
