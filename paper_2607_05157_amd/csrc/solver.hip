// Batched BiCGStab for D x = b (one independent recurrence per right-hand
// side, Sec. 1: every stochastic sample needs one solve with D), in FP64 or
// as an FP64 defect-correction loop around an FP32-arithmetic inner solve
// whose vectors are stored in FP32 or FP16 (with a per-site-per-RHS scale).
//
// Per iteration the vector work is:
//   v = D p                 (operator, fused rhat^dag v)
//   s = r - alpha v
//   t = D s                 (operator, fused t^dag s and ||t||^2)
//   x += alpha p + omega s,  r = s - omega t   (fused rhat^dag r, ||r||^2)
//   p = r + beta (p - omega v)
// Per-RHS scalars live on the device; small reduction kernels turn the
// per-block dot partials into alpha, omega, beta and the convergence flags, so
// the host reads one "still iterating" flag per iteration, one iteration
// behind the device so the queue never drains.  All sums use
// a fixed order, so results are bit-reproducible run to run.
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace wdt {

__global__ void k_init_state(RhsState *st, const double2 *partials, int G, int N, double tol,
                             const int *mask, const double *tolr, const double *bbv) {
    init_state_body(st, partials, G, N, tol, mask, tolr, bbv, blockIdx.x);
}
__global__ void k_scalar_alpha(RhsState *st, const double2 *partials, int G, int N) {
    scalar_alpha_body(st, partials, G, N, blockIdx.x);
}
__global__ void k_scalar_omega(RhsState *st, const double2 *partials, int G, int N) {
    scalar_omega_body(st, partials, G, N, blockIdx.x);
}
__global__ void k_scalar_beta(RhsState *st, const double2 *partials, int G, int N) {
    scalar_beta_body(st, partials, G, N, blockIdx.x);
}
__global__ void k_scalar_omega_beta(RhsState *st, const double2 *partials, int G, int N) {
    scalar_omega_beta_body(st, partials, G, N, blockIdx.x);
}
__global__ void k_scalar_check(RhsState *st, const double2 *partials, int G, int N) {
    scalar_check_body(st, partials, G, N, blockIdx.x);
}
__global__ void k_live(const RhsState *st, int N, int *live, int *host) {
    live_body(st, N, live, host);
}
// out[r] = the sum of partials slot 0 over G blocks
__global__ void k_sum_to(double *out, const double2 *partials, int G, int N) {
    const double2 v = block_sum(partials, 0, G, N, blockIdx.x);
    if (threadIdx.x == 0) out[blockIdx.x] = v.x;
}

// The vector kernels of an iteration return at once when no RHS is iterating
// (*live == 0): the host learns of convergence one iteration late, and the
// iteration it has already queued by then costs only its launches.
#define WDT_LIVE_GUARD \
    if (live && *live == 0) return;

#define WDT_BLOCK_CTX blockIdx.y, xcd_block(blockIdx.x, gridDim.x), gridDim.x

template <class S, bool STREAMV = false>
__global__ __launch_bounds__(256) void k_update_s(Geom g, int N, int NT, int SB,
                                                  const RhsState *__restrict__ st, SpinorPtr<S> rv,
                                                  SpinorPtr<S> vv, SpinorPtr<S> sv,
                                                  const int *live) {
    WDT_LIVE_GUARD
    update_s_body<S, STREAMV>(g, N, NT, SB, st, rv, vv, sv, WDT_BLOCK_CTX);
}
template <class S, bool STREAMV = false>
__global__ __launch_bounds__(256) void k_update_xr(Geom g, int N, int NT, int SB,
                                                   const RhsState *__restrict__ st, SpinorPtr<S> xv,
                                                   SpinorPtr<S> pv, SpinorPtr<S> sv,
                                                   SpinorPtr<S> tv, SpinorPtr<S> rv,
                                                   SpinorPtr<S> rhat, double2 *partials,
                                                   const int *live) {
    WDT_LIVE_GUARD
    update_xr_body<S, STREAMV>(g, N, NT, SB, st, xv, pv, sv, tv, rv, rhat, partials, WDT_BLOCK_CTX);
}
template <class S, bool STREAMV = false>
__global__ __launch_bounds__(256) void k_update_p(Geom g, int N, int NT, int SB,
                                                  const RhsState *__restrict__ st, SpinorPtr<S> rv,
                                                  SpinorPtr<S> pv, SpinorPtr<S> vv,
                                                  const int *live) {
    WDT_LIVE_GUARD
    update_p_body<S, STREAMV>(g, N, NT, SB, st, rv, pv, vv, WDT_BLOCK_CTX);
}
template <class S, bool STREAMV = false>
__global__ __launch_bounds__(256) void k_update_xrp(Geom g, int N, int NT, int SB,
                                                    const RhsState *__restrict__ st, SpinorPtr<S> xv,
                                                    SpinorPtr<S> pv, SpinorPtr<S> sv,
                                                    SpinorPtr<S> tv, SpinorPtr<S> rv,
                                                    SpinorPtr<S> vv, double2 *partials,
                                                    const int *live) {
    WDT_LIVE_GUARD
    update_xrp_body<S, STREAMV>(g, N, NT, SB, st, xv, pv, sv, tv, rv, vv, partials, WDT_BLOCK_CTX);
}
template <class S>
__global__ __launch_bounds__(256) void k_norm(Geom g, int N, int NT, int SB, SpinorPtr<S> src,
                                              double2 *__restrict__ partials) {
    norm_body<S>(g, N, NT, SB, src, partials, WDT_BLOCK_CTX);
}
template <class SS, class SD, bool ADD>
__global__ __launch_bounds__(256) void k_convert(Geom g, int N, int NT, int SB,
                                                 SpinorPtr<SS> src, SpinorPtr<SD> dst,
                                                 SpinorPtr<SD> dst2,
                                                 const double *__restrict__ f,
                                                 double2 *__restrict__ partials) {
    convert_body<SS, SD, ADD>(g, N, NT, SB, src, dst, dst2, f, partials, WDT_BLOCK_CTX);
}

// ---------------------------------------------------------------------------
// Host side.

LaunchTuning &tuning() {
    static LaunchTuning t;
    return t;
}

// Default RHS tile: the largest divisor of N not above a per-precision target
// (narrower tiles for wider storage keep the per-site footprint small), or
// the target itself.
static int default_nt(int N, int prec) {
    const int target = prec == WDT_FP64 ? 8 : prec == WDT_FP32 ? 16 : 48;
    if (N <= target) return N;
    for (int d = target; d >= 8; --d)
        if (N % d == 0) return d;
    return target;
}

static int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            cus = p.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

Shape site_shape(const wdt_lattice_s &lat, int N, int prec) {
    const LaunchTuning &tu = tuning();
    const int64_t V = lat.V;
    Shape sh;
    int NT = tu.nt > 0 ? tu.nt : default_nt(N, prec);
    NT = std::min(std::min(NT, N), 256);
    sh.NT = NT;
    sh.tiles = (N + NT - 1) / NT;
    int SB = std::max(1, 256 / NT);
    if (tu.sb > 0) {
        SB = std::min(tu.sb, SB);
    } else {
        // prefer full wavefronts: largest SB <= 256/NT with NT*SB a multiple of 64
        for (int sb = SB; sb >= 1; --sb)
            if ((NT * sb) % 64 == 0) {
                SB = sb;
                break;
            }
    }
    sh.SB = SB;
    sh.threads = ((NT * SB + 63) / 64) * 64;
    const int64_t ngroups = (V + SB - 1) / SB;
    // about as many blocks as the GPU keeps resident (operator kernel occupancy)
    // FP64 sweeps are limited by L2 capacity (wide sites): one block per CU
    // keeps the XCD front small; narrower formats fill the CU
    int per_cu = prec == WDT_FP64 ? 1 : op_blocks_per_cu(prec, N, sh.threads, 0);
    if (per_cu <= 0) per_cu = 2;
    const int64_t Gdef = (int64_t)device_cus() * per_cu;
    int64_t G = std::min<int64_t>(ngroups, tu.gmax > 0 ? tu.gmax : Gdef);
    // XCD-aware renumbering needs a multiple of 8 (a tuner override is taken
    // as given, so that the plain round-robin mapping can be measured too)
    if (G >= 8 && tu.gmax <= 0) G = (G / 8) * 8;
    sh.G = (int)std::max<int64_t>(G, 1);
    // streaming vector kernels have no reuse to protect: fill the CUs
    int64_t Gv = std::min<int64_t>(ngroups, (int64_t)device_cus() * 4);
    if (Gv >= 8) Gv = (Gv / 8) * 8;
    sh.Gv = (int)std::max<int64_t>(Gv, 1);
    // processing-order tile: z-slabs thin enough that two t-strides of the
    // input tile fit in about 2 MB of L2, whole extent in t
    const int Lz = lat.dims[2];
    const double foot = (double)NT * site_bytes(prec);
    int bz = Lz;
    if (tu.bz > 0 && Lz % tu.bz == 0) {
        bz = tu.bz;
    } else {
        for (int d = Lz; d >= 1; --d)
            if (Lz % d == 0) {
                bz = d;
                if (2.0 * lat.dims[0] * lat.dims[1] * d * foot <= (prec == WDT_FP64 ? 2.0e6 : 6.0e6))
                    break;
            }
    }
    sh.bz = bz;
    sh.bt = lat.dims[3];
    sh.serial = tu.serial > 0;
    // One site per wavefront (operator only; batches of 48 or 64): the links
    // go through the scalar cache, which frees the vector memory pipeline
    // that otherwise limits the operator.  Four blocks per CU: more resident
    // blocks only widen each XCD's front beyond what its L2 holds.
    sh.wps = (tu.wps > 0 || (tu.wps < 0 && tu.nt == 0)) && (N == 48 || N == 64);
    if (sh.wps) {
        const int pw = 4;
        int64_t Gw = std::min<int64_t>((V + 3) / 4, tu.gmax > 0 ? tu.gmax : (int64_t)device_cus() * pw);
        if (Gw >= 8 && tu.gmax <= 0) Gw = (Gw / 8) * 8;
        sh.G = (int)std::max<int64_t>(Gw, 1);
    }
    // Brick order of the site sweep: each XCD's front, its share of the
    // resident blocks, covers one slice of a compact brick of columns and
    // moves through t, so spatial neighbours are read while their lines are
    // in flight or fresh in the XCD's L2 and t-neighbours one slice later.
    sh.sweep_brick = make_int4(0, 0, 0, 0);
    if (tu.brick > 0) {
        const int bx = tu.brick / 10000, by = (tu.brick / 100) % 100, bz = tu.brick % 100;
        if (bx > 0 && by > 0 && bz > 0 && lat.dims[0] % bx == 0 && lat.dims[1] % by == 0 &&
            lat.dims[2] % bz == 0)
            sh.sweep_brick = make_int4(bx, by, bz, 0);
    } else if (tu.brick == 0 && sh.wps) {
        const int64_t front = (int64_t)std::max(1, sh.G / 8) * 4;  // sites per XCD front
        int64_t best_vol = 0;
        double best_surface = 1e30;
        for (int bx = 1; bx <= lat.dims[0]; ++bx) {
            if (lat.dims[0] % bx) continue;
            for (int by = 1; by <= lat.dims[1]; ++by) {
                if (lat.dims[1] % by) continue;
                for (int bz = 1; bz <= lat.dims[2]; ++bz) {
                    if (lat.dims[2] % bz) continue;
                    const int64_t vol = (int64_t)bx * by * bz;
                    if (vol > front) continue;
                    const double surface = 2.0 / bx + 2.0 / by + 2.0 / bz;
                    if (vol > best_vol || (vol == best_vol && surface < best_surface)) {
                        sh.sweep_brick = make_int4(bx, by, bz, 0);
                        best_vol = vol;
                        best_surface = surface;
                    }
                }
            }
        }
        // bricks far smaller than the front gain nothing over the plain order
        if (best_vol * 4 < front) sh.sweep_brick = make_int4(0, 0, 0, 0);
    }
    // One-parity sweeps (even-odd solvers): a brick slice holds half as many
    // sites of the parity, so the brick may be twice the front; x extent even.
    sh.parity_brick = make_int4(0, 0, 0, 0);
    if (tu.brick > 0) {
        if (sh.sweep_brick.x > 0 && sh.sweep_brick.x % 2 == 0) sh.parity_brick = sh.sweep_brick;
    } else if (tu.brick == 0 && sh.wps && lat.even_odd_ok()) {
        const int64_t front = (int64_t)std::max(1, sh.G / 8) * 4;
        int64_t best_vol = 0;
        double best_surface = 1e30;
        for (int bx = 2; bx <= lat.dims[0]; bx += 2) {
            if (lat.dims[0] % bx) continue;
            for (int by = 1; by <= lat.dims[1]; ++by) {
                if (lat.dims[1] % by) continue;
                for (int bz = 1; bz <= lat.dims[2]; ++bz) {
                    if (lat.dims[2] % bz) continue;
                    const int64_t vol = (int64_t)bx * by * bz;
                    if (vol > 2 * front) continue;
                    const double surface = 2.0 / bx + 2.0 / by + 2.0 / bz;
                    if (vol > best_vol || (vol == best_vol && surface < best_surface)) {
                        sh.parity_brick = make_int4(bx, by, bz, 0);
                        best_vol = vol;
                        best_surface = surface;
                    }
                }
            }
        }
        if (best_vol * 2 < front) sh.parity_brick = make_int4(0, 0, 0, 0);
    }
    // t-marching operator: chunks of tc slices over bricks of columns
    sh.tc = 0;
    sh.brick = make_int4(0, 0, 0, 0);
    const int Lt = lat.dims[3];
    const int tcq = tu.tchunk > 0 ? tu.tchunk : 0;
    // columns per block: 4 with one column per wavefront, else the site tile
    const int CBm = sh.wps ? 4 : SB;
    if (tcq > 0 && Lt % tcq == 0) {
        int pm = sh.wps ? op_blocks_per_cu(prec, N, 256, 3) : op_blocks_per_cu(prec, N, sh.threads, 1);
        if (pm <= 0) pm = 2;
        const int64_t resident = tu.gmax > 0 ? tu.gmax : (int64_t)device_cus() * pm;
        // columns one XCD marches at once: its share of the resident blocks
        const int64_t cap = std::max<int64_t>(1, resident / 8) * CBm;
        int4 best = make_int4(0, 0, 0, 0);
        double best_surface = 1e30;
        int64_t best_vol = 0;
        for (int bx = CBm; bx <= lat.dims[0]; bx += CBm) {
            if (lat.dims[0] % bx) continue;
            for (int by = 1; by <= lat.dims[1]; ++by) {
                if (lat.dims[1] % by) continue;
                for (int bz = 1; bz <= lat.dims[2]; ++bz) {
                    if (lat.dims[2] % bz) continue;
                    const int64_t vol = (int64_t)bx * by * bz;
                    if (vol > cap) continue;
                    // neighbour reads that leave the brick, per site
                    const double surface = 2.0 / bx + 2.0 / by + 2.0 / bz;
                    if (vol > best_vol || (vol == best_vol && surface < best_surface)) {
                        best = make_int4(bx, by, bz, 0);
                        best_vol = vol;
                        best_surface = surface;
                    }
                }
            }
        }
        if (best_vol > 0) {
            sh.tc = tcq;
            sh.brick = best;
            const int64_t upb = best_vol / CBm;
            const int64_t units = (V / Lt) / CBm * (Lt / tcq);
            int64_t Gm;
            if (tu.gmax > 0) {
                Gm = std::min<int64_t>(units, tu.gmax);
            } else {
                // whole bricks per XCD round
                const int64_t k = std::max<int64_t>(1, resident / (8 * upb));
                Gm = std::min<int64_t>(units, 8 * upb * k);
                if (Gm >= 8) Gm = (Gm / 8) * 8;
            }
            sh.G = (int)std::max<int64_t>(Gm, 1);
        }
    }
    return sh;
}

Geom shaped_geom(const wdt_lattice_s &lat, const Shape &sh) {
    Geom g = lat.geom();
    g.bz = sh.bz;
    g.bt = sh.bt;
    if (sh.tc == 0 && sh.sweep_brick.x > 0) {
        g.bx = sh.sweep_brick.x;
        g.by = sh.sweep_brick.y;
        g.bz = sh.sweep_brick.z;
    }
    return g;
}

namespace {

struct SolveWs {
    RhsState *st;
    double2 *partials;
    void *vec[8];
};

template <class S>
SpinorPtr<S> sp(void *p, int V, int N) {
    return make_spinor<S>(p, V, N);
}

int ensure_ws(wdt_gauge_s *g, size_t bytes) {
    if (g->ws.bytes >= bytes) return WDT_OK;
    if (g->ws.ptr) WDT_HIP(hipFree(g->ws.ptr));
    g->ws.ptr = nullptr;
    g->ws.bytes = 0;
    hipError_t e = hipMalloc(&g->ws.ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(WDT_ENOMEM, "workspace allocation of %zu bytes failed", bytes);
    }
    g->ws.bytes = bytes;
    return WDT_OK;
}

struct Bicg {
    wdt_gauge_s *g;
    double m0;
    int N, V;
    Shape sh;
    Geom geo;
    int NT;
    dim3 grid;
    hipStream_t stream;
    RhsState *st;
    double2 *part;
    bool eo = false;  // iterate on the even-site Schur complement
    int *live = nullptr;            // device flag: some RHS is iterating
    int *live_host = nullptr;       // two host-mapped slots the iterations write in turn
    int *live_dev_slots = nullptr;  // the same slots, device address
};

// Two host-mapped ints per gauge handle for the iteration loop's flag.
int ensure_live_slots(wdt_gauge_s *g) {
    if (g->live_host) return WDT_OK;
    void *h = nullptr;
    if (hipHostMalloc(&h, 256, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(WDT_ENOMEM, "host-mapped flag allocation failed");
    }
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(h);
        return set_error(WDT_EHIP, "host-mapped flag: no device address");
    }
    g->live_host = (int *)h;
    g->live_dev = (int *)d;
    return WDT_OK;
}

// Binds the flag slots: the device flag at `dev_flag` (workspace memory).
int bind_live(Bicg &B, int *dev_flag) {
    WDT_TRY(ensure_live_slots(B.g));
    B.live = dev_flag;
    B.live_host = B.g->live_host;
    B.live_dev_slots = B.g->live_dev;
    return WDT_OK;
}

// Even-odd preconditioning: on when every extent is even, unless the tuner
// switches it off.
bool use_even_odd(const wdt_gauge_s *g) {
    const int eo = tuning().eo;
    return g->lat.even_odd_ok() && eo != 0;
}

// The geometry of the sites of one parity, in plain order.
Geom parity_geom(const wdt_lattice_s &lat, int parity) {
    Geom g = lat.geom();
    g.parity = parity;
    g.nsites = (int)(lat.V / 2);
    return g;
}

// Even-odd (Schur) preconditioning on a lattice with every extent even.
// With a = 4 + m0 and H the hop sum (D = a - H/2), the odd sites are
// eliminated:
//   M x_e = a x_e - (1/(4a)) H_eo H_oe x_e = b_e + (1/(2a)) H_eo b_o =: b'_e,
//   x_o = (1/a) b_o + (1/(2a)) H_oe x_e.
// With a clover term the site's own term is the block A = a + C(x) and 1/a
// becomes A_oo^-1 (inverse blocks on the odd sites, applied in the hop
// launch that produces the odd-site vector):
//   M x_e = A_ee x_e - (1/4) H_eo A_oo^-1 H_oe x_e,
//   x_o = A_oo^-1 (b_o + (1/2) H_oe x_e).
// The residual of x = (x_e, x_o) is then b'_e - M x_e on the even sites and
// exactly zero on the odd ones, so the Schur residual is the true residual.
// Vectors keep the full-lattice layout; the iteration touches even sites only
// and uses the odd sites of its output vector as scratch for H_oe x_e.
int apply_op(Bicg &B, int prec, int epi, const void *in, void *out, const void *aux) {
    const double a = 4.0 + B.m0;
    if (!B.eo) {
        HopSpec h;
        h.self = in;
        h.cs = a;
        h.ch = -0.5;
        h.live = B.live;
        h.clover = B.g->C64 != nullptr;
        return launch_hop(B.g, prec, 0, epi, h, in, out, aux, B.N, B.part, B.sh, B.stream);
    }
    const bool clov = B.g->C64 != nullptr;
    HopSpec h1;
    h1.parity = 1;
    h1.cs = 0.0;
    h1.ch = 1.0;
    h1.live = B.live;
    h1.clover_inv = clov;
    WDT_TRY(launch_hop(B.g, prec, 0, EPI_NONE, h1, in, out, nullptr, B.N, nullptr, B.sh, B.stream));
    HopSpec h2;
    h2.parity = 0;
    h2.self = in;
    h2.cs = a;
    h2.ch = clov ? -0.25 : -1.0 / (4.0 * a);
    h2.clover = clov;
    h2.live = B.live;
    return launch_hop(B.g, prec, 0, epi, h2, out, out, aux, B.N, B.part, B.sh, B.stream);
}

// x_o = (1/a) b_o + (1/(2a)) H_oe x_e in place on the odd sites of x
// (with a clover term x_o = A_oo^-1 (b_o + (1/2) H_oe x_e)).
int schur_odd(Bicg &B, int prec, const void *b, void *x) {
    const double a = 4.0 + B.m0;
    const bool clov = B.g->C64 != nullptr;
    HopSpec h;
    h.parity = 1;
    h.self = b;
    h.cs = clov ? 1.0 : 1.0 / a;
    h.ch = clov ? 0.5 : 1.0 / (2.0 * a);
    h.clover_inv = clov;
    return launch_hop(B.g, prec, 0, EPI_NONE, h, x, x, nullptr, B.N, nullptr, B.sh, B.stream);
}

// Runs BiCGStab iterations in storage S until every RHS is inactive or
// `max_iter` is reached.  x, r, rhat, p, v, s, t are S-format vectors; the
// state must have been initialised (rho, active, tolerances).
//
// Convergence is checked after every iteration without stalling the device:
// each iteration ends with a one-block kernel that writes "some RHS is still
// iterating" to a device flag and to a host-mapped slot.  The host queues
// iteration k, then waits for the end of iteration k - 1 and reads its slot;
// if nothing was left to do, iteration k's kernels find the device flag clear
// and return at once, and the loop ends.  `iters_done` counts the iterations
// that ran.
template <class S>
int bicgstab_iterate(Bicg &B, int prec, void *x, void *r, void *rhat, void *p, void *v, void *s,
                     void *t, int max_iter, int *iters_done) {
    const int V = B.V, N = B.N;
    const Shape &sh = B.sh;
    int it = 0;
    // p = r
    WDT_HIP(hipMemcpyAsync(p, r, spinor_bytes(V, N, prec), hipMemcpyDeviceToDevice, B.stream));
    const double vb = (double)B.geo.nsites * N * site_bytes(prec);  // one vector pass
    static const char *nm_s[4] = {"axpy_s_fp64", "axpy_s_fp32", "axpy_s_fp16", "axpy_s_bf16"};
    static const char *nm_xr[4] = {"update_xr_fp64", "update_xr_fp32", "update_xr_fp16",
                                   "update_xr_bf16"};
    static const char *nm_p[4] = {"update_p_fp64", "update_p_fp32", "update_p_fp16",
                                  "update_p_bf16"};
    static const char *nm_xrp[4] = {"update_xrp_fp64", "update_xrp_fp32", "update_xrp_fp16",
                                    "update_xrp_bf16"};
    // the inner solves of the mixed solver take the fused end of iteration
    constexpr bool fused = !std::is_same<S, F64>::value;
    // FP64 vectors beyond the last-level cache (256 MB of Infinity Cache)
    // stream past it; smaller ones stay cached for the next pass
    const bool stream_vecs = !fused && (double)(B.geo.nsites) * N * 12 * 16 > 256.0 * (1 << 20);
    EventGuard ev[2];
    for (auto &e : ev) WDT_HIP(hipEventCreateWithFlags(&e.e, hipEventDisableTiming));
    hipLaunchKernelGGL(k_live, dim3(1), dim3(256), 0, B.stream, B.st, N, B.live, (int *)nullptr);
    volatile int *slot = B.live_host;
    while (it < max_iter) {
        const size_t mark = prof_mark();
        WDT_TRY(apply_op(B, prec, EPI_DOT_AUX, p, v, rhat));
        hipLaunchKernelGGL(k_scalar_alpha, dim3(N), dim3(256), 0, B.stream, B.st, B.part, sh.G, N);
        {
            ProfScope pr(nm_s[prec], 3 * vb, B.stream);
            if (stream_vecs)
                hipLaunchKernelGGL((k_update_s<S, true>), B.grid, dim3(sh.threads), 0, B.stream,
                                   B.geo, N, B.NT, sh.SB, B.st, sp<S>(r, V, N), sp<S>(v, V, N),
                                   sp<S>(s, V, N), (const int *)B.live);
            else
                hipLaunchKernelGGL((k_update_s<S>), B.grid, dim3(sh.threads), 0, B.stream, B.geo,
                                   N, B.NT, sh.SB, B.st, sp<S>(r, V, N), sp<S>(v, V, N),
                                   sp<S>(s, V, N), (const int *)B.live);
        }
        if constexpr (fused) {
            WDT_TRY(apply_op(B, prec, EPI_DOT_TSR, s, t, rhat));
            hipLaunchKernelGGL(k_scalar_omega_beta, dim3(N), dim3(256), 0, B.stream, B.st, B.part,
                               sh.G, N);
            {
                ProfScope pr(nm_xrp[prec], 8 * vb, B.stream);
                hipLaunchKernelGGL((k_update_xrp<S>), B.grid, dim3(sh.threads), 0, B.stream, B.geo,
                                   N, B.NT, sh.SB, B.st, sp<S>(x, V, N), sp<S>(p, V, N),
                                   sp<S>(s, V, N), sp<S>(t, V, N), sp<S>(r, V, N),
                                   sp<S>(v, V, N), B.part, (const int *)B.live);
            }
            hipLaunchKernelGGL(k_scalar_check, dim3(N), dim3(256), 0, B.stream, B.st, B.part, sh.Gv,
                               N);
        } else {
            WDT_TRY(apply_op(B, prec, EPI_DOT_TS, s, t, nullptr));
            hipLaunchKernelGGL(k_scalar_omega, dim3(N), dim3(256), 0, B.stream, B.st, B.part, sh.G,
                               N);
            {
                ProfScope pr(nm_xr[prec], 7 * vb, B.stream);
                if (stream_vecs)
                    hipLaunchKernelGGL((k_update_xr<S, true>), B.grid, dim3(sh.threads), 0,
                                       B.stream, B.geo, N, B.NT, sh.SB, B.st, sp<S>(x, V, N),
                                       sp<S>(p, V, N), sp<S>(s, V, N), sp<S>(t, V, N),
                                       sp<S>(r, V, N), sp<S>(rhat, V, N), B.part,
                                       (const int *)B.live);
                else
                    hipLaunchKernelGGL((k_update_xr<S>), B.grid, dim3(sh.threads), 0, B.stream,
                                       B.geo, N, B.NT, sh.SB, B.st, sp<S>(x, V, N), sp<S>(p, V, N),
                                       sp<S>(s, V, N), sp<S>(t, V, N), sp<S>(r, V, N),
                                       sp<S>(rhat, V, N), B.part, (const int *)B.live);
            }
            hipLaunchKernelGGL(k_scalar_beta, dim3(N), dim3(256), 0, B.stream, B.st, B.part, sh.Gv,
                               N);
            {
                ProfScope pr(nm_p[prec], 4 * vb, B.stream);
                if (stream_vecs)
                    hipLaunchKernelGGL((k_update_p<S, true>), B.grid, dim3(sh.threads), 0,
                                       B.stream, B.geo, N, B.NT, sh.SB, B.st, sp<S>(r, V, N),
                                       sp<S>(p, V, N), sp<S>(v, V, N), (const int *)B.live);
                else
                    hipLaunchKernelGGL((k_update_p<S>), B.grid, dim3(sh.threads), 0, B.stream,
                                       B.geo, N, B.NT, sh.SB, B.st, sp<S>(r, V, N),
                                       sp<S>(p, V, N), sp<S>(v, V, N), (const int *)B.live);
            }
        }
        hipLaunchKernelGGL(k_live, dim3(1), dim3(256), 0, B.stream, B.st, N, B.live,
                           B.live_dev_slots + (it & 1));
        WDT_HIP(hipGetLastError());
        WDT_HIP(hipEventRecord(ev[it & 1].e, B.stream));
        ++it;
        if (it >= 2) {
            // iteration it - 2 (slot it & 1) has ended: was the one just queued needed?
            WDT_HIP(hipEventSynchronize(ev[it & 1].e));
            if (slot[it & 1] == 0) {
                prof_discard(mark);
                --it;
                break;
            }
        }
    }
    *iters_done = it;
    return WDT_OK;
}

}  // namespace

// FP64 solve with reliable restarts on the true residual.
static int solve_fp64(wdt_gauge_s *g, double m0, const void *b, void *x, int N,
                      const wdt_solve_params &P, wdt_rhs_stats *stats, hipStream_t stream) {
    const int V = (int)g->lat.V;
    const Shape sh = site_shape(g->lat, N, WDT_FP64);
    const Geom geo = shaped_geom(g->lat, sh);
    const int NT = sh.NT;
    const size_t vb = spinor_bytes(V, N, WDT_FP64);
    const size_t part_bytes = (size_t)3 * std::max(sh.G, sh.Gv) * N * sizeof(double2);
    const size_t st_bytes = ((sizeof(RhsState) * N + 255) / 256) * 256;
    const size_t part_off = 6 * vb;
    const size_t st_off = part_off + ((part_bytes + 255) / 256) * 256;
    const size_t bb_off = st_off + st_bytes;
    const size_t live_off = bb_off + ((sizeof(double) * N + 255) / 256) * 256;
    WDT_TRY(ensure_ws(g, live_off + 256));
    char *base = (char *)g->ws.ptr;
    void *r = base, *rhat = base + vb, *p = base + 2 * vb, *v = base + 3 * vb, *s = base + 4 * vb,
         *t = base + 5 * vb;
    double *bbv = (double *)(base + bb_off);
    Bicg B{g, m0, N, V, sh, geo, NT, dim3(sh.Gv, sh.tiles), stream,
           (RhsState *)(base + st_off), (double2 *)(base + part_off)};
    B.eo = use_even_odd(g);
    if (B.eo) B.geo = parity_geom(g->lat, 0);
    if (B.eo && g->C64) WDT_TRY(ensure_clover_inverse(g, 4.0 + m0, stream));
    WDT_TRY(bind_live(B, (int *)(base + live_off)));
    WDT_HIP(hipMemsetAsync(B.st, 0, sizeof(RhsState) * N, stream));
    if (!P.x0_is_guess) WDT_HIP(hipMemsetAsync(x, 0, vb, stream));
    std::vector<RhsState> hs(N);
    std::vector<int> total_it(N, 0), restarts(N, 0);
    int budget = P.max_iter;
    int rc = WDT_OK;
    if (B.eo) {
        // Even-odd: x_o is kept equal to (b_o + H_oe x_e / 2) / a, so the odd
        // rows of the residual vanish, b - D x is the even-site residual of
        // one one-parity launch, and it is also the Schur system's residual.
        // ||b||^2 over the whole lattice, once:
        hipLaunchKernelGGL((k_norm<F64>), B.grid, dim3(sh.threads), 0, stream, geo, N, NT, sh.SB,
                           sp<F64>(const_cast<void *>(b), V, N), B.part);
        hipLaunchKernelGGL(k_sum_to, dim3(N), dim3(256), 0, stream, bbv, B.part, sh.Gv, N);
        WDT_TRY(schur_odd(B, WDT_FP64, b, x));
    }
    for (int round = 0;; ++round) {
        // r = b - D x (true residual), rhat = r
        if (B.eo) {
            HopSpec h;
            h.parity = 0;
            h.self = x;
            h.cs = 4.0 + m0;
            h.ch = -0.5;
            h.clover = g->C64 != nullptr;
            WDT_TRY(launch_hop(g, WDT_FP64, 0, EPI_RESID, h, x, r, b, N, B.part, sh, stream));
        } else {
            WDT_TRY(launch_dslash(g, m0, WDT_FP64, 0, EPI_RESID, x, r, b, N, B.part, sh, stream));
        }
        hipLaunchKernelGGL(k_init_state, dim3(N), dim3(256), 0, stream, B.st, B.part, sh.G, N,
                           P.tol, (const int *)nullptr, (const double *)nullptr,
                           (const double *)(B.eo ? bbv : nullptr));
        WDT_HIP(hipMemcpyAsync(rhat, r, vb, hipMemcpyDeviceToDevice, stream));
        WDT_HIP(hipMemcpyAsync(hs.data(), B.st, sizeof(RhsState) * N, hipMemcpyDeviceToHost, stream));
        WDT_HIP(hipStreamSynchronize(stream));
        bool any = false;
        for (int k = 0; k < N; ++k) any = any || hs[k].active;
        if (!any || budget <= 0 || round > 50) {
            for (int k = 0; k < N; ++k) {
                if (stats) {
                    stats[k].iterations = total_it[k];
                    stats[k].outer = 0;
                    stats[k].converged = (!hs[k].active && hs[k].flag == 1) ? 1 : 0;
                    stats[k].restarts = restarts[k];
                    stats[k].true_residual = hs[k].bb > 0 ? std::sqrt(hs[k].rr / hs[k].bb) : 0.0;
                }
                if (hs[k].active || hs[k].flag != 1) rc = WDT_WNOTCONVERGED;
            }
            return rc;
        }
        for (int k = 0; k < N; ++k)
            if (hs[k].active && round > 0) restarts[k] += 1;
        // iteration counters restart from 0 in the state; accumulate host side
        std::vector<int> before(N);
        for (int k = 0; k < N; ++k) before[k] = hs[k].iters;
        int done = 0;
        WDT_TRY(bicgstab_iterate<F64>(B, WDT_FP64, x, r, rhat, p, v, s, t, budget, &done));
        if (B.eo) WDT_TRY(schur_odd(B, WDT_FP64, b, x));
        WDT_HIP(hipMemcpyAsync(hs.data(), B.st, sizeof(RhsState) * N, hipMemcpyDeviceToHost, stream));
        WDT_HIP(hipStreamSynchronize(stream));
        for (int k = 0; k < N; ++k) total_it[k] += hs[k].iters - before[k];
        budget -= done;
    }
}

// FP64 defect correction around an inner solve in storage S (F32 or F16).
// Iterations one inner solve of the defect correction may take.
constexpr int kInnerCap = 500;

template <class S>
static int solve_mixed(wdt_gauge_s *g, double m0, const void *b, void *x, int N, int prec,
                       const wdt_solve_params &P, wdt_rhs_stats *stats, hipStream_t stream) {
    const int V = (int)g->lat.V;
    const Shape sh = site_shape(g->lat, N, prec);
    const Geom geo = shaped_geom(g->lat, sh);
    const int NT = sh.NT;
    const size_t vb64 = spinor_bytes(V, N, WDT_FP64);
    const size_t vbl = ((spinor_bytes(V, N, prec) + 255) / 256) * 256;
    const size_t part_bytes = (size_t)3 * std::max(sh.G, sh.Gv) * N * sizeof(double2);
    const size_t st_bytes = ((sizeof(RhsState) * N + 255) / 256) * 256;
    const size_t nrow = ((N + 31) / 32) * 32;  // per-RHS array stride (doubles)
    const size_t low_off = vb64;
    const size_t part_off = low_off + 7 * vbl;
    const size_t st_off = part_off + ((part_bytes + 255) / 256) * 256;
    const size_t mask_off = st_off + st_bytes;
    const size_t fac_off = mask_off + ((sizeof(int) * N + 255) / 256) * 256;
    const size_t live_off = fac_off + ((4 * nrow * sizeof(double) + 255) / 256) * 256;
    WDT_TRY(ensure_ws(g, live_off + 256));
    char *base = (char *)g->ws.ptr;
    void *r64 = base;
    void *lo[7];
    for (int i = 0; i < 7; ++i) lo[i] = base + low_off + i * vbl;
    void *rS = lo[0], *rhat = lo[1], *p = lo[2], *v = lo[3], *s = lo[4], *t = lo[5], *e = lo[6];
    int *mask = (int *)(base + mask_off);
    // per RHS: 1/||r|| into the inner solve, ||r|| back out, the inner
    // tolerance, ||b||^2 (even-odd)
    double *fin = (double *)(base + fac_off);
    double *fout = fin + nrow, *tolr = fin + 2 * nrow, *bbv = fin + 3 * nrow;
    std::vector<double> hfac(3 * nrow, 0.0);
    Bicg B{g, m0, N, V, sh, geo, NT, dim3(sh.Gv, sh.tiles), stream,
           (RhsState *)(base + st_off), (double2 *)(base + part_off)};
    B.eo = use_even_odd(g);
    if (B.eo) B.geo = parity_geom(g->lat, 0);
    if (B.eo && g->C64) WDT_TRY(ensure_clover_inverse(g, 4.0 + m0, stream));
    WDT_TRY(bind_live(B, (int *)(base + live_off)));
    const dim3 grid(sh.Gv, sh.tiles);
    // the sites the defect correction updates: all, or the even ones
    const Geom &ug = B.geo;
    const double a = 4.0 + m0;
    if (!P.x0_is_guess) WDT_HIP(hipMemsetAsync(x, 0, vb64, stream));
    std::vector<RhsState> hs(N);
    std::vector<int> hmask(N);
    std::vector<int> total_it(N, 0), outer(N, 0);
    const double inner_tol = P.inner_tol > 0 ? P.inner_tol : 3e-3;
    const int max_outer = P.max_outer > 0 ? P.max_outer : 30;
    int budget = P.max_iter;
    int rc = WDT_OK;
    WDT_HIP(hipMemsetAsync(B.st, 0, sizeof(RhsState) * N, stream));
    if (B.eo) {
        // Even-odd: x_o is kept equal to (b_o + H_oe x_e / 2) / a in FP64, so
        // the odd rows of the residual vanish and b - D x is the even-site
        // residual r_e = b_e - a x_e + H_eo x_o / 2 of one one-parity
        // launch; the inner solves take the Schur system M e_e = r_e, and
        // only x_e is corrected.  ||b||^2 over the whole lattice, once:
        hipLaunchKernelGGL((k_norm<F64>), grid, dim3(sh.threads), 0, stream, geo, N, NT, sh.SB,
                           sp<F64>(const_cast<void *>(b), V, N), B.part);
        hipLaunchKernelGGL(k_sum_to, dim3(N), dim3(256), 0, stream, bbv, B.part, sh.Gv, N);
        WDT_TRY(schur_odd(B, WDT_FP64, b, x));
    }
    for (int o = 0;; ++o) {
        // FP64 true residual r64 = b - D x
        if (B.eo) {
            HopSpec h;
            h.parity = 0;
            h.self = x;
            h.cs = a;
            h.ch = -0.5;
            h.clover = g->C64 != nullptr;
            WDT_TRY(launch_hop(g, WDT_FP64, 0, EPI_RESID, h, x, r64, b, N, B.part, sh, stream));
        } else {
            WDT_TRY(launch_dslash(g, m0, WDT_FP64, 0, EPI_RESID, x, r64, b, N, B.part, sh, stream));
        }
        hipLaunchKernelGGL(k_init_state, dim3(N), dim3(256), 0, stream, B.st, B.part, sh.G, N,
                           P.tol, (const int *)nullptr, (const double *)nullptr,
                           (const double *)(B.eo ? bbv : nullptr));
        WDT_HIP(hipMemcpyAsync(hs.data(), B.st, sizeof(RhsState) * N, hipMemcpyDeviceToHost, stream));
        WDT_HIP(hipStreamSynchronize(stream));
        bool any = false;
        for (int k = 0; k < N; ++k) {
            hmask[k] = hs[k].active;
            any = any || hs[k].active;
        }
        if (!any || o >= max_outer || budget <= 0) {
            for (int k = 0; k < N; ++k) {
                if (stats) {
                    stats[k].iterations = total_it[k];
                    stats[k].outer = outer[k];
                    stats[k].converged = (!hs[k].active && hs[k].flag == 1) ? 1 : 0;
                    stats[k].restarts = 0;
                    stats[k].true_residual = hs[k].bb > 0 ? std::sqrt(hs[k].rr / hs[k].bb) : 0.0;
                }
                if (hs[k].active || hs[k].flag != 1) rc = WDT_WNOTCONVERGED;
            }
            return rc;
        }
        for (int k = 0; k < N; ++k) outer[k] += hmask[k];
        WDT_HIP(hipMemcpyAsync(mask, hmask.data(), sizeof(int) * N, hipMemcpyHostToDevice, stream));
        // The inner system is D e = r / ||r|| (unit norm whatever the scale of
        // b, so the low-precision data stays far from under- and overflow as
        // the residual falls); x += ||r|| e afterwards.  Its tolerance is
        // inner_tol, or what is left to reach tol if that is less demanding
        // (the last correction of a RHS stops as soon as it suffices).
        for (int k = 0; k < N; ++k) {
            const double nr = std::sqrt(hs[k].rr);
            const bool ok = hmask[k] && nr > 0 && std::isfinite(nr);
            hfac[k] = ok ? 1.0 / nr : 0.0;
            hfac[nrow + k] = ok ? nr : 0.0;
            const double left = ok ? 0.5 * P.tol * std::sqrt(hs[k].bb) / nr : 0.0;
            hfac[2 * nrow + k] = std::min(0.5, std::max(inner_tol, left));
        }
        WDT_HIP(hipMemcpyAsync(fin, hfac.data(), sizeof(double) * hfac.size(), hipMemcpyHostToDevice,
                               stream));
        WDT_HIP(hipMemsetAsync(e, 0, vbl, stream));
        if (B.eo) {
            // rS_e = rhat_e = r_e / ||r|| and its norm for the inner state (the
            // inner iteration reads the even sites only)
            hipLaunchKernelGGL((k_convert<F64, S, false>), grid, dim3(sh.threads), 0, stream, ug,
                               N, NT, sh.SB, sp<F64>(r64, V, N), sp<S>(rS, V, N),
                               sp<S>(rhat, V, N), (const double *)fin, B.part);
            hipLaunchKernelGGL(k_init_state, dim3(N), dim3(256), 0, stream, B.st, B.part, sh.Gv,
                               N, inner_tol, (const int *)mask, (const double *)tolr,
                               (const double *)nullptr);
        } else {
            // inner system D e = r (low precision), e = 0, rhat = r
            hipLaunchKernelGGL((k_convert<F64, S, false>), grid, dim3(sh.threads), 0, stream, geo,
                               N, NT, sh.SB, sp<F64>(r64, V, N), sp<S>(rS, V, N), SpinorPtr<S>{},
                               (const double *)fin, (double2 *)nullptr);
            // ||r||^2 in the stored precision: residual of e = 0 against rS
            WDT_TRY(launch_dslash(g, m0, prec, 0, EPI_RESID, e, rhat, rS, N, B.part, sh, stream));
            hipLaunchKernelGGL(k_init_state, dim3(N), dim3(256), 0, stream, B.st, B.part, sh.G, N,
                               inner_tol, (const int *)mask, (const double *)tolr,
                               (const double *)nullptr);
            WDT_HIP(hipMemcpyAsync(rS, rhat, spinor_bytes(V, N, prec), hipMemcpyDeviceToDevice,
                                   stream));
        }
        std::vector<int> before(N);
        WDT_HIP(hipMemcpyAsync(hs.data(), B.st, sizeof(RhsState) * N, hipMemcpyDeviceToHost, stream));
        WDT_HIP(hipStreamSynchronize(stream));
        for (int k = 0; k < N; ++k) before[k] = hs[k].iters;
        int done = 0;
        // an inner solve that stops converging in low precision would spend the
        // whole budget; each one gets at most kInnerCap iterations
        WDT_TRY(bicgstab_iterate<S>(B, prec, e, rS, rhat, p, v, s, t, std::min(budget, kInnerCap),
                                    &done));
        WDT_HIP(hipMemcpyAsync(hs.data(), B.st, sizeof(RhsState) * N, hipMemcpyDeviceToHost, stream));
        WDT_HIP(hipStreamSynchronize(stream));
        for (int k = 0; k < N; ++k) total_it[k] += hs[k].iters - before[k];
        budget -= done;
        // x += ||r|| e (even-odd: x_e, then x_o from b_o and x_e)
        hipLaunchKernelGGL((k_convert<S, F64, true>), grid, dim3(sh.threads), 0, stream, ug, N, NT,
                           sh.SB, sp<S>(e, V, N), sp<F64>(x, V, N), SpinorPtr<F64>{},
                           (const double *)fout, (double2 *)nullptr);
        WDT_HIP(hipGetLastError());
        if (B.eo) WDT_TRY(schur_odd(B, WDT_FP64, b, x));
    }
    (void)rc;
}

}  // namespace wdt

extern "C" int wdt_solve(wdt_gauge g, double m0, const void *dev_b, void *dev_x, int32_t n_rhs,
                         const wdt_solve_params *params, wdt_rhs_stats *stats, void *stream) {
    using namespace wdt;
    WDT_CHECK(g != nullptr, "wdt_solve: null gauge handle");
    WDT_CHECK(dev_b != nullptr && dev_x != nullptr, "wdt_solve: null vector");
    WDT_CHECK(dev_b != dev_x, "wdt_solve: b and x must not overlap");
    WDT_CHECK(params != nullptr, "wdt_solve: null params");
    WDT_CHECK(n_rhs >= 1, "wdt_solve: n_rhs must be >= 1");
    WDT_CHECK(params->tol > 0 && params->tol < 1, "wdt_solve: tol must be in (0, 1)");
    WDT_CHECK(params->max_iter >= 1, "wdt_solve: max_iter must be >= 1");
    const hipStream_t st = (hipStream_t)stream;
    switch (params->prec) {
        case WDT_FP64:
            return solve_fp64(g, m0, dev_b, dev_x, n_rhs, *params, stats, st);
        case WDT_FP32:
            return solve_mixed<F32>(g, m0, dev_b, dev_x, n_rhs, WDT_FP32, *params, stats, st);
        case WDT_FP16:
            return solve_mixed<F16>(g, m0, dev_b, dev_x, n_rhs, WDT_FP16, *params, stats, st);
        case WDT_BF16:
            return solve_mixed<B16>(g, m0, dev_b, dev_x, n_rhs, WDT_BF16, *params, stats, st);
        default:
            return set_error(WDT_EINVAL, "wdt_solve: bad precision %d", params->prec);
    }
}
