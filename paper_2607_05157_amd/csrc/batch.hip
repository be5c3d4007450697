// Many small, uneven systems D_i x = b_i (different lattices, links, masses
// and RHS counts) solved together: every phase of the batched BiCGStab is ONE
// launch that covers all systems (each block looks up its system in a table),
// and one iteration of the recurrence is captured as a hipGraph and replayed,
// so a batch of tiny lattices costs a handful of launches per iteration
// instead of a handful per system.  FP64.
//
// Blocks are dealt to systems in proportion to their work (V * N); each
// system's range starts at a multiple of 8 blocks, so the XCD-aware
// renumbering of the single-system kernels carries over unchanged.  Systems
// converge at different iterations: at every convergence check the block
// budget is dealt again over the systems that still have active RHS (finished
// ones get none), which only rewrites the device-side system table between
// graph replays.
//
// Systems whose lattice has every extent even (and no clover term) are
// solved even-odd preconditioned, like the single-system solver: the iteration runs on the
// even sites with M = a - H_eo H_oe / (4a) (a = 4 + m0), the restart turns the
// true residual into the Schur right-hand side, and the odd sites of x are
// rebuilt from b and the even sites at the end of every round.
#include "kernels.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

namespace wdt {

enum VecId { V_X = 0, V_B, V_R, V_RHAT, V_P, V_V, V_S, V_T, V_COUNT };

struct SysDesc {
    Geom g;
    const double2 *U;
    const double *C;  // clover term or null (then eo = 0)
    double diag;
    int eo;  // 1: even-odd preconditioned (every extent even)
    int N, NT, SB, tiles, G;
    int block_begin, nblocks;
    int rhs_begin;
    double2 *part;
    double2 *vec[V_COUNT];
};

__device__ __forceinline__ int find_sys(const SysDesc *sys, int nsys, int block) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sys[mid].block_begin <= block) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_rhs(const SysDesc *sys, int nsys, int rhs) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sys[mid].rhs_begin <= rhs) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

#define WDT_SYS_CTX                                                         \
    const int si = find_sys(sys, nsys, blockIdx.x);                         \
    const SysDesc &d = sys[si];                                             \
    const int lbg = blockIdx.x - d.block_begin;                             \
    if (lbg >= d.nblocks) return;                                           \
    const int tile = lbg / d.G, lb = xcd_block(lbg - tile * d.G, d.G);     \
    auto sp = [&](int id) { return make_spinor<F64>(d.vec[id], d.g.V, d.N); };

// The sites of one parity (parity >= 0) or all sites.
__device__ __forceinline__ Geom sys_geom(const SysDesc &d, int parity) {
    Geom g = d.g;
    if (parity >= 0) {
        g.parity = parity;
        g.nsites = g.V / 2;
    }
    return g;
}

// The sites the iteration's vector updates touch: the even ones under even-odd.
__device__ __forceinline__ Geom iter_geom(const SysDesc &d) { return sys_geom(d, d.eo ? 0 : -1); }

// Full operator: out = D in (with the epilogue EPI), every system.
template <int EPI>
__global__ __launch_bounds__(256) void kb_dslash(const SysDesc *sys, int nsys, int in, int out,
                                                 int aux) {
    WDT_SYS_CTX
    if (d.C)
        dslash_body<F64, 0, false, EPI, false, 1>(d.g, d.U, d.C, sp(in), d.diag, -0.5, sp(in),
                                                     sp(out), sp(aux >= 0 ? aux : in), d.N, d.NT,
                                                     d.SB, d.part, tile, tile + 1, lb, d.G);
    else
        dslash_body<F64, 0, false, EPI>(d.g, d.U, nullptr, sp(in), d.diag, -0.5, sp(in), sp(out),
                                        sp(aux >= 0 ? aux : in),
                                        d.N, d.NT, d.SB, d.part, tile, tile + 1, lb, d.G);
}

// The iteration's operator, first half: even-odd systems put H_oe in on the
// odd sites of out; the others do nothing here.
__global__ __launch_bounds__(256) void kb_op_odd(const SysDesc *sys, int nsys, int in, int out) {
    WDT_SYS_CTX
    if (!d.eo) return;
    dslash_body<F64, 0, false, EPI_NONE>(sys_geom(d, 1), d.U, nullptr, sp(in), 0.0, 1.0, sp(in), sp(out),
                                         sp(in), d.N, d.NT, d.SB, nullptr, tile, tile + 1, lb,
                                         d.G);
}

// Second half: even-odd systems out_e = a in_e - H_eo out_o / (4a) (the Schur
// operator); the others out = D in.
template <int EPI>
__global__ __launch_bounds__(256) void kb_op_even(const SysDesc *sys, int nsys, int in, int out,
                                                  int aux) {
    WDT_SYS_CTX
    const SpinorPtr<F64> pa = sp(aux >= 0 ? aux : in);
    if (d.eo)
        dslash_body<F64, 0, false, EPI>(sys_geom(d, 0), d.U, nullptr, sp(in), d.diag,
                                        -0.25 / d.diag, sp(out), sp(out), pa, d.N, d.NT, d.SB,
                                        d.part, tile, tile + 1, lb, d.G);
    else if (d.C)
        dslash_body<F64, 0, false, EPI, false, 1>(d.g, d.U, d.C, sp(in), d.diag, -0.5, sp(in),
                                                     sp(out), pa, d.N, d.NT, d.SB, d.part, tile,
                                                     tile + 1, lb, d.G);
    else
        dslash_body<F64, 0, false, EPI>(d.g, d.U, nullptr, sp(in), d.diag, -0.5, sp(in), sp(out),
                                        pa, d.N, d.NT, d.SB, d.part, tile, tile + 1, lb, d.G);
}

// Even-odd systems: r_e += H_eo r_o / (2a) in place (the Schur right-hand
// side of the correction equation), partials d0 = d1 = ||r_e||^2.
__global__ __launch_bounds__(256) void kb_schur_rhs(const SysDesc *sys, int nsys) {
    WDT_SYS_CTX
    if (!d.eo) return;
    dslash_body<F64, 0, false, EPI_NORM>(sys_geom(d, 0), d.U, nullptr, sp(V_R), 1.0, 0.5 / d.diag,
                                         sp(V_R), sp(V_R), sp(V_R), d.N, d.NT, d.SB, d.part,
                                         tile, tile + 1, lb, d.G);
}

// Even-odd systems: x_o = b_o / a + H_oe x_e / (2a) in place.
__global__ __launch_bounds__(256) void kb_schur_odd(const SysDesc *sys, int nsys) {
    WDT_SYS_CTX
    if (!d.eo) return;
    dslash_body<F64, 0, false, EPI_NONE>(sys_geom(d, 1), d.U, nullptr, sp(V_B), 1.0 / d.diag,
                                         0.5 / d.diag, sp(V_X), sp(V_X), sp(V_X), d.N, d.NT,
                                         d.SB, nullptr, tile, tile + 1, lb, d.G);
}

__global__ __launch_bounds__(256) void kb_update_s(const SysDesc *sys, int nsys,
                                                   const RhsState *st) {
    WDT_SYS_CTX
    update_s_body<F64>(iter_geom(d), d.N, d.NT, d.SB, st + d.rhs_begin, sp(V_R), sp(V_V), sp(V_S),
                       tile, lb, d.G);
}

__global__ __launch_bounds__(256) void kb_update_xr(const SysDesc *sys, int nsys,
                                                    const RhsState *st) {
    WDT_SYS_CTX
    update_xr_body<F64>(iter_geom(d), d.N, d.NT, d.SB, st + d.rhs_begin, sp(V_X), sp(V_P),
                        sp(V_S), sp(V_T), sp(V_R), sp(V_RHAT), d.part, tile, lb, d.G);
}

__global__ __launch_bounds__(256) void kb_update_p(const SysDesc *sys, int nsys,
                                                   const RhsState *st) {
    WDT_SYS_CTX
    update_p_body<F64>(iter_geom(d), d.N, d.NT, d.SB, st + d.rhs_begin, sp(V_R), sp(V_P), sp(V_V),
                       tile, lb, d.G);
}

// dst = src (or dst = 0 when src < 0)
__global__ __launch_bounds__(256) void kb_copy(const SysDesc *sys, int nsys, int src, int dst) {
    WDT_SYS_CTX
    const Geom &g = d.g;
    const int N = d.N, NT = d.NT, SB = d.SB;
    SpinorPtr<F64> ps = sp(src >= 0 ? src : dst), pd = sp(dst);
    SITE_LOOP_BEGIN_AT(tile, lb, d.G)
    cplx<double> a[12];
    if (src >= 0) {
        load_site<F64>(ps, s, r, a);
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) a[k] = {0.0, 0.0};
    }
    store_site<F64>(pd, s, r, a);
    SITE_LOOP_END
}

#define WDT_RHS_CTX                                         \
    const int si = find_rhs(sys, nsys, blockIdx.x);         \
    const SysDesc &d = sys[si];                             \
    const int r = blockIdx.x - d.rhs_begin;                 \
    RhsState *s0 = st + d.rhs_begin;

__global__ void kb_init(const SysDesc *sys, int nsys, RhsState *st, double tol) {
    WDT_RHS_CTX
    init_state_body(s0, d.part, d.G, d.N, tol, nullptr, nullptr, nullptr, r);
}
__global__ void kb_alpha(const SysDesc *sys, int nsys, RhsState *st) {
    WDT_RHS_CTX
    scalar_alpha_body(s0, d.part, d.G, d.N, r);
}
__global__ void kb_omega(const SysDesc *sys, int nsys, RhsState *st) {
    WDT_RHS_CTX
    scalar_omega_body(s0, d.part, d.G, d.N, r);
}
__global__ void kb_beta(const SysDesc *sys, int nsys, RhsState *st) {
    WDT_RHS_CTX
    scalar_beta_body(s0, d.part, d.G, d.N, r);
}
// even-odd systems: rho = ||r_e||^2 of the Schur right-hand side
__global__ void kb_rho(const SysDesc *sys, int nsys, RhsState *st) {
    WDT_RHS_CTX
    if (d.eo) scalar_rho_body(s0, d.part, d.G, d.N, r);
}

}  // namespace wdt

using namespace wdt;

struct wdt_batch_s {
    int nsys = 0;
    std::vector<const wdt_gauge_s *> gauges;
    std::vector<double> m0;
    std::vector<int> nrhs;
    std::vector<SysDesc> host;
    SysDesc *dev = nullptr;
    RhsState *st = nullptr;
    int total_rhs = 0, total_blocks = 0;
    int grid_blocks = 0;    // grid of the captured iteration (>= total_blocks)
    int cus = 256;
    std::vector<int> gcap;  // per system: most blocks per tile (partials capacity)
    int blocks_per_cu = 4;  // block budget of the plan (tuned)
    int tile_cap = 16;      // largest RHS tile (tuned)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

namespace {

// Orders the batch's stream after the caller's stream on entry and the
// caller's stream after the batch's on every path out, errors included, so
// the caller never runs ahead of kernels the batch still has in flight.
struct StreamJoin {
    hipStream_t caller, own;
    hipEvent_t ev = nullptr;
    int rc = WDT_OK;
    StreamJoin(hipStream_t c, hipStream_t o) : caller(c), own(o) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(ev, caller) != hipSuccess || hipStreamWaitEvent(own, ev, 0) != hipSuccess) {
            (void)hipGetLastError();
            rc = set_error(WDT_EHIP, "batch: stream ordering failed");
        }
    }
    ~StreamJoin() {
        if (!ev) return;
        if (hipEventRecord(ev, own) == hipSuccess) (void)hipStreamWaitEvent(caller, ev, 0);
        (void)hipEventDestroy(ev);
    }
};

int free_plan(wdt_batch_s *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->grid_blocks = 0;
    if (b->ws) (void)hipFree(b->ws);
    b->ws = nullptr;
    b->ws_bytes = 0;
    return WDT_OK;
}

// Deals the block budget over the systems with active[i] != 0, in proportion
// to V * N, at least 8 blocks per tile, at most gcap; a multiple of 8 each.
void assign_blocks(wdt_batch_s *b, const std::vector<char> &active) {
    double work = 0;
    for (int i = 0; i < b->nsys; ++i)
        if (active[i]) work += (double)b->gauges[i]->lat.V * b->nrhs[i];
    const double budget = (double)b->cus * b->blocks_per_cu;
    int blk = 0;
    for (int i = 0; i < b->nsys; ++i) {
        SysDesc &d = b->host[i];
        d.block_begin = blk;
        if (!active[i] || work <= 0) {
            d.G = 8;
            d.nblocks = 0;
            continue;
        }
        int64_t G = (int64_t)std::llround(budget * (double)b->gauges[i]->lat.V * d.N / work / d.tiles);
        G = std::max<int64_t>(8, std::min<int64_t>(G, b->gcap[i]));
        d.G = (int)((G / 8) * 8);
        d.nblocks = d.tiles * d.G;
        blk += d.nblocks;
    }
    b->total_blocks = blk;
}

// Lays out shapes and workspace for the current tuning values and deals the
// blocks over all systems.
int make_plan(wdt_batch_s *b) {
    WDT_TRY(free_plan(b));
    {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            b->cus = p.multiProcessorCount;
    }
    const double budget = (double)b->cus * b->blocks_per_cu;
    b->host.assign(b->nsys, SysDesc{});
    b->gcap.assign(b->nsys, 8);
    size_t off = 0;
    int rhs = 0;
    std::vector<size_t> vec_off(b->nsys), part_off(b->nsys);
    for (int i = 0; i < b->nsys; ++i) {
        const wdt_gauge_s *g = b->gauges[i];
        SysDesc &d = b->host[i];
        const int N = b->nrhs[i];
        d.N = N;
        int NT = std::min(N, b->tile_cap);
        for (int t = NT; t >= 8; --t)
            if (N % t == 0) {
                NT = t;
                break;
            }
        d.NT = NT;
        d.tiles = (N + NT - 1) / NT;
        int SB = std::max(1, 256 / NT);
        for (int sb = SB; sb >= 1; --sb)
            if ((NT * sb) % 64 == 0) {
                SB = sb;
                break;
            }
        d.SB = SB;
        // most blocks this system can get: the whole budget, or one per group
        const int64_t ngroups = (g->lat.V + SB - 1) / SB;
        int64_t cap = std::min<int64_t>(ngroups, (int64_t)std::ceil(budget / d.tiles));
        b->gcap[i] = (int)std::max<int64_t>(8, (cap / 8) * 8);
        d.rhs_begin = rhs;
        rhs += N;
        d.g = g->lat.geom();
        d.U = g->U64;
        d.C = g->C64;
        d.diag = 4.0 + b->m0[i];
        d.eo = (g->lat.even_odd_ok() && tuning().eo != 0 && !g->C64) ? 1 : 0;
        vec_off[i] = off;
        off += ((size_t)6 * spinor_bytes(g->lat.V, N, WDT_FP64) + 255) / 256 * 256;
        part_off[i] = off;
        off += ((size_t)2 * b->gcap[i] * N * sizeof(double2) + 255) / 256 * 256;
    }
    b->total_rhs = rhs;
    const size_t st_off = off;
    off += ((size_t)rhs * sizeof(RhsState) + 255) / 256 * 256;
    const size_t dev_off = off;
    off += ((size_t)b->nsys * sizeof(SysDesc) + 255) / 256 * 256;
    if (hipMalloc(&b->ws, off) != hipSuccess) {
        (void)hipGetLastError();
        b->ws = nullptr;
        return set_error(WDT_ENOMEM, "batch workspace of %zu bytes", off);
    }
    b->ws_bytes = off;
    char *base = (char *)b->ws;
    for (int i = 0; i < b->nsys; ++i) {
        SysDesc &d = b->host[i];
        const size_t vb = spinor_bytes(b->gauges[i]->lat.V, d.N, WDT_FP64);
        for (int v = V_R; v < V_COUNT; ++v)
            d.vec[v] = (double2 *)(base + vec_off[i] + (size_t)(v - V_R) * vb);
        d.vec[V_X] = d.vec[V_B] = nullptr;
        d.part = (double2 *)(base + part_off[i]);
    }
    b->st = (RhsState *)(base + st_off);
    b->dev = (SysDesc *)(base + dev_off);
    assign_blocks(b, std::vector<char>(b->nsys, 1));
    return WDT_OK;
}

int upload(wdt_batch_s *b) {
    WDT_HIP(hipMemcpyAsync(b->dev, b->host.data(), sizeof(SysDesc) * b->nsys,
                           hipMemcpyHostToDevice, b->stream));
    return WDT_OK;
}

// One BiCGStab iteration for every system (ten launches over grid_blocks
// blocks; blocks past the last system's range return at once).
int enqueue_iteration(wdt_batch_s *b) {
    const dim3 gb(b->grid_blocks), gr(b->total_rhs), t(256);
    hipLaunchKernelGGL(kb_op_odd, gb, t, 0, b->stream, b->dev, b->nsys, (int)V_P, (int)V_V);
    hipLaunchKernelGGL(kb_op_even<EPI_DOT_AUX>, gb, t, 0, b->stream, b->dev, b->nsys, (int)V_P,
                       (int)V_V, (int)V_RHAT);
    hipLaunchKernelGGL(kb_alpha, gr, t, 0, b->stream, b->dev, b->nsys, b->st);
    hipLaunchKernelGGL(kb_update_s, gb, t, 0, b->stream, b->dev, b->nsys, b->st);
    hipLaunchKernelGGL(kb_op_odd, gb, t, 0, b->stream, b->dev, b->nsys, (int)V_S, (int)V_T);
    hipLaunchKernelGGL(kb_op_even<EPI_DOT_TS>, gb, t, 0, b->stream, b->dev, b->nsys, (int)V_S,
                       (int)V_T, -1);
    hipLaunchKernelGGL(kb_omega, gr, t, 0, b->stream, b->dev, b->nsys, b->st);
    hipLaunchKernelGGL(kb_update_xr, gb, t, 0, b->stream, b->dev, b->nsys, b->st);
    hipLaunchKernelGGL(kb_beta, gr, t, 0, b->stream, b->dev, b->nsys, b->st);
    hipLaunchKernelGGL(kb_update_p, gb, t, 0, b->stream, b->dev, b->nsys, b->st);
    WDT_HIP(hipGetLastError());
    return WDT_OK;
}

// (Re)captures the iteration graph when the current plan needs more blocks
// than the captured grid has.
int capture(wdt_batch_s *b) {
    if (b->exec && b->total_blocks <= b->grid_blocks) return WDT_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->grid_blocks = b->total_blocks;
    WDT_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_iteration(b);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc < 0) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return set_error(WDT_EHIP, "graph capture: %s", hipGetErrorString(e));
    b->graph = g;
    WDT_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return WDT_OK;
}

// r = b - D x, states from the true residual; even-odd systems then take the
// Schur right-hand side r_e + H_eo r_o / (2a) for r and its norm for rho;
// rhat = r, p = r.
int restart(wdt_batch_s *b, double tol) {
    const dim3 gb(b->total_blocks), gr(b->total_rhs), t(256);
    hipLaunchKernelGGL(kb_dslash<EPI_RESID>, gb, t, 0, b->stream, b->dev, b->nsys, (int)V_X,
                       (int)V_R, (int)V_B);
    hipLaunchKernelGGL(kb_init, gr, t, 0, b->stream, b->dev, b->nsys, b->st, tol);
    hipLaunchKernelGGL(kb_schur_rhs, gb, t, 0, b->stream, b->dev, b->nsys);
    hipLaunchKernelGGL(kb_rho, gr, t, 0, b->stream, b->dev, b->nsys, b->st);
    hipLaunchKernelGGL(kb_copy, gb, t, 0, b->stream, b->dev, b->nsys, (int)V_R, (int)V_RHAT);
    hipLaunchKernelGGL(kb_copy, gb, t, 0, b->stream, b->dev, b->nsys, (int)V_R, (int)V_P);
    WDT_HIP(hipGetLastError());
    return WDT_OK;
}

}  // namespace

extern "C" {

int wdt_batch_create(const wdt_gauge *gauges, const double *m0, const int32_t *n_rhs,
                     int32_t n_sys, wdt_batch *out) {
    WDT_CHECK(gauges && m0 && n_rhs && out && n_sys >= 1, "wdt_batch_create: bad argument");
    wdt_batch_s *b = new (std::nothrow) wdt_batch_s;
    if (!b) return set_error(WDT_ENOMEM, "wdt_batch_create: host allocation");
    b->nsys = n_sys;
    for (int i = 0; i < n_sys; ++i) {
        if (!gauges[i] || n_rhs[i] < 1) {
            delete b;
            return set_error(WDT_EINVAL, "wdt_batch_create: system %d: null gauge or n_rhs < 1", i);
        }
        b->gauges.push_back(gauges[i]);
        b->m0.push_back(m0[i]);
        b->nrhs.push_back(n_rhs[i]);
    }
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return set_error(WDT_EHIP, "wdt_batch_create: stream creation failed");
    }
    const int rc = make_plan(b);
    if (rc < 0) {
        (void)hipStreamDestroy(b->stream);
        delete b;
        return rc;
    }
    *out = b;
    return WDT_OK;
}

int wdt_batch_destroy(wdt_batch b) {
    if (!b) return WDT_OK;
    (void)hipStreamSynchronize(b->stream);
    free_plan(b);
    (void)hipStreamDestroy(b->stream);
    delete b;
    return WDT_OK;
}

int wdt_batch_tune(wdt_batch b, int32_t iters, double *best_ms) {
    WDT_CHECK(b && iters >= 1, "wdt_batch_tune: bad argument");
    const int bpcs[] = {2, 4, 8};
    const int tiles[] = {8, 16, 48};
    double best = 1e300;
    int bb = b->blocks_per_cu, bt = b->tile_cap;
    EventGuard g0, g1;
    WDT_HIP(hipEventCreate(&g0.e));
    WDT_HIP(hipEventCreate(&g1.e));
    hipEvent_t e0 = g0.e, e1 = g1.e;
    for (int bpc : bpcs)
        for (int tc : tiles) {
            b->blocks_per_cu = bpc;
            b->tile_cap = tc;
            WDT_TRY(make_plan(b));
            for (int i = 0; i < b->nsys; ++i) b->host[i].vec[V_X] = b->host[i].vec[V_B] = b->host[i].vec[V_R];
            WDT_TRY(upload(b));
            // timing data: zero vectors and inactive states (the kernels' cost
            // does not depend on the values)
            hipLaunchKernelGGL(kb_copy, dim3(b->total_blocks), dim3(256), 0, b->stream, b->dev,
                               b->nsys, -1, (int)V_R);
            for (int v = V_RHAT; v < V_COUNT; ++v)
                hipLaunchKernelGGL(kb_copy, dim3(b->total_blocks), dim3(256), 0, b->stream, b->dev,
                                   b->nsys, (int)V_R, v);
            WDT_HIP(hipMemsetAsync(b->st, 0, sizeof(RhsState) * b->total_rhs, b->stream));
            WDT_TRY(capture(b));
            WDT_HIP(hipGraphLaunch(b->exec, b->stream));
            WDT_HIP(hipEventRecord(e0, b->stream));
            for (int k = 0; k < iters; ++k) WDT_HIP(hipGraphLaunch(b->exec, b->stream));
            WDT_HIP(hipEventRecord(e1, b->stream));
            WDT_HIP(hipEventSynchronize(e1));
            float ms = 0;
            WDT_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bb = bpc;
                bt = tc;
            }
        }
    b->blocks_per_cu = bb;
    b->tile_cap = bt;
    WDT_TRY(make_plan(b));
    if (best_ms) *best_ms = best / iters;
    return WDT_OK;
}

int wdt_batch_solve(wdt_batch b, void *const *dev_b, void *const *dev_x,
                    const wdt_solve_params *P, wdt_rhs_stats *stats, void *stream) {
    WDT_CHECK(b && dev_b && dev_x && P, "wdt_batch_solve: bad argument");
    WDT_CHECK(P->prec == WDT_FP64, "wdt_batch_solve: only WDT_FP64 is supported");
    WDT_CHECK(P->tol > 0 && P->tol < 1 && P->max_iter >= 1, "wdt_batch_solve: bad tolerance");
    for (int i = 0; i < b->nsys; ++i) {
        WDT_CHECK(dev_b[i] && dev_x[i] && dev_b[i] != dev_x[i], "wdt_batch_solve: system %d", i);
        b->host[i].vec[V_B] = (double2 *)dev_b[i];
        b->host[i].vec[V_X] = (double2 *)dev_x[i];
        // the gauge's clover term as it is now (it may have been set, changed
        // or removed since the plan was made)
        b->host[i].C = b->gauges[i]->C64;
        b->host[i].eo = (b->gauges[i]->lat.even_odd_ok() && tuning().eo != 0 &&
                         !b->gauges[i]->C64) ? 1 : 0;
    }
    // the batch stream runs after the caller's stream, and the caller's after it
    StreamJoin join((hipStream_t)stream, b->stream);
    if (join.rc < 0) return join.rc;
    assign_blocks(b, std::vector<char>(b->nsys, 1));
    WDT_TRY(upload(b));
    if (!P->x0_is_guess)
        hipLaunchKernelGGL(kb_copy, dim3(b->total_blocks), dim3(256), 0, b->stream, b->dev,
                           b->nsys, -1, (int)V_X);
    WDT_HIP(hipMemsetAsync(b->st, 0, sizeof(RhsState) * b->total_rhs, b->stream));
    WDT_TRY(capture(b));
    const int check = P->check_every > 0 ? P->check_every : 5;
    std::vector<RhsState> hs(b->total_rhs);
    std::vector<int> total_it(b->total_rhs, 0), restarts(b->total_rhs, 0), before(b->total_rhs);
    const std::vector<char> all(b->nsys, 1);
    std::vector<char> act(b->nsys, 1), dealt(b->nsys, 1);
    // which systems still have an active RHS (from the host copy of the states)
    auto active_systems = [&]() {
        bool any = false;
        for (int i = 0; i < b->nsys; ++i) {
            const SysDesc &d = b->host[i];
            char a = 0;
            for (int k = 0; k < d.N; ++k) a |= hs[d.rhs_begin + k].active ? 1 : 0;
            act[i] = a;
            any = any || a;
        }
        return any;
    };
    // deal the blocks over the active systems when that set has changed
    auto redeal = [&]() -> int {
        if (act == dealt) return WDT_OK;
        assign_blocks(b, act);
        dealt = act;
        WDT_TRY(upload(b));
        return capture(b);
    };
    int budget = P->max_iter, rc = WDT_OK;
    for (int round = 0;; ++round) {
        // the true residual is taken for every system
        if (dealt != all) {
            assign_blocks(b, all);
            dealt = all;
            WDT_TRY(upload(b));
        }
        WDT_TRY(restart(b, P->tol));
        WDT_HIP(hipMemcpyAsync(hs.data(), b->st, sizeof(RhsState) * b->total_rhs,
                               hipMemcpyDeviceToHost, b->stream));
        WDT_HIP(hipStreamSynchronize(b->stream));
        bool any = false;
        for (auto &s : hs) any = any || s.active;
        if (!any || budget <= 0 || round > 50) {
            for (int k = 0; k < b->total_rhs; ++k) {
                if (stats) {
                    stats[k].iterations = total_it[k];
                    stats[k].outer = 0;
                    stats[k].converged = (!hs[k].active && hs[k].flag == 1) ? 1 : 0;
                    stats[k].restarts = restarts[k];
                    stats[k].true_residual = hs[k].bb > 0 ? std::sqrt(hs[k].rr / hs[k].bb) : 0.0;
                }
                if (hs[k].active || hs[k].flag != 1) rc = WDT_WNOTCONVERGED;
            }
            break;
        }
        for (int k = 0; k < b->total_rhs; ++k) {
            if (hs[k].active && round > 0) restarts[k] += 1;
            before[k] = hs[k].iters;
        }
        active_systems();
        WDT_TRY(redeal());
        int it = 0;
        while (it < budget) {
            WDT_HIP(hipGraphLaunch(b->exec, b->stream));
            ++it;
            if (it % check == 0) {
                WDT_HIP(hipMemcpyAsync(hs.data(), b->st, sizeof(RhsState) * b->total_rhs,
                                       hipMemcpyDeviceToHost, b->stream));
                WDT_HIP(hipStreamSynchronize(b->stream));
                if (!active_systems()) break;
                WDT_TRY(redeal());
            }
        }
        // odd sites of x from b and the even sites (a full-lattice launch:
        // every system, dealt like the restart)
        if (dealt != all) {
            assign_blocks(b, all);
            dealt = all;
            WDT_TRY(upload(b));
        }
        hipLaunchKernelGGL(kb_schur_odd, dim3(b->total_blocks), dim3(256), 0, b->stream, b->dev,
                           b->nsys);
        WDT_HIP(hipGetLastError());
        WDT_HIP(hipMemcpyAsync(hs.data(), b->st, sizeof(RhsState) * b->total_rhs,
                               hipMemcpyDeviceToHost, b->stream));
        WDT_HIP(hipStreamSynchronize(b->stream));
        for (int k = 0; k < b->total_rhs; ++k) total_it[k] += hs[k].iters - before[k];
        budget -= it;
    }
    return rc;
}

int wdt_batch_info(wdt_batch b, int32_t *total_blocks, int32_t *blocks_per_cu, int32_t *tile_cap) {
    WDT_CHECK(b, "wdt_batch_info: null batch");
    if (total_blocks) *total_blocks = b->total_blocks;
    if (blocks_per_cu) *blocks_per_cu = b->blocks_per_cu;
    if (tile_cap) *tile_cap = b->tile_cap;
    return WDT_OK;
}

}  // extern "C"
