// Host-side internals of libwdt: handle structs, error reporting and the
// launch functions the translation units share.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdarg.h>

#include <string>
#include <vector>

#include "wdt.h"
#include "device.h"

struct wdt_lattice_s {
    int dims[4];
    int bc_t;
    int64_t V;
    int device;
    // every extent even: the checkerboard is consistent across the wrap
    bool even_odd_ok() const {
        return dims[0] % 2 == 0 && dims[1] % 2 == 0 && dims[2] % 2 == 0 && dims[3] % 2 == 0;
    }
    wdt::Geom geom() const {
        wdt::Geom g;
        for (int i = 0; i < 4; ++i) g.L[i] = dims[i];
        g.stride[0] = 1;
        g.stride[1] = dims[0];
        g.stride[2] = dims[0] * dims[1];
        g.stride[3] = dims[0] * dims[1] * dims[2];
        g.V = (int)V;
        g.Lxyz = g.stride[3];
        g.bc_t = bc_t;
        g.bz = dims[2];
        g.bt = dims[3];
        g.bx = g.by = 0;
        g.parity = -1;
        g.nsites = g.V;
        return g;
    }
};

// Grow-only device workspace owned by a gauge handle (solver vectors,
// reduction partials, per-RHS scalars).
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct wdt_gauge_s {
    wdt_lattice_s lat;
    double2 *U64 = nullptr;
    float2 *U32 = nullptr;
    // FP16 operator links: per element u = (ur, ui) the pair (ur, -ui), (ui, ur)
    // of packed halves, so that both parts of u h are single half dot products
    __half2 *U16 = nullptr;
    // clover term (null without one): per site the two chiral 6 x 6 Hermitian
    // blocks, packed as 36 reals each (CLOVER_REALS per site); FP64 and FP32
    double *C64 = nullptr;
    float *C32 = nullptr;
    double csw = 0.0;
    // (a + C)^-1 in the same packed form for the even-odd solves, for the
    // a = 4 + m0 in ci_a (NaN: not computed since the term last changed)
    double *Ci64 = nullptr;
    float *Ci32 = nullptr;
    double ci_a = __builtin_nan("");
    Workspace ws;
    // two host-mapped ints (host and device address) for the solvers' loop flag
    int *live_host = nullptr;
    int *live_dev = nullptr;
};

namespace wdt {

int set_error(int code, const char *fmt, ...);
const char *last_error();

#define WDT_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::wdt::set_error(WDT_EHIP, "%s failed: %s (%s:%d)", #expr,                 \
                                    hipGetErrorString(e_), __FILE__, __LINE__);              \
    } while (0)

#define WDT_CHECK(cond, ...)                                              \
    do {                                                                  \
        if (!(cond)) return ::wdt::set_error(WDT_EINVAL, __VA_ARGS__);    \
    } while (0)

#define WDT_TRY(expr)              \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ < 0) return rc_;   \
    } while (0)

size_t spinor_bytes(int64_t V, int N, int prec);
// bytes of one (site, rhs) spinor and of one link in a precision
size_t site_bytes(int prec);
size_t link_bytes(int prec);

// Launch timing (see wdt_profile_enable): construct before a launch, destroy
// after it; records an event pair on `stream` when profiling is on.
struct ProfScope {
    ProfScope(const char *name, double bytes, hipStream_t stream);
    ~ProfScope();
    hipEvent_t stop;
    hipStream_t stream;
};
// A position in the timing record, and dropping what was recorded after it
// (launches that turned out to have nothing to do).
size_t prof_mark();
void prof_discard(size_t mark);

// Destroys an event on every path out of a scope.
struct EventGuard {
    hipEvent_t e = nullptr;
    EventGuard() = default;
    EventGuard(const EventGuard &) = delete;
    EventGuard &operator=(const EventGuard &) = delete;
    ~EventGuard() {
        if (e) (void)hipEventDestroy(e);
    }
};

// Launch shape of the (site, rhs) kernels: the RHS batch is cut into tiles
// of NT right-hand sides (grid.y); blocks of NT*SB threads handle SB sites of
// one tile at a time, and G blocks (a multiple of 8 when large) sweep the
// lattice for each tile.  Tiles keep the per-site working set small enough
// for the caches to serve the neighbour re-reads of the operator.
struct Shape {
    int NT;       // right-hand sides per tile
    int tiles;    // ceil(N / NT)
    int SB;       // sites per block iteration
    int threads;  // block size (NT*SB rounded up to a multiple of 64)
    int G;        // operator blocks per tile (about the number the GPU holds at once)
    int Gv;       // blocks per tile of the vector (BLAS-1) kernels
    int bz, bt;   // processing-order tile (see site_of)
    bool serial;  // operator blocks sweep the RHS tiles one after the other
    int tc;       // > 0: the operator marches along t in chunks of tc slices (SB columns
                  // per block, G blocks over the units); 0: it sweeps sites
    int4 brick;   // march: column bricks (x, y, z extents; x a multiple of SB)
    int4 sweep_brick;  // sweep in brick order (x, y, z extents) when x > 0
    int4 parity_brick; // one-parity sweeps: brick order (x extent even) when x > 0
    bool wps;     // operator: one site per wavefront (64 RHS lanes, 4 sites per block)
};
Shape site_shape(const wdt_lattice_s &lat, int N, int prec);
// Resident blocks per CU of the operator kernel for (prec, N, block size).
// mode: 0 site sweep, 1 t-march, 2 site sweep with one site per wavefront,
// 3 t-march with one site (column) per wavefront
int op_blocks_per_cu(int prec, int N, int threads, int mode);
// The lattice geometry with the processing order of a shape.
wdt::Geom shaped_geom(const wdt_lattice_s &lat, const Shape &sh);

// Launch-shape overrides for the tuner (0 = automatic).
struct LaunchTuning {
    int nt = 0, sb = 0, gmax = 0, bz = 0;
    int serial = -1;  // RHS tiles one after the other in each block: 1 on, 0 off, -1 automatic
    int tchunk = -1;  // operator marches along t in chunks of this many slices: 0 off, -1 automatic
    int brick = 0;    // sweep order bricks: 0 automatic, -1 off, else x*10000 + y*100 + z
    int wps = -1;     // operator one site per wavefront: 1 on, 0 off, -1 automatic
    int eo = -1;      // solvers: even-odd preconditioning 1 on, 0 off, -1 automatic
};
LaunchTuning &tuning();

// Stream-ordered scratch that is released on every path out of a scope.
struct AsyncScratch {
    void *p = nullptr;
    hipStream_t s = nullptr;
    explicit AsyncScratch(hipStream_t st) : s(st) {}
    ~AsyncScratch() {
        if (p) (void)hipFreeAsync(p, s);
    }
    bool alloc(size_t bytes) {
        if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return false;
        }
        return true;
    }
};

// Epilogues of the operator kernel.
enum Epi { EPI_NONE = 0, EPI_DOT_AUX = 1, EPI_DOT_TS = 2, EPI_RESID = 3, EPI_DOT_TSR = 4,
           EPI_NORM = 5 };

// out = D in (or D^dag in); optional fused per-RHS dot partials written to
// partials[(d*G + block)*N + r] as complex doubles.
//  EPI_DOT_AUX: d0 = aux^dag out
//  EPI_DOT_TS:  d0 = out^dag in, d1 = ||out||^2
//  EPI_DOT_TSR: as EPI_DOT_TS, and d2 = aux^dag out
//  EPI_RESID:   out = aux - D in; d0 = ||out||^2, d1 = ||aux||^2
//  EPI_NORM:    d0 = d1 = ||out||^2
int launch_dslash(const wdt_gauge_s *g, double m0, int prec, int dagger, int epi,
                  const void *in, void *out, const void *aux, int N, double2 *partials,
                  const Shape &sh, hipStream_t stream);

// The general form out = cs * self + ch * H in (H the hop sum of D: D = (4 + m0)
// - H / 2) on the sites of one parity (parity 0 or 1; lattices with every
// extent even) or on all sites (parity -1).  self = nullptr means in.
// clover: out += C self, C the gauge's clover term (cs != 0 only).
// clover_inv: out = (a + C)^-1 (cs self + ch H in) instead, with the inverse
// blocks of ensure_clover_inverse (no epilogue, D only).
struct HopSpec {
    int parity = -1;
    const void *self = nullptr;
    double cs = 0.0, ch = 1.0;
    bool clover = false;
    bool clover_inv = false;
    // solver iterations: the launch does nothing when *live == 0 (device flag)
    const int *live = nullptr;
};
int launch_hop(const wdt_gauge_s *g, int prec, int dagger, int epi, const HopSpec &hs,
               const void *in, void *out, const void *aux, int N, double2 *partials,
               const Shape &sh, hipStream_t stream);

// Reals per site of the packed clover term: two chiral blocks of 36.
constexpr int CLOVER_REALS = 72;

// Makes g->Ci64 / Ci32 hold (a + C(x))^-1 on every site (no-op when they
// already do for this a).  Stream-ordered on `stream`.
int ensure_clover_inverse(wdt_gauge_s *g, double a, hipStream_t stream);

}  // namespace wdt
