// Handles, errors, gauge upload, torus colouring search, layout bridge.
#include "internal.h"

#include <stdio.h>
#include <string.h>

#include <cstdlib>
#include <new>

namespace wdt {

static thread_local char g_err[512] = "";

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

const char *last_error() { return g_err; }

size_t spinor_bytes(int64_t V, int N, int prec) {
    switch (prec) {
        case WDT_FP64: return (size_t)V * 12 * N * 16;
        case WDT_FP32: return (size_t)V * 12 * N * 8;
        case WDT_FP16: return (size_t)V * 12 * N * 4 + (size_t)V * N * 4;
        case WDT_BF16: return (size_t)V * 12 * N * 4;
        default: return 0;
    }
}

size_t site_bytes(int prec) {
    return prec == WDT_FP64 ? 192 : prec == WDT_FP32 ? 96 : prec == WDT_BF16 ? 48 : 52;
}
size_t link_bytes(int prec) {
    return prec == WDT_FP64 ? 144 : 72;  // FP32 links (also BF16); FP16: two packed halves per element
}

// ---------------------------------------------------------------------------
// Launch timing registry.
namespace {
struct ProfClass {
    std::string name;
    int64_t calls = 0;
    double ms = 0, bytes = 0;
};
struct ProfPending {
    int cls;
    hipEvent_t a, b;
    double bytes;
};
struct ProfState {
    bool on = false;
    size_t drained = 0;  // entries drained so far (marks count from the start)
    std::vector<ProfClass> classes;
    std::vector<ProfPending> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        hipEvent_t e;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
    int cls(const char *name) {
        for (size_t i = 0; i < classes.size(); ++i)
            if (classes[i].name == name) return (int)i;
        classes.push_back(ProfClass{name});
        return (int)classes.size() - 1;
    }
    void drain() {
        for (auto &p : pending) {
            float ms = 0.f;
            if (p.a && p.b && hipEventSynchronize(p.b) == hipSuccess &&
                hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                classes[p.cls].calls += 1;
                classes[p.cls].ms += ms;
                classes[p.cls].bytes += p.bytes;
            }
            if (p.a) pool.push_back(p.a);
            if (p.b) pool.push_back(p.b);
        }
        drained += pending.size();
        pending.clear();
    }
};
ProfState g_prof;
}  // namespace

ProfScope::ProfScope(const char *name, double bytes, hipStream_t s) : stop(nullptr), stream(s) {
    if (!g_prof.on) return;
    if (g_prof.pending.size() > 4096) g_prof.drain();
    ProfPending p{g_prof.cls(name), g_prof.get(), g_prof.get(), bytes};
    if (!p.a || !p.b) return;
    (void)hipEventRecord(p.a, s);
    g_prof.pending.push_back(p);
    stop = p.b;
}

ProfScope::~ProfScope() {
    if (stop) (void)hipEventRecord(stop, stream);
}

size_t prof_mark() { return g_prof.drained + g_prof.pending.size(); }

void prof_discard(size_t mark) {
    if (mark < g_prof.drained) return;  // already counted
    const size_t keep = mark - g_prof.drained;
    for (size_t i = keep; i < g_prof.pending.size(); ++i) {
        if (g_prof.pending[i].a) g_prof.pool.push_back(g_prof.pending[i].a);
        if (g_prof.pending[i].b) g_prof.pool.push_back(g_prof.pending[i].b);
    }
    if (keep < g_prof.pending.size()) g_prof.pending.resize(keep);
}

// Converts FP64 links to the FP32 copy (FP32 operator) and to the paired
// half form of the FP16 operator: element u -> (ur, -ui), (ui, ur).
__global__ void k_links_lower(const double2 *__restrict__ U, float2 *__restrict__ U32,
                              __half2 *__restrict__ U16, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 u = U[i];
        U32[i] = make_float2((float)u.x, (float)u.y);
        U16[2 * i] = __floats2half2_rn((float)u.x, -(float)u.y);
        U16[2 * i + 1] = __floats2half2_rn((float)u.y, (float)u.x);
    }
}

// natural [N][V*12] <-> batch [V*12][N] (complex double): a tiled transpose
// of a row-major [rows][cols] matrix; 1D grid over 32x32 tiles.
__global__ void k_transpose_c128(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                 int64_t rows, int64_t cols) {
    __shared__ double2 tile[32][33];
    const int64_t ntc = (cols + 31) / 32;
    const int64_t tr = (int64_t)blockIdx.x / ntc, tc = (int64_t)blockIdx.x % ntc;
    const int64_t r0 = tr * 32, c0 = tc * 32;
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int64_t rr = r0 + j, cc = c0 + threadIdx.x;
        if (rr < rows && cc < cols) tile[j][threadIdx.x] = src[rr * cols + cc];
    }
    __syncthreads();
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int64_t cc = c0 + j, rr = r0 + threadIdx.x;
        if (rr < rows && cc < cols) dst[cc * rows + rr] = tile[threadIdx.x][j];
    }
}

static int transpose(const void *src, void *dst, int64_t rows, int64_t cols, hipStream_t s) {
    const int64_t tiles = ((rows + 31) / 32) * ((cols + 31) / 32);
    if (tiles > 2147483647LL) return set_error(WDT_EINVAL, "transpose too large");
    hipLaunchKernelGGL(k_transpose_c128, dim3((unsigned)tiles), dim3(32, 8), 0, s,
                       (const double2 *)src, (double2 *)dst, rows, cols);
    WDT_HIP(hipGetLastError());
    return WDT_OK;
}

}  // namespace wdt

using namespace wdt;

extern "C" {

const char *wdt_error_string(int code) {
    switch (code) {
        case WDT_OK: return "ok";
        case WDT_WNOTCONVERGED: return "some right-hand sides did not converge";
        case WDT_EINVAL: return "invalid argument";
        case WDT_ENOMEM: return "out of memory";
        case WDT_EHIP: return "HIP runtime error";
        case WDT_ESEARCH: return "no colouring found";
        case WDT_ENODEVICE: return "no usable gfx950 device";
        default: return "unknown error";
    }
}

int wdt_last_error_detail(char *buf, size_t len) {
    if (!buf || len == 0) return WDT_EINVAL;
    snprintf(buf, len, "%s", last_error());
    return WDT_OK;
}

const char *wdt_version(void) { return "wdt 0.1 gfx950"; }

int wdt_init(int hip_device) {
    int n = 0;
    WDT_HIP(hipGetDeviceCount(&n));
    if (hip_device < 0 || hip_device >= n)
        return set_error(WDT_ENODEVICE, "device %d not present (%d devices)", hip_device, n);
    WDT_HIP(hipSetDevice(hip_device));
    hipDeviceProp_t prop;
    WDT_HIP(hipGetDeviceProperties(&prop, hip_device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(WDT_ENODEVICE, "device %d is %s, this library is built for gfx950",
                         hip_device, prop.gcnArchName);
    return WDT_OK;
}

int wdt_lattice_create(const int32_t dims[4], int32_t bc_t, wdt_lattice *out) {
    WDT_CHECK(dims != nullptr && out != nullptr, "wdt_lattice_create: null argument");
    WDT_CHECK(bc_t == 1 || bc_t == -1, "wdt_lattice_create: bc_t must be +1 or -1");
    int64_t V = 1;
    for (int i = 0; i < 4; ++i) {
        WDT_CHECK(dims[i] >= 2, "wdt_lattice_create: extent %d of direction %d < 2", dims[i], i);
        V *= dims[i];
    }
    WDT_CHECK(V * 12 < 2147483647LL, "wdt_lattice_create: volume %lld too large", (long long)V);
    wdt_lattice_s *L = new (std::nothrow) wdt_lattice_s;
    if (!L) return set_error(WDT_ENOMEM, "wdt_lattice_create: host allocation");
    for (int i = 0; i < 4; ++i) L->dims[i] = dims[i];
    L->bc_t = bc_t;
    L->V = V;
    L->device = 0;
    (void)hipGetDevice(&L->device);
    *out = L;
    return WDT_OK;
}

int wdt_lattice_destroy(wdt_lattice lat) {
    delete lat;
    return WDT_OK;
}

int wdt_lattice_volume(wdt_lattice lat, int64_t *volume) {
    WDT_CHECK(lat && volume, "wdt_lattice_volume: null argument");
    *volume = lat->V;
    return WDT_OK;
}

int64_t wdt_spinor_bytes(wdt_lattice lat, int32_t n_rhs, int32_t prec) {
    if (!lat || n_rhs < 1 || prec < WDT_FP64 || prec > WDT_BF16)
        return set_error(WDT_EINVAL, "wdt_spinor_bytes: bad argument");
    return (int64_t)spinor_bytes(lat->V, n_rhs, prec);
}

int wdt_gauge_create(wdt_lattice lat, const double *host_links, wdt_gauge *out) {
    WDT_CHECK(lat && host_links && out, "wdt_gauge_create: null argument");
    wdt_gauge_s *g = new (std::nothrow) wdt_gauge_s;
    if (!g) return set_error(WDT_ENOMEM, "wdt_gauge_create: host allocation");
    g->lat = *lat;
    const int64_t n = lat->V * 4 * 9;
    hipError_t e1 = hipMalloc(&g->U64, n * sizeof(double2));
    hipError_t e2 = hipMalloc(&g->U32, n * sizeof(float2));
    hipError_t e3 = hipMalloc(&g->U16, 2 * n * sizeof(__half2));
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        (void)hipGetLastError();
        if (g->U64) (void)hipFree(g->U64);
        if (g->U32) (void)hipFree(g->U32);
        if (g->U16) (void)hipFree(g->U16);
        delete g;
        return set_error(WDT_ENOMEM, "wdt_gauge_create: device allocation failed");
    }
    hipError_t e = hipMemcpy(g->U64, host_links, n * sizeof(double2), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_links_lower, dim3(1024), dim3(256), 0, 0, g->U64, g->U32, g->U16, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(g->U64);
        (void)hipFree(g->U32);
        (void)hipFree(g->U16);
        delete g;
        return set_error(WDT_EHIP, "wdt_gauge_create: %s", hipGetErrorString(e));
    }
    *out = g;
    return WDT_OK;
}

int wdt_gauge_destroy(wdt_gauge g) {
    if (!g) return WDT_OK;
    (void)hipFree(g->U64);
    (void)hipFree(g->U32);
    (void)hipFree(g->U16);
    if (g->C64) (void)hipFree(g->C64);
    if (g->C32) (void)hipFree(g->C32);
    if (g->Ci64) (void)hipFree(g->Ci64);
    if (g->Ci32) (void)hipFree(g->Ci32);
    if (g->ws.ptr) (void)hipFree(g->ws.ptr);
    if (g->live_host) (void)hipHostFree(g->live_host);
    delete g;
    return WDT_OK;
}

int wdt_gauge_get(wdt_gauge g, double *host_links) {
    WDT_CHECK(g && host_links, "wdt_gauge_get: null argument");
    WDT_HIP(hipMemcpy(host_links, g->U64, g->lat.V * 36 * sizeof(double2), hipMemcpyDeviceToHost));
    return WDT_OK;
}

int wdt_set_launch_shape(const wdt_launch_shape *sh) {
    WDT_CHECK(sh != nullptr, "wdt_set_launch_shape: null shape");
    WDT_CHECK(sh->rhs_tile >= 0 && sh->rhs_tile <= 256, "wdt_set_launch_shape: rhs_tile must be 0..256");
    WDT_CHECK(sh->sites_per_block >= 0 && sh->sites_per_block <= 256,
              "wdt_set_launch_shape: sites_per_block must be 0..256");
    WDT_CHECK(sh->max_blocks >= 0, "wdt_set_launch_shape: max_blocks must be >= 0");
    WDT_CHECK(sh->z_slab >= 0, "wdt_set_launch_shape: z_slab must be >= 0");
    WDT_CHECK(sh->serial_tiles >= -1 && sh->serial_tiles <= 1,
              "wdt_set_launch_shape: serial_tiles must be -1, 0 or 1");
    WDT_CHECK(sh->t_chunk >= -1, "wdt_set_launch_shape: t_chunk must be >= -1");
    const bool brick_off = sh->brick[0] == -1 && sh->brick[1] == -1 && sh->brick[2] == -1;
    const bool brick_auto = sh->brick[0] == 0 && sh->brick[1] == 0 && sh->brick[2] == 0;
    WDT_CHECK(brick_off || brick_auto ||
                  (sh->brick[0] > 0 && sh->brick[1] > 0 && sh->brick[2] > 0 &&
                   sh->brick[0] < 100 && sh->brick[1] < 100 && sh->brick[2] < 100),
              "wdt_set_launch_shape: brick must be {0,0,0}, {-1,-1,-1} or three extents 1..99");
    LaunchTuning &t = tuning();
    t.nt = sh->rhs_tile;
    t.sb = sh->sites_per_block;
    t.gmax = sh->max_blocks;
    t.bz = sh->z_slab;
    t.serial = sh->serial_tiles;
    t.tchunk = sh->t_chunk;
    t.brick = brick_off ? -1 : brick_auto ? 0 : sh->brick[0] * 10000 + sh->brick[1] * 100 + sh->brick[2];
    WDT_CHECK(sh->wave_per_site >= -1 && sh->wave_per_site <= 1,
              "wdt_set_launch_shape: wave_per_site must be -1, 0 or 1");
    t.wps = sh->wave_per_site;
    WDT_CHECK(sh->even_odd >= -1 && sh->even_odd <= 1,
              "wdt_set_launch_shape: even_odd must be -1, 0 or 1");
    t.eo = sh->even_odd;
    return WDT_OK;
}

int wdt_profile_enable(int on) {
    if (on) {
        g_prof.drain();
        g_prof.classes.clear();
    }
    g_prof.on = on != 0;
    return WDT_OK;
}

int wdt_profile_read(wdt_prof_entry *out, int32_t max, int32_t *n) {
    WDT_CHECK(n != nullptr, "wdt_profile_read: null count");
    g_prof.drain();
    *n = (int32_t)g_prof.classes.size();
    for (int i = 0; i < *n && i < max && out; ++i) {
        snprintf(out[i].name, sizeof(out[i].name), "%s", g_prof.classes[i].name.c_str());
        out[i].calls = g_prof.classes[i].calls;
        out[i].ms = g_prof.classes[i].ms;
        out[i].bytes = g_prof.classes[i].bytes;
    }
    return WDT_OK;
}

int wdt_pack_spinor(wdt_lattice lat, const void *dev_natural, void *dev_batch, int32_t n_rhs,
                    void *stream) {
    WDT_CHECK(lat && dev_natural && dev_batch && n_rhs >= 1, "wdt_pack_spinor: bad argument");
    WDT_CHECK(dev_natural != dev_batch, "wdt_pack_spinor: buffers must not overlap");
    return transpose(dev_natural, dev_batch, n_rhs, lat->V * 12, (hipStream_t)stream);
}

int wdt_unpack_spinor(wdt_lattice lat, const void *dev_batch, void *dev_natural, int32_t n_rhs,
                      void *stream) {
    WDT_CHECK(lat && dev_natural && dev_batch && n_rhs >= 1, "wdt_unpack_spinor: bad argument");
    WDT_CHECK(dev_natural != dev_batch, "wdt_unpack_spinor: buffers must not overlap");
    return transpose(dev_batch, dev_natural, lat->V * 12, n_rhs, (hipStream_t)stream);
}

}  // extern "C"
