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
    __half2 *U16 = nullptr;
    Workspace ws;
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

// Launch shape of the (site, rhs) kernels: blocks of N*SB threads handle SB
// sites at a time; G blocks (a multiple of 8 when large) sweep the lattice.
struct Shape {
    int SB;       // sites per block iteration
    int threads;  // block size (N*SB rounded up to a multiple of 64)
    int G;        // grid size
    int chunk;    // site groups per block
};
Shape site_shape(int64_t V, int N);

// Epilogues of the operator kernel.
enum Epi { EPI_NONE = 0, EPI_DOT_AUX = 1, EPI_DOT_TS = 2, EPI_RESID = 3 };

// out = D in (or D^dag in); optional fused per-RHS dot partials written to
// partials[(d*G + block)*N + r] as complex doubles.
//  EPI_DOT_AUX: d0 = aux^dag out
//  EPI_DOT_TS:  d0 = out^dag in, d1 = ||out||^2
//  EPI_RESID:   out = aux - D in; d0 = ||out||^2, d1 = ||aux||^2
int launch_dslash(const wdt_gauge_s *g, double m0, int prec, int dagger, int epi,
                  const void *in, void *out, const void *aux, int N, double2 *partials,
                  const Shape &sh, hipStream_t stream);

}  // namespace wdt
