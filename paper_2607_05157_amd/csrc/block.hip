// Block kernels over FP64 batches for the low-mode subspace of the
// deflated estimator (Sec. 2, eq. defl-split: the projector V V^dag on k
// low modes of Q = gamma5 D).  Both are tall-skinny dense products with the
// long index running over sites and spin-colour:
//   block_dot:     G = X^dag Y            (nx x ny, summed over 12 V rows)
//   block_combine: Y = beta Y + X W       (W small, nx x ny)
// They are bound by reading the batches (FP64 matrix and vector peaks are the
// same on this chip, so MFMA would not raise the ceiling); both keep the
// batch layout [V][12][n] (RHS innermost), so a site's rows are contiguous.
#include "internal.h"

#include <vector>

namespace wdt {

constexpr int kBlockMax = 64;  // largest nx, ny
constexpr int kDotSites = 2;   // sites staged in LDS per step

// Per-block partial sums of X^dag Y: block b accumulates its share of the
// sites; thread t owns the entries e = t + 256 m (i = e / ny, j = e % ny).
__global__ __launch_bounds__(256) void k_block_dot(const double2 *__restrict__ X, int nx,
                                                   const double2 *__restrict__ Y, int ny,
                                                   int64_t V, double2 *__restrict__ part) {
    __shared__ double2 xs[kDotSites * 12 * kBlockMax];
    __shared__ double2 ys[kDotSites * 12 * kBlockMax];
    const int tid = threadIdx.x;
    const int ne = nx * ny;
    constexpr int M = kBlockMax * kBlockMax / 256;
    double ar[M], ai[M];
#pragma unroll
    for (int m = 0; m < M; ++m) ar[m] = ai[m] = 0.0;
    const int64_t nsteps = (V + kDotSites - 1) / kDotSites;
    for (int64_t st = blockIdx.x; st < nsteps; st += gridDim.x) {
        const int64_t s0 = st * kDotSites;
        const int ns = (int)((V - s0) < kDotSites ? (V - s0) : kDotSites);
        const int nxr = ns * 12 * nx, nyr = ns * 12 * ny;
        __syncthreads();
        for (int q = tid; q < nxr; q += 256) xs[q] = X[s0 * 12 * nx + q];
        for (int q = tid; q < nyr; q += 256) ys[q] = Y[s0 * 12 * ny + q];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = tid + 256 * m;
            if (e >= ne) break;
            const int i = e / ny, j = e - (e / ny) * ny;
            double sr = 0.0, si = 0.0;
            for (int rrow = 0; rrow < ns * 12; ++rrow) {
                const double2 a = xs[rrow * nx + i], b = ys[rrow * ny + j];
                // conj(a) b
                sr += a.x * b.x + a.y * b.y;
                si += a.x * b.y - a.y * b.x;
            }
            ar[m] += sr;
            ai[m] += si;
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = tid + 256 * m;
        if (e < ne) part[(size_t)blockIdx.x * ne + e] = make_double2(ar[m], ai[m]);
    }
}

// out[e] = sum over the G block partials, in block order.
__global__ void k_block_dot_reduce(const double2 *__restrict__ part, int G, int ne,
                                   double2 *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double2 s = make_double2(0.0, 0.0);
    for (int b = 0; b < G; ++b) {
        const double2 v = part[(size_t)b * ne + e];
        s.x += v.x;
        s.y += v.y;
    }
    out[e] = s;
}

// Y[row][j] = beta Y[row][j] + sum_i X[row][i] W[i][j], rows = 12 V (site,
// spin-colour); one thread per output element, j fastest (coalesced stores;
// the X row is read by the ny threads of one row together).
__global__ __launch_bounds__(256) void k_block_combine(const double2 *__restrict__ X, int nx,
                                                       const double2 *__restrict__ W, int ny,
                                                       double beta, int64_t rows,
                                                       double2 *__restrict__ Y) {
    const int64_t n = rows * ny;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = q / ny;
        const int j = (int)(q - row * ny);
        const double2 *xr = X + row * nx;
        double sr = 0.0, si = 0.0;
        for (int i = 0; i < nx; ++i) {
            const double2 a = xr[i], w = W[i * ny + j];
            sr += a.x * w.x - a.y * w.y;
            si += a.x * w.y + a.y * w.x;
        }
        double2 y = make_double2(sr, si);
        if (beta != 0.0) {
            const double2 o = Y[q];
            y.x += beta * o.x;
            y.y += beta * o.y;
        }
        Y[q] = y;
    }
}

}  // namespace wdt

using namespace wdt;

extern "C" {

int wdt_block_dot(wdt_lattice lat, const void *dev_x, int32_t nx, const void *dev_y, int32_t ny,
                  double *host_out, void *stream) {
    WDT_CHECK(lat && dev_x && dev_y && host_out, "wdt_block_dot: null argument");
    WDT_CHECK(nx >= 1 && nx <= kBlockMax && ny >= 1 && ny <= kBlockMax,
              "wdt_block_dot: nx and ny must be 1..%d", kBlockMax);
    const hipStream_t st = (hipStream_t)stream;
    const int ne = nx * ny;
    const int64_t nsteps = (lat->V + kDotSites - 1) / kDotSites;
    const int G = (int)std::min<int64_t>(nsteps, 1024);
    AsyncScratch scratch(st);
    if (!scratch.alloc(sizeof(double2) * ((size_t)G + 1) * ne))
        return set_error(WDT_ENOMEM, "wdt_block_dot: scratch allocation failed");
    double2 *part = (double2 *)scratch.p;
    double2 *out = part + (size_t)G * ne;
    hipLaunchKernelGGL(k_block_dot, dim3(G), dim3(256), 0, st, (const double2 *)dev_x, nx,
                       (const double2 *)dev_y, ny, lat->V, part);
    hipLaunchKernelGGL(k_block_dot_reduce, dim3((ne + 255) / 256), dim3(256), 0, st, part, G, ne,
                       out);
    WDT_HIP(hipGetLastError());
    WDT_HIP(hipMemcpyAsync(host_out, out, sizeof(double2) * ne, hipMemcpyDeviceToHost, st));
    WDT_HIP(hipStreamSynchronize(st));
    return WDT_OK;
}

int wdt_block_combine(wdt_lattice lat, const void *dev_x, int32_t nx, const double *W, int32_t ny,
                      double beta, void *dev_y, void *stream) {
    WDT_CHECK(lat && dev_x && W && dev_y, "wdt_block_combine: null argument");
    WDT_CHECK(nx >= 1 && nx <= kBlockMax && ny >= 1 && ny <= kBlockMax,
              "wdt_block_combine: nx and ny must be 1..%d", kBlockMax);
    const hipStream_t st = (hipStream_t)stream;
    const int64_t rows = lat->V * 12;
    {
        // X and Y must not overlap
        const char *x0 = (const char *)dev_x, *x1 = x0 + sizeof(double2) * rows * nx;
        const char *y0 = (const char *)dev_y, *y1 = y0 + sizeof(double2) * rows * ny;
        WDT_CHECK(x1 <= y0 || y1 <= x0, "wdt_block_combine: dev_x and dev_y overlap");
    }
    AsyncScratch scratch(st);
    if (!scratch.alloc(sizeof(double2) * (size_t)nx * ny))
        return set_error(WDT_ENOMEM, "wdt_block_combine: scratch allocation failed");
    double2 *dw = (double2 *)scratch.p;
    WDT_HIP(hipMemcpyAsync(dw, W, sizeof(double2) * (size_t)nx * ny, hipMemcpyHostToDevice, st));
    const int64_t n = rows * ny;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_block_combine, dim3(blocks), dim3(256), 0, st, (const double2 *)dev_x, nx,
                       dw, ny, beta, rows, (double2 *)dev_y);
    WDT_HIP(hipGetLastError());
    // W is host memory: the copy above must finish before the caller reuses it
    WDT_HIP(hipStreamSynchronize(st));
    return WDT_OK;
}

}  // extern "C"
