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

// Threads of k_block_dot: ceil(nx/4) x ceil(ny/4) tiles of 4 x 4 entries,
// and as many groups of them as fit in 256 threads; group g takes every
// groups-th staged row and writes its own partial.
__host__ __device__ inline int dot_groups(int nx, int ny) {
    const int ntile = ((nx + 3) / 4) * ((ny + 3) / 4);
    return ntile >= 256 ? 1 : 256 / ntile;
}
// sites staged per step: as many as the LDS arrays hold for these widths
__host__ __device__ inline int dot_sites(int nx, int ny) {
    const int w = nx > ny ? nx : ny;
    const int s = kDotSites * kBlockMax / w;
    return s < 1 ? 1 : s > 16 ? 16 : s;
}

// Per-block partial sums of X^dag Y: block b accumulates its share of the
// sites, staged dot_sites at a time in LDS.  A thread owns a 4 x 4 tile of
// entries: per staged row it reads 4 X and 4 Y elements for 16 complex
// multiply-adds.  The groups' tiles are added up in LDS in group order;
// partials: [G][nx * ny].
__global__ __launch_bounds__(256) void k_block_dot(const double2 *__restrict__ X, int nx,
                                                   const double2 *__restrict__ Y, int ny,
                                                   int64_t V, double2 *__restrict__ part) {
    __shared__ double2 stage[2 * kDotSites * 12 * kBlockMax];
    double2 *xs = stage, *ys = stage + kDotSites * 12 * kBlockMax;
    const int tid = threadIdx.x;
    const int ty = (ny + 3) / 4, ntile = ((nx + 3) / 4) * ty;
    const int groups = dot_groups(nx, ny), spb = dot_sites(nx, ny);
    const int g = tid / ntile, tile = tid - (tid / ntile) * ntile;
    const bool act = g < groups;
    const int i0 = 4 * (tile / ty), j0 = 4 * (tile % ty);
    double ar[4][4], ai[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) ar[a][c] = ai[a][c] = 0.0;
    const int64_t nsteps = (V + spb - 1) / spb;
    for (int64_t st = blockIdx.x; st < nsteps; st += gridDim.x) {
        const int64_t s0 = st * spb;
        const int ns = (int)((V - s0) < spb ? (V - s0) : spb);
        const int nxr = ns * 12 * nx, nyr = ns * 12 * ny;
        __syncthreads();
        for (int q = tid; q < nxr; q += 256) xs[q] = X[s0 * 12 * nx + q];
        for (int q = tid; q < nyr; q += 256) ys[q] = Y[s0 * 12 * ny + q];
        __syncthreads();
        if (act) {
            for (int rrow = g; rrow < ns * 12; rrow += groups) {
                double2 xa[4], yc[4];
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    xa[a] = (i0 + a < nx) ? xs[rrow * nx + i0 + a] : make_double2(0.0, 0.0);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    yc[c] = (j0 + c < ny) ? ys[rrow * ny + j0 + c] : make_double2(0.0, 0.0);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        // conj(x) y
                        ar[a][c] += xa[a].x * yc[c].x + xa[a].y * yc[c].y;
                        ai[a][c] += xa[a].x * yc[c].y - xa[a].y * yc[c].x;
                    }
            }
        }
    }
    const int ne = nx * ny;
    double2 *pp = part + (size_t)blockIdx.x * ne;
    if (groups == 1) {
        if (!act) return;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (i0 + a < nx && j0 + c < ny)
                    pp[(i0 + a) * ny + j0 + c] = make_double2(ar[a][c], ai[a][c]);
        return;
    }
    // groups > 1 means ntile <= 128, so ne <= 2048 fits the staging area
    double2 *acc = stage;
    __syncthreads();
    for (int gg = 0; gg < groups; ++gg) {
        if (g == gg) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (i0 + a < nx && j0 + c < ny) {
                        const int e = (i0 + a) * ny + j0 + c;
                        const double2 o = gg ? acc[e] : make_double2(0.0, 0.0);
                        acc[e] = make_double2(o.x + ar[a][c], o.y + ai[a][c]);
                    }
        }
        __syncthreads();
    }
    for (int e = tid; e < ne; e += 256) pp[e] = acc[e];
}

// out[e] = sum over the G partials, in order.
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
// spin-colour).  W is staged in LDS once per block; each thread computes a
// tile of kRows consecutive rows x kCols consecutive columns, so per i it
// reads kRows X elements and kCols W elements for kRows x kCols complex
// multiply-adds (column groups fastest across threads: coalesced stores).
constexpr int kCols = 4, kRows = 4;
__global__ __launch_bounds__(256) void k_block_combine(const double2 *__restrict__ X, int nx,
                                                       const double2 *__restrict__ W, int ny,
                                                       double beta, int64_t rows,
                                                       double2 *__restrict__ Y) {
    __shared__ double2 ws[kBlockMax * kBlockMax];
    for (int q = threadIdx.x; q < nx * ny; q += blockDim.x) ws[q] = W[q];
    __syncthreads();
    const int ngr = (ny + kCols - 1) / kCols;        // column groups per row group
    const int64_t nrg = (rows + kRows - 1) / kRows;  // row groups
    const int64_t n = nrg * ngr;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r0 = (q / ngr) * kRows;
        const int j0 = (int)(q % ngr) * kCols;
        double sr[kRows][kCols], si[kRows][kCols];
#pragma unroll
        for (int a = 0; a < kRows; ++a)
#pragma unroll
            for (int c = 0; c < kCols; ++c) sr[a][c] = si[a][c] = 0.0;
        for (int i = 0; i < nx; ++i) {
            double2 xa[kRows], wc[kCols];
#pragma unroll
            for (int a = 0; a < kRows; ++a)
                xa[a] = (r0 + a < rows) ? X[(r0 + a) * nx + i] : make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < kCols; ++c)
                wc[c] = (j0 + c < ny) ? ws[i * ny + j0 + c] : make_double2(0.0, 0.0);
#pragma unroll
            for (int a = 0; a < kRows; ++a)
#pragma unroll
                for (int c = 0; c < kCols; ++c) {
                    sr[a][c] += xa[a].x * wc[c].x - xa[a].y * wc[c].y;
                    si[a][c] += xa[a].x * wc[c].y + xa[a].y * wc[c].x;
                }
        }
#pragma unroll
        for (int a = 0; a < kRows; ++a) {
            if (r0 + a >= rows) break;
            double2 *yr = Y + (r0 + a) * ny + j0;
#pragma unroll
            for (int c = 0; c < kCols; ++c) {
                if (j0 + c < ny) {
                    double2 y = make_double2(sr[a][c], si[a][c]);
                    if (beta != 0.0) {
                        const double2 o = yr[c];
                        y.x += beta * o.x;
                        y.y += beta * o.y;
                    }
                    yr[c] = y;
                }
            }
        }
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
    const int64_t nsteps = (lat->V + dot_sites(nx, ny) - 1) / dot_sites(nx, ny);
    const int G = (int)std::min<int64_t>(nsteps, 1024);
    const int np = G;  // partials
    AsyncScratch scratch(st);
    if (!scratch.alloc(sizeof(double2) * ((size_t)np + 1) * ne))
        return set_error(WDT_ENOMEM, "wdt_block_dot: scratch allocation failed");
    double2 *part = (double2 *)scratch.p;
    double2 *out = part + (size_t)np * ne;
    hipLaunchKernelGGL(k_block_dot, dim3(G), dim3(256), 0, st, (const double2 *)dev_x, nx,
                       (const double2 *)dev_y, ny, lat->V, part);
    hipLaunchKernelGGL(k_block_dot_reduce, dim3((ne + 255) / 256), dim3(256), 0, st, part, np, ne,
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
    // about the blocks the GPU holds at once (64 KB of LDS each): every block
    // stages W once and then strides over the rows
    const int64_t n = ((rows + kRows - 1) / kRows) * ((ny + kCols - 1) / kCols);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 512);
    hipLaunchKernelGGL(k_block_combine, dim3(blocks), dim3(256), 0, st, (const double2 *)dev_x, nx,
                       dw, ny, beta, rows, (double2 *)dev_y);
    WDT_HIP(hipGetLastError());
    // W is host memory: the copy above must finish before the caller reuses it
    WDT_HIP(hipStreamSynchronize(st));
    return WDT_OK;
}

}  // extern "C"
