// The clover (Sheikholeslami-Wohlert) term of the Wilson-Dirac operator.
//
// The paper's operator is the Wilson-Dirac one (Sec. 1); ensembles generated
// with the O(a)-improved action add to the site's own 12 x 12 block
//   C(x) = -(c_sw / 2) sum_{mu < nu} sigma_{mu nu} (x) F_{mu nu}(x),
//   sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu],  F = (Q - Q^dag) / (8i),
// Q_{mu nu}(x) the sum of the four plaquettes of the (mu, nu) plane that
// start and end at x, all traversed in the same sense (mu first, then nu,
// rotated about x).  F keeps its colour trace.  The sign is the one whose
// tree-level c_sw = 1 cancels the Wilson term's O(a) shift.
//
// sigma_{mu nu} commutes with gamma5 = diag(1, 1, -1, -1), so C is block
// diagonal in the chiralities: two Hermitian 6 x 6 blocks per site (spins 0-1
// and 2-3, index 3 * spin + colour inside the block).  Each is stored as 36
// reals: the real diagonal, then the 15 elements above it row by row as
// (re, im).  The term is built once per gauge (one thread per site, FP64,
// from the FP64 links; the FP32 copy is rounded from it) and applied by the
// operator kernels as part of the site's own term.
#include "kernels.h"

#include <cmath>
#include <new>

namespace wdt {

namespace {

struct M3 {
    double2 e[9];
};

// A B with A, B optionally adjoint (compile-time)
template <bool DA, bool DB>
__device__ M3 mul3(const M3 &A, const M3 &B) {
    M3 C;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double2 a = DA ? A.e[3 * k + i] : A.e[3 * i + k];
                double2 b = DB ? B.e[3 * j + k] : B.e[3 * k + j];
                if (DA) a.y = -a.y;
                if (DB) b.y = -b.y;
                re += a.x * b.x - a.y * b.y;
                im += a.x * b.y + a.y * b.x;
            }
            C.e[3 * i + j] = make_double2(re, im);
        }
    }
    return C;
}

__device__ M3 link(const double2 *__restrict__ U, int site, int mu) {
    M3 m;
    const double2 *q = U + ((size_t)site * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.e[k] = q[k];
    return m;
}

// The spin blocks of -(c_sw/2) sigma_{mu nu} for the six planes mu < nu:
// sb[p][h][a][b] = that factor times sigma's element (2h + a, 2h + b).
struct SigmaBlocks {
    double2 sb[6][2][2][2];
};

}  // namespace

__global__ __launch_bounds__(128) void k_clover_build(const double2 *__restrict__ U, Geom g,
                                                      SigmaBlocks sig, double *__restrict__ C64,
                                                      float *__restrict__ C32) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    int c[4];
    {
        int q = s;
        for (int mu = 0; mu < 4; ++mu) {
            c[mu] = q % g.L[mu];
            q /= g.L[mu];
        }
    }
    // site index of x + a mu_hat + b nu_hat (periodic: gauge loops carry no
    // fermion boundary factor)
    auto shift = [&](int mu, int a, int nu, int b) {
        int d[4] = {c[0], c[1], c[2], c[3]};
        d[mu] = (d[mu] + a + g.L[mu]) % g.L[mu];
        d[nu] = (d[nu] + b + g.L[nu]) % g.L[nu];
        return d[0] + g.L[0] * (d[1] + g.L[1] * (d[2] + g.L[2] * d[3]));
    };
    double2 blk[2][6][6];
#pragma unroll
    for (int h = 0; h < 2; ++h)
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) blk[h][i][j] = make_double2(0.0, 0.0);
    int p = 0;
    for (int mu = 0; mu < 4; ++mu) {
        for (int nu = mu + 1; nu < 4; ++nu, ++p) {
            const int xm = shift(mu, -1, nu, 0), xn = shift(mu, 0, nu, -1);
            const int xpm = shift(mu, 1, nu, 0), xpn = shift(mu, 0, nu, 1);
            const int xmn = shift(mu, -1, nu, -1), xm_pn = shift(mu, -1, nu, 1);
            const int xp_mn = shift(mu, 1, nu, -1);
            // the four leaves, each from x back to x in the same sense
            const M3 l1 = mul3<false, true>(mul3<false, false>(link(U, s, mu), link(U, xpm, nu)),
                                            mul3<false, false>(link(U, s, nu), link(U, xpn, mu)));
            const M3 l2 = mul3<false, false>(
                mul3<false, true>(link(U, s, nu), link(U, xm_pn, mu)),
                mul3<true, false>(link(U, xm, nu), link(U, xm, mu)));
            const M3 l3 = mul3<true, false>(
                mul3<false, false>(link(U, xmn, nu), link(U, xm, mu)),
                mul3<false, false>(link(U, xmn, mu), link(U, xn, nu)));
            const M3 l4 = mul3<false, true>(
                mul3<true, false>(link(U, xn, nu), link(U, xn, mu)),
                mul3<false, true>(link(U, s, mu), link(U, xp_mn, nu)));
            // F = (Q - Q^dag) / (8i)
            double2 F[9];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int ij = 3 * i + j, ji = 3 * j + i;
                    const double zr = (l1.e[ij].x + l2.e[ij].x + l3.e[ij].x + l4.e[ij].x) -
                                      (l1.e[ji].x + l2.e[ji].x + l3.e[ji].x + l4.e[ji].x);
                    const double zi = (l1.e[ij].y + l2.e[ij].y + l3.e[ij].y + l4.e[ij].y) +
                                      (l1.e[ji].y + l2.e[ji].y + l3.e[ji].y + l4.e[ji].y);
                    F[ij] = make_double2(zi * 0.125, -zr * 0.125);
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const double2 w = sig.sb[p][h][a][b];
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) {
                                const double2 f = F[3 * i + j];
                                double2 &o = blk[h][3 * a + i][3 * b + j];
                                o.x += w.x * f.x - w.y * f.y;
                                o.y += w.x * f.y + w.y * f.x;
                            }
                    }
        }
    }
    double *o64 = C64 + (size_t)s * CLOVER_REALS;
    float *o32 = C32 + (size_t)s * CLOVER_REALS;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double v[36];
        for (int i = 0; i < 6; ++i) v[i] = blk[h][i][i].x;
        int q = 6;
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j, q += 2) {
                v[q] = blk[h][i][j].x;
                v[q + 1] = blk[h][i][j].y;
            }
        for (int k = 0; k < 36; ++k) {
            o64[36 * h + k] = v[k];
            o32[36 * h + k] = (float)v[k];
        }
    }
}

// (a + C)^-1 per site and chirality, one thread each: the packed 6 x 6 block
// plus a on the diagonal, inverted by Gauss-Jordan elimination with partial
// pivoting in FP64, written back in the packed form (the inverse of a
// Hermitian matrix is Hermitian: its diagonal's real part and the elements
// above it are kept); FP32 copy rounded from it.
__global__ __launch_bounds__(128) void k_clover_inverse(const double *__restrict__ C, double a,
                                                        int nblk, double *__restrict__ Ci64,
                                                        float *__restrict__ Ci32) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk) return;
    const double *A = C + (size_t)t * 36;
    double2 M[6][12];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 12; ++j) M[i][j] = make_double2(0.0, 0.0);
    for (int i = 0; i < 6; ++i) {
        M[i][i] = make_double2(a + A[i], 0.0);
        M[i][6 + i] = make_double2(1.0, 0.0);
    }
    int q = 6;
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j, q += 2) {
            M[i][j] = make_double2(A[q], A[q + 1]);
            M[j][i] = make_double2(A[q], -A[q + 1]);
        }
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        double best = M[col][col].x * M[col][col].x + M[col][col].y * M[col][col].y;
        for (int i = col + 1; i < 6; ++i) {
            const double m = M[i][col].x * M[i][col].x + M[i][col].y * M[i][col].y;
            if (m > best) {
                best = m;
                piv = i;
            }
        }
        if (piv != col)
            for (int j = 0; j < 12; ++j) {
                const double2 tmp = M[col][j];
                M[col][j] = M[piv][j];
                M[piv][j] = tmp;
            }
        // row col /= pivot
        const double2 p = M[col][col];
        const double inv = 1.0 / (p.x * p.x + p.y * p.y);
        const double2 rp = make_double2(p.x * inv, -p.y * inv);
        for (int j = 0; j < 12; ++j) {
            const double2 v = M[col][j];
            M[col][j] = make_double2(v.x * rp.x - v.y * rp.y, v.x * rp.y + v.y * rp.x);
        }
        for (int i = 0; i < 6; ++i) {
            if (i == col) continue;
            const double2 f = M[i][col];
            for (int j = 0; j < 12; ++j) {
                const double2 v = M[col][j];
                M[i][j].x -= f.x * v.x - f.y * v.y;
                M[i][j].y -= f.x * v.y + f.y * v.x;
            }
        }
    }
    double *o64 = Ci64 + (size_t)t * 36;
    float *o32 = Ci32 + (size_t)t * 36;
    for (int i = 0; i < 6; ++i) {
        o64[i] = M[i][6 + i].x;
        o32[i] = (float)M[i][6 + i].x;
    }
    q = 6;
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j, q += 2) {
            o64[q] = M[i][6 + j].x;
            o64[q + 1] = M[i][6 + j].y;
            o32[q] = (float)M[i][6 + j].x;
            o32[q + 1] = (float)M[i][6 + j].y;
        }
}

int ensure_clover_inverse(wdt_gauge_s *g, double a, hipStream_t stream) {
    if (!g->C64) return set_error(WDT_EINVAL, "clover inverse blocks without a clover term");
    if (g->Ci64 && g->ci_a == a) return WDT_OK;
    const size_t n = (size_t)g->lat.V * CLOVER_REALS;
    if (!g->Ci64) {
        double *c64 = nullptr;
        float *c32 = nullptr;
        const hipError_t e1 = hipMalloc(&c64, n * sizeof(double));
        const hipError_t e2 = e1 == hipSuccess ? hipMalloc(&c32, n * sizeof(float)) : e1;
        if (e1 != hipSuccess || e2 != hipSuccess) {
            (void)hipGetLastError();
            if (c64) (void)hipFree(c64);
            return set_error(WDT_ENOMEM, "clover inverse blocks: device allocation failed");
        }
        g->Ci64 = c64;
        g->Ci32 = c32;
    }
    const int nblk = (int)(g->lat.V * 2);
    const int threads = 128;
    hipLaunchKernelGGL(k_clover_inverse, dim3((nblk + threads - 1) / threads), dim3(threads), 0,
                       stream, g->C64, a, nblk, g->Ci64, g->Ci32);
    WDT_HIP(hipGetLastError());
    g->ci_a = a;
    return WDT_OK;
}

// The DeGrand-Rossi gamma matrices (mu = x, y, z, t), in which gamma5 =
// diag(1, 1, -1, -1); the operator kernels' spin projectors use the same basis.
static void gamma_dr(int mu, double2 (&m)[4][4]) {
    for (auto &row : m)
        for (auto &e : row) e = make_double2(0.0, 0.0);
    switch (mu) {
        case 0:
            m[0][3] = make_double2(0, 1);
            m[1][2] = make_double2(0, 1);
            m[2][1] = make_double2(0, -1);
            m[3][0] = make_double2(0, -1);
            break;
        case 1:
            m[0][3] = make_double2(-1, 0);
            m[1][2] = make_double2(1, 0);
            m[2][1] = make_double2(1, 0);
            m[3][0] = make_double2(-1, 0);
            break;
        case 2:
            m[0][2] = make_double2(0, 1);
            m[1][3] = make_double2(0, -1);
            m[2][0] = make_double2(0, -1);
            m[3][1] = make_double2(0, 1);
            break;
        default:
            m[0][2] = make_double2(1, 0);
            m[1][3] = make_double2(1, 0);
            m[2][0] = make_double2(1, 0);
            m[3][1] = make_double2(1, 0);
            break;
    }
}

static SigmaBlocks sigma_blocks(double csw) {
    SigmaBlocks S;
    int p = 0;
    for (int mu = 0; mu < 4; ++mu) {
        for (int nu = mu + 1; nu < 4; ++nu, ++p) {
            double2 gm[4][4], gn[4][4];
            gamma_dr(mu, gm);
            gamma_dr(nu, gn);
            for (int h = 0; h < 2; ++h)
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        const int r = 2 * h + a, q = 2 * h + b;
                        // [gamma_mu, gamma_nu]_{rq}
                        double cr = 0.0, ci = 0.0;
                        for (int k = 0; k < 4; ++k) {
                            const double2 x = gm[r][k], y = gn[k][q];
                            const double2 u = gn[r][k], v = gm[k][q];
                            cr += (x.x * y.x - x.y * y.y) - (u.x * v.x - u.y * v.y);
                            ci += (x.x * y.y + x.y * y.x) - (u.x * v.y + u.y * v.x);
                        }
                        // -(csw/2) * (i/2) * commutator
                        const double f = -0.25 * csw;
                        S.sb[p][h][a][b] = make_double2(-f * ci, f * cr);
                    }
        }
    }
    return S;
}

}  // namespace wdt

extern "C" int wdt_gauge_set_clover(wdt_gauge g, double csw) {
    using namespace wdt;
    WDT_CHECK(g != nullptr, "wdt_gauge_set_clover: null gauge handle");
    WDT_CHECK(std::isfinite(csw), "wdt_gauge_set_clover: c_sw must be finite");
    // the inverse blocks belong to the old term
    g->ci_a = std::nan("");
    if (csw == 0.0) {
        if (g->C64) (void)hipFree(g->C64);
        if (g->C32) (void)hipFree(g->C32);
        if (g->Ci64) (void)hipFree(g->Ci64);
        if (g->Ci32) (void)hipFree(g->Ci32);
        g->C64 = nullptr;
        g->C32 = nullptr;
        g->Ci64 = nullptr;
        g->Ci32 = nullptr;
        g->csw = 0.0;
        return WDT_OK;
    }
    const size_t n = (size_t)g->lat.V * CLOVER_REALS;
    if (!g->C64) {
        double *c64 = nullptr;
        float *c32 = nullptr;
        const hipError_t e1 = hipMalloc(&c64, n * sizeof(double));
        const hipError_t e2 = e1 == hipSuccess ? hipMalloc(&c32, n * sizeof(float)) : e1;
        if (e1 != hipSuccess || e2 != hipSuccess) {
            (void)hipGetLastError();
            if (c64) (void)hipFree(c64);
            return set_error(WDT_ENOMEM, "wdt_gauge_set_clover: device allocation failed");
        }
        g->C64 = c64;
        g->C32 = c32;
    }
    const Geom geo = g->lat.geom();
    const int threads = 128;
    hipLaunchKernelGGL(k_clover_build, dim3((geo.V + threads - 1) / threads), dim3(threads), 0, 0,
                       g->U64, geo, sigma_blocks(csw), g->C64, g->C32);
    WDT_HIP(hipGetLastError());
    WDT_HIP(hipDeviceSynchronize());
    g->csw = csw;
    return WDT_OK;
}

extern "C" int wdt_gauge_get_clover(wdt_gauge g, double *host_packed) {
    using namespace wdt;
    WDT_CHECK(g != nullptr && host_packed != nullptr, "wdt_gauge_get_clover: null argument");
    WDT_CHECK(g->C64 != nullptr, "wdt_gauge_get_clover: the gauge has no clover term");
    WDT_HIP(hipMemcpy(host_packed, g->C64, (size_t)g->lat.V * CLOVER_REALS * sizeof(double),
                      hipMemcpyDeviceToHost));
    return WDT_OK;
}
