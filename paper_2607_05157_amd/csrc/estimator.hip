// Noise / probing sources (Sec. 1 and Sec. 3), trace contractions (Sec. 1,
// Sec. 4), the backward force of eta^dag D^-1 eta, and the torus colouring
// search (Sec. 3, eq. coloring-formula).
#include "internal.h"

#include <algorithm>
#include <array>
#include <cstdlib>
#include <vector>

namespace wdt {

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014): word number c of the stream started
// from state 0 is mix((c + 1) * golden).
__device__ __forceinline__ uint64_t splitmix_word(uint64_t c) {
    uint64_t z = (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <class S>
__global__ __launch_bounds__(256) void k_sources(Geom g, const wdt_source_desc *__restrict__ desc,
                                                 int N, int NT, int SB, SpinorPtr<S> out) {
    using R = typename S::real;
    SITE_LOOP_BEGIN
    const wdt_source_desc d = desc[r];
    int c[4];
    c[0] = s % g.L[0];
    int q = s / g.L[0];
    c[1] = q % g.L[1];
    q /= g.L[1];
    c[2] = q % g.L[2];
    c[3] = q / g.L[2];
    bool keep = true;
    if (d.n_c > 0) {
        long long col = 0;
        for (int j = 0; j < 4; ++j) col += (long long)d.sigma[j] * c[j];
        keep = (int)(col % d.n_c) == d.colour;
    }
    if (d.t0 >= 0) keep = keep && (c[3] == d.t0);
    cplx<R> v[12];
    const uint64_t base = (d.seed << 40) + (uint64_t)s * 12ull;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const bool on = keep && (d.component < 0 || d.component == k);
        const uint64_t w = splitmix_word(base + (uint64_t)k);
        const R sign = (w >> 63) ? R(-1) : R(1);
        v[k] = {on ? sign : R(0), R(0)};
    }
    store_site<S>(out, s, r, v);
    SITE_LOOP_END
}

struct SpinMat {
    double2 m[16];
};

// Per-slice contraction partials: block (b, t) covers part of slice t.
// mode 0: conj(v) B x;  mode 1: ||x||^2.
template <int MODE>
__global__ __launch_bounds__(256) void k_contract(Geom g, SpinorPtr<F64> src, SpinorPtr<F64> sol,
                                                  int N, int NT, int SB, int chunk, SpinMat Bm,
                                                  double2 *partials) {
    __shared__ double2 red[256];
    const int tid = threadIdx.x;
    const int rl = tid % NT;
    const int ry = tid / NT;
    const int r = blockIdx.z * NT + rl;
    const bool live = (ry < SB) && (r < N);
    const int t = blockIdx.y;
    const int nsl = g.Lxyz;
    const int ngroups = (nsl + SB - 1) / SB;
    const int g0 = blockIdx.x * chunk;
    const int g1 = min(ngroups, g0 + chunk);
    double ar = 0, ai = 0;
    if (live) {
        for (int grp = g0; grp < g1; ++grp) {
            const int sl = grp * SB + ry;
            if (sl >= nsl) break;
            const int s = t * nsl + sl;
            cplx<double> x[12];
            load_site<F64>(sol, s, r, x);
            if constexpr (MODE == 1) {
#pragma unroll
                for (int k = 0; k < 12; ++k) ar += x[k].re * x[k].re + x[k].im * x[k].im;
            } else {
                cplx<double> v[12];
                load_site<F64>(src, s, r, v);
#pragma unroll
                for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        cplx<double> bx = {0, 0};
#pragma unroll
                        for (int sq = 0; sq < 4; ++sq) {
                            const double2 b = Bm.m[sp * 4 + sq];
                            bx = cfma(bx, cplx<double>{b.x, b.y}, x[3 * sq + cc]);
                        }
                        const cplx<double> p = cconjmul(v[3 * sp + cc], bx);
                        ar += p.re;
                        ai += p.im;
                    }
            }
        }
    }
    red[tid] = make_double2(ar, ai);
    __syncthreads();
    if (ry == 0 && r < N) {
        double2 a = red[rl];
        for (int y = 1; y < SB; ++y) {
            a.x += red[y * NT + rl].x;
            a.y += red[y * NT + rl].y;
        }
        partials[((size_t)t * gridDim.x + blockIdx.x) * N + r] = a;
    }
}

// out[r][t] = sum_b partials[t][b][r]; one thread per (r, t), fixed order.
__global__ void k_contract_reduce(const double2 *__restrict__ partials, int nb, int N, int Lt,
                                  double2 *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * Lt) return;
    const int r = i / Lt, t = i % Lt;
    double2 a = make_double2(0, 0);
    for (int b = 0; b < nb; ++b) {
        const double2 p = partials[((size_t)t * nb + b) * N + r];
        a.x += p.x;
        a.y += p.y;
    }
    out[i] = a;
}

// grad_U[x][mu] = sum_r g_r conj(A_r) + conj(g_r) B_r   (see wdt.h)
template <int MU>
__device__ __forceinline__ void force_site(const Geom &g, SpinorPtr<F64> xs, SpinorPtr<F64> ys,
                                           const double2 *__restrict__ gout, int N, int s,
                                           const SiteNbr &nb, double2 *__restrict__ grad) {
    const int f = nb.fwd[MU];
    const double phi = (MU == 3 && nb.fwd_wrap_t && g.bc_t < 0) ? -1.0 : 1.0;
    cplx<double> acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = {0, 0};
    for (int r = 0; r < N; ++r) {
        cplx<double> yx[12], xf[12], xx[12], yf[12];
        load_site<F64>(ys, s, r, yx);
        load_site<F64>(xs, f, r, xf);
        load_site<F64>(xs, s, r, xx);
        load_site<F64>(ys, f, r, yf);
        // (1 - gamma_mu) x(x+mu) and (1 + gamma_mu) x(x) as full spinors
        cplx<double> hm[6], hp[6], pm[12], pp[12];
        project<MU, -1>(xf, hm);
        project<MU, +1>(xx, hp);
#pragma unroll
        for (int k = 0; k < 12; ++k) pm[k] = pp[k] = {0, 0};
        reconstruct_add<MU, -1>(pm, hm);
        reconstruct_add<MU, +1>(pp, hp);
        const cplx<double> gr = {gout[r].x, gout[r].y};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                cplx<double> A = {0, 0}, Bv = {0, 0};
#pragma unroll
                for (int sp = 0; sp < 4; ++sp) {
                    A = cfmaconj(A, yx[3 * sp + a], pm[3 * sp + b]);
                    Bv = cfmaconj(Bv, yf[3 * sp + b], pp[3 * sp + a]);
                }
                A = cscale(A, 0.5 * phi);
                Bv = cscale(Bv, 0.5 * phi);
                // g conj(A) + conj(g) B
                const cplx<double> Ac = {A.re, -A.im};
                acc[3 * a + b] = cadd(acc[3 * a + b], cadd(cmul(gr, Ac), cconjmul(gr, Bv)));
            }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k)
        grad[((size_t)s * 4 + MU) * 9 + k] = make_double2(acc[k].re, acc[k].im);
}

__global__ __launch_bounds__(256) void k_force(Geom g, SpinorPtr<F64> xs, SpinorPtr<F64> ys,
                                               const double2 *__restrict__ gout, int N,
                                               double2 *__restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V * 4) return;
    const int s = i >> 2, mu = i & 3;
    const SiteNbr nb = neighbours(g, s);
    switch (mu) {
        case 0: force_site<0>(g, xs, ys, gout, N, s, nb, grad); break;
        case 1: force_site<1>(g, xs, ys, gout, N, s, nb, grad); break;
        case 2: force_site<2>(g, xs, ys, gout, N, s, nb, grad); break;
        default: force_site<3>(g, xs, ys, gout, N, s, nb, grad); break;
    }
}

// Slice-wise contraction into host_out (complex [N][Lt]); synchronises.
static int contract(const wdt_lattice_s *lat, const void *src, const void *sol, int N,
                    const double *B, int mode, double2 *host_out, hipStream_t stream) {
    const Geom g = lat->geom();
    const int Lt = g.L[3];
    const Shape sh = site_shape(*lat, N, WDT_FP64);
    const int NT = sh.NT;
    // blocks per slice and site groups per block for the slice-wise sums
    const int ngs = (g.Lxyz + sh.SB - 1) / sh.SB;
    const int nb = std::max(1, std::min(ngs, 2048 / std::max(1, Lt)));
    const int chunk = (ngs + nb - 1) / nb;
    SpinMat Bm;
    for (int i = 0; i < 16; ++i)
        Bm.m[i] = B ? make_double2(B[2 * i], B[2 * i + 1])
                    : make_double2((i % 5 == 0) ? 1.0 : 0.0, 0.0);
    const size_t pbytes = (size_t)Lt * nb * N * sizeof(double2);
    const size_t obytes = (size_t)N * Lt * sizeof(double2);
    AsyncScratch scratch(stream);
    if (!scratch.alloc(pbytes + obytes))
        return set_error(WDT_ENOMEM, "contract: scratch allocation failed");
    double2 *buf = (double2 *)scratch.p;
    const dim3 grid(nb, Lt, sh.tiles);
    SpinorPtr<F64> ps = make_spinor<F64>(const_cast<void *>(src), g.V, N);
    SpinorPtr<F64> px = make_spinor<F64>(const_cast<void *>(sol), g.V, N);
    if (mode == WDT_CONTRACT_DOT)
        hipLaunchKernelGGL(k_contract<0>, grid, dim3(sh.threads), 0, stream, g, ps, px, N, NT,
                           sh.SB, chunk, Bm, buf);
    else
        hipLaunchKernelGGL(k_contract<1>, grid, dim3(sh.threads), 0, stream, g, ps, px, N, NT,
                           sh.SB, chunk, Bm, buf);
    double2 *outd = (double2 *)((char *)buf + pbytes);
    hipLaunchKernelGGL(k_contract_reduce, dim3((N * Lt + 255) / 256), dim3(256), 0, stream, buf,
                       nb, N, Lt, outd);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host_out, outd, obytes, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return set_error(WDT_EHIP, "contract: %s", hipGetErrorString(e));
    return WDT_OK;
}

// ---------------------------------------------------------------------------
// Torus colouring (host).  Colour differences that must not vanish mod n_c,
// grouped by the last coordinate they involve so that a sigma prefix can be
// rejected as soon as it is fixed.

namespace {

struct Forbidden {
    int nD;
    std::vector<std::vector<std::array<int, 4>>> by_last;  // [level] -> difference vectors
};

int fdiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// Enumerate displacement vectors delta with 0 < |delta|_1 <= d that reach a
// different site, and for each the coordinate differences a_j =
// delta_j - L_j * w_j over both wrap counts a start coordinate can produce.
void collect(const int *L, int nD, int d, int j, std::array<int, 4> &delta, int used,
             Forbidden &F) {
    if (j == nD) {
        bool same = true;
        int last = -1;
        for (int i = 0; i < nD; ++i) {
            if (((delta[i] % L[i]) + L[i]) % L[i] != 0) same = false;
            if (delta[i] != 0) last = i;
        }
        if (used == 0 || same) return;
        // expand wrap choices
        std::vector<std::array<int, 4>> vs(1, std::array<int, 4>{0, 0, 0, 0});
        for (int i = 0; i < nD; ++i) {
            const int w0 = fdiv(delta[i], L[i]);
            const int w1 = fdiv(delta[i] + L[i] - 1, L[i]);
            std::vector<std::array<int, 4>> nx;
            for (auto v : vs) {
                v[i] = delta[i] - L[i] * w0;
                nx.push_back(v);
                if (w1 != w0) {
                    v[i] = delta[i] - L[i] * w1;
                    nx.push_back(v);
                }
            }
            vs.swap(nx);
        }
        for (auto &v : vs) {
            int lv = 0;
            for (int i = 0; i < nD; ++i)
                if (v[i] != 0) lv = i;
            (void)last;
            F.by_last[lv].push_back(v);
        }
        return;
    }
    for (int a = -(d - used); a <= d - used; ++a) {
        delta[j] = a;
        collect(L, nD, d, j + 1, delta, used + std::abs(a), F);
    }
    delta[j] = 0;
}

Forbidden build(const int *L, int nD, int d) {
    Forbidden F;
    F.nD = nD;
    F.by_last.assign(nD, {});
    std::array<int, 4> delta{0, 0, 0, 0};
    collect(L, nD, d, 0, delta, 0, F);
    return F;
}

bool level_ok(const Forbidden &F, const int *sig, int level, int nc) {
    for (const auto &v : F.by_last[level]) {
        long long s = 0;
        for (int i = 0; i <= level; ++i) s += (long long)sig[i] * v[i];
        if (((s % nc) + nc) % nc == 0) return false;
    }
    return true;
}

bool assign(const Forbidden &F, int *sig, int level, int nc) {
    for (int v = 0; v < nc; ++v) {
        sig[level] = v;
        if (!level_ok(F, sig, level, nc)) continue;
        if (level + 1 == F.nD || assign(F, sig, level + 1, nc)) return true;
    }
    return false;
}

}  // namespace

}  // namespace wdt

using namespace wdt;

extern "C" {

int wdt_colouring_search(const int32_t *dims, int32_t nD, int32_t d, int32_t max_nc,
                         int32_t *n_c, int32_t *sigma) {
    WDT_CHECK(dims && n_c && sigma, "wdt_colouring_search: null argument");
    WDT_CHECK(nD >= 1 && nD <= 4, "wdt_colouring_search: nD must be 1..4");
    WDT_CHECK(d >= 1, "wdt_colouring_search: d must be >= 1");
    int L[4];
    for (int i = 0; i < nD; ++i) {
        WDT_CHECK(dims[i] >= 2, "wdt_colouring_search: extent < 2");
        L[i] = dims[i];
    }
    const Forbidden F = build(L, nD, d);
    int sig[4] = {0, 0, 0, 0};
    for (int nc = 2; nc <= max_nc; ++nc) {
        if (assign(F, sig, 0, nc)) {
            *n_c = nc;
            for (int i = 0; i < nD; ++i) sigma[i] = sig[i];
            return WDT_OK;
        }
    }
    return set_error(WDT_ESEARCH, "no torus colouring at distance %d with n_c <= %d", d, max_nc);
}

int wdt_colouring_check(const int32_t *dims, int32_t nD, int32_t d, int32_t n_c,
                        const int32_t *sigma) {
    WDT_CHECK(dims && sigma, "wdt_colouring_check: null argument");
    WDT_CHECK(nD >= 1 && nD <= 4 && d >= 1 && n_c >= 1, "wdt_colouring_check: bad argument");
    int L[4], sig[4] = {0, 0, 0, 0};
    for (int i = 0; i < nD; ++i) {
        L[i] = dims[i];
        sig[i] = sigma[i];
    }
    const Forbidden F = build(L, nD, d);
    for (int lv = 0; lv < nD; ++lv)
        if (!level_ok(F, sig, lv, n_c)) return 1;
    return WDT_OK;
}

int wdt_sources(wdt_lattice lat, const wdt_source_desc *desc, int32_t n_rhs, void *dev_out,
                int32_t prec, void *stream) {
    WDT_CHECK(lat && desc && dev_out && n_rhs >= 1, "wdt_sources: bad argument");
    WDT_CHECK(prec >= WDT_FP64 && prec <= WDT_BF16, "wdt_sources: bad precision");
    for (int r = 0; r < n_rhs; ++r) {
        WDT_CHECK(desc[r].seed < (1ull << 24), "wdt_sources: seed %llu must be < 2^24",
                  (unsigned long long)desc[r].seed);
        if (desc[r].n_c > 0)
            WDT_CHECK(desc[r].colour >= 0 && desc[r].colour < desc[r].n_c,
                      "wdt_sources: colour out of range");
        WDT_CHECK(desc[r].component < 12, "wdt_sources: component must be < 12");
        WDT_CHECK(desc[r].t0 < lat->dims[3], "wdt_sources: t0 out of range");
    }
    const hipStream_t st = (hipStream_t)stream;
    AsyncScratch scratch(st);
    if (!scratch.alloc(sizeof(wdt_source_desc) * n_rhs))
        return set_error(WDT_ENOMEM, "wdt_sources: scratch allocation failed");
    wdt_source_desc *dd = (wdt_source_desc *)scratch.p;
    WDT_HIP(hipMemcpyAsync(dd, desc, sizeof(wdt_source_desc) * n_rhs, hipMemcpyHostToDevice, st));
    const Shape sh = site_shape(*lat, n_rhs, prec);
    const Geom g = shaped_geom(*lat, sh);
    const int NT = sh.NT;
    const dim3 grid(sh.G, sh.tiles);
    switch (prec) {
        case WDT_FP64:
            hipLaunchKernelGGL(k_sources<F64>, grid, dim3(sh.threads), 0, st, g, dd, n_rhs, NT,
                               sh.SB, make_spinor<F64>(dev_out, g.V, n_rhs));
            break;
        case WDT_FP32:
            hipLaunchKernelGGL(k_sources<F32>, grid, dim3(sh.threads), 0, st, g, dd, n_rhs, NT,
                               sh.SB, make_spinor<F32>(dev_out, g.V, n_rhs));
            break;
        case WDT_BF16:
            hipLaunchKernelGGL(k_sources<B16>, grid, dim3(sh.threads), 0, st, g, dd, n_rhs, NT,
                               sh.SB, make_spinor<B16>(dev_out, g.V, n_rhs));
            break;
        default:
            hipLaunchKernelGGL(k_sources<F16>, grid, dim3(sh.threads), 0, st, g, dd, n_rhs, NT,
                               sh.SB, make_spinor<F16>(dev_out, g.V, n_rhs));
            break;
    }
    WDT_HIP(hipGetLastError());
    return WDT_OK;
}

int wdt_contract(wdt_lattice lat, const void *dev_src, const void *dev_sol, int32_t n_rhs,
                 const double *spin_B, int32_t mode, double *host_out, void *stream) {
    WDT_CHECK(lat && dev_sol && host_out && n_rhs >= 1, "wdt_contract: bad argument");
    WDT_CHECK(mode == WDT_CONTRACT_DOT || mode == WDT_CONTRACT_NORM2, "wdt_contract: bad mode");
    WDT_CHECK(mode == WDT_CONTRACT_NORM2 || dev_src != nullptr, "wdt_contract: null source");
    const int Lt = lat->dims[3];
    if (mode == WDT_CONTRACT_DOT)
        return contract(lat, dev_src, dev_sol, n_rhs, spin_B, mode, (double2 *)host_out,
                        (hipStream_t)stream);
    std::vector<double2> tmp((size_t)n_rhs * Lt);
    WDT_TRY(contract(lat, dev_sol, dev_sol, n_rhs, nullptr, mode, tmp.data(), (hipStream_t)stream));
    for (size_t i = 0; i < tmp.size(); ++i) host_out[i] = tmp[i].x;
    return WDT_OK;
}

int wdt_force(wdt_gauge g, const void *dev_x, const void *dev_y, int32_t n_rhs,
              const double *grad_out, void *dev_grad_U, double *grad_m0, void *stream) {
    WDT_CHECK(g && dev_x && dev_y && grad_out && dev_grad_U && grad_m0 && n_rhs >= 1,
              "wdt_force: bad argument");
    WDT_CHECK(g->C64 == nullptr,
              "wdt_force: the derivative of the clover term is not implemented");
    const hipStream_t st = (hipStream_t)stream;
    const Geom geo = g->lat.geom();
    AsyncScratch scratch(st);
    if (!scratch.alloc(sizeof(double2) * n_rhs))
        return set_error(WDT_ENOMEM, "wdt_force: scratch allocation failed");
    double2 *dg = (double2 *)scratch.p;
    WDT_HIP(hipMemcpyAsync(dg, grad_out, sizeof(double2) * n_rhs, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_force, dim3((geo.V * 4 + 255) / 256), dim3(256), 0, st, geo,
                       make_spinor<F64>(const_cast<void *>(dev_x), geo.V, n_rhs),
                       make_spinor<F64>(const_cast<void *>(dev_y), geo.V, n_rhs), dg, n_rhs,
                       (double2 *)dev_grad_U);
    WDT_HIP(hipGetLastError());
    // df/dm0 = -y^dag x per RHS: the slice contraction of (y, x) summed over t
    const int Lt = geo.L[3];
    std::vector<double2> yx((size_t)n_rhs * Lt);
    WDT_TRY(contract(&g->lat, dev_y, dev_x, n_rhs, nullptr, WDT_CONTRACT_DOT, yx.data(), st));
    double acc = 0.0;
    for (int r = 0; r < n_rhs; ++r) {
        double dr = 0, di = 0;
        for (int t = 0; t < Lt; ++t) {
            dr -= yx[(size_t)r * Lt + t].x;
            di -= yx[(size_t)r * Lt + t].y;
        }
        // Re(g conj(df/dm0))
        acc += grad_out[2 * r] * dr + grad_out[2 * r + 1] * di;
    }
    *grad_m0 = acc;
    return WDT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// out = gamma5 in (DeGrand-Rossi gamma5 = diag(1, 1, -1, -1) on spins), FP64
// batches; with D^dag = gamma5 D gamma5 (Sec. 2: Q = Gamma5 D is Hermitian)
// it turns a solve with D into one with D^dag: D^-dag eta = g5 D^-1 g5 eta.
namespace wdt {
__global__ void k_gamma5(const double2 *__restrict__ in, double2 *__restrict__ out, int64_t V,
                         int N) {
    const int64_t n = V * 12 * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)((i / N) % 12);
        const double2 v = in[i];
        out[i] = (k >= 6) ? make_double2(-v.x, -v.y) : v;
    }
}
}  // namespace wdt

extern "C" int wdt_gamma5(wdt_lattice lat, const void *dev_in, void *dev_out, int32_t n_rhs,
                          void *stream) {
    using namespace wdt;
    WDT_CHECK(lat && dev_in && dev_out && n_rhs >= 1, "wdt_gamma5: bad argument");
    hipLaunchKernelGGL(k_gamma5, dim3(2048), dim3(256), 0, (hipStream_t)stream,
                       (const double2 *)dev_in, (double2 *)dev_out, lat->V, n_rhs);
    WDT_HIP(hipGetLastError());
    return WDT_OK;
}
