/*
 * wdt.h: C interface of libwdt, a stochastic trace estimator for the
 * Wilson-Dirac operator on AMD Instinct MI355X (gfx950).
 *
 * It computes the pieces of the Hutchinson / probing / dilution estimate of
 * tr[B(t) D^-1(t,t')] (Frommer, Jimenez-Merchan, Lang, Papace,
 * Ramirez-Hidalgo, "Variance reduction with probing and Multilevel Monte Carlo
 * in Lattice QCD", Sec. 1 and Sec. 3): it creates the lattice and the gauge
 * field, generates noise and probing vectors, solves D x = eta for a batch of
 * right-hand sides, and contracts the solutions into trace samples.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Operator.  (D psi)(x) = (4 + m0) psi(x)
 *              - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
 *                           + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ]
 *   with DeGrand-Rossi gamma matrices, mu = x, y, z, t, periodic in space and
 *   with the factor bc_t (+1 or -1) on hops across t = Lt-1 <-> 0.  The paper
 *   (Sec. 1) describes D as 12x12 spin-colour blocks on the nearest-neighbour
 *   torus; the form above is the standard Wilson operator without clover term.
 * Sites.  site = x + Lx*(y + Ly*(z + Lz*t)); each time slice is contiguous.
 * Components.  k = 3*spin + colour (12 per site).
 * Device spinor batches ("dev" pointers, device memory owned by the caller):
 *   WDT_FP64: complex double  [V][12][n_rhs], re/im interleaved (16 B each).
 *   WDT_FP32: complex float   [V][12][n_rhs] (8 B each).
 *   WDT_FP16: [V][12][n_rhs] half2 (re, im) followed, in the same buffer, by
 *             [V][n_rhs] float scales; value = half * scale.  Use
 *             wdt_spinor_bytes for the size.
 *   WDT_BF16: [V][12][n_rhs] bfloat16 pairs, one 32-bit word each (re in the
 *             low 16 bits, im in the high 16 bits), no scale; the operator
 *             computes in FP32 with FP32 links.
 *   The right-hand side index is innermost so that a site's SU(3) links are
 *   loaded once and reused across the batch.
 * Host links: double [V][4][3][3][2] = U_mu(x)[a][b] (re, im).
 * Streams.  `stream` is a hipStream_t (NULL = default stream).  Calls are
 *   asynchronous on that stream unless they return host data, in which case
 *   they synchronise the stream before returning.  wdt_solve keeps its
 *   workspace with the gauge handle: solves with one gauge on different
 *   streams must be ordered by the caller (one stream per gauge handle, or
 *   an event between them).
 * Errors.  Every function returns an int: 0 success, > 0 a warning with
 *   results written, < 0 an error (no output written or output undefined).
 *   wdt_error_string maps a code to text; wdt_last_error_detail gives the
 *   message of the most recent failure on the calling thread.  No C++
 *   exception or abort crosses this interface.
 * Threading.  Handles may be used from one host thread at a time.
 */
#ifndef WDT_H
#define WDT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    WDT_OK = 0,
    WDT_WNOTCONVERGED = 1,  /* solve finished; some RHS missed the tolerance */
    WDT_EINVAL = -1,        /* bad argument (dims, sizes, null pointers, enums) */
    WDT_ENOMEM = -2,        /* device or host allocation failed */
    WDT_EHIP = -3,          /* a HIP runtime call failed */
    WDT_ESEARCH = -4,       /* no colouring found within max_nc */
    WDT_ENODEVICE = -5      /* no usable gfx950 device */
};

enum { WDT_FP64 = 0, WDT_FP32 = 1, WDT_FP16 = 2, WDT_BF16 = 3 };

typedef struct wdt_lattice_s *wdt_lattice;
typedef struct wdt_gauge_s *wdt_gauge;

const char *wdt_error_string(int code);
/* Copies the last error message of this thread into buf (NUL-terminated). */
int wdt_last_error_detail(char *buf, size_t len);

/* Library version and the device it was built for (e.g. "gfx950"). */
const char *wdt_version(void);

/* Selects the HIP device used by the calling thread and checks it is gfx950. */
int wdt_init(int hip_device);

/*
 * Lattice geometry (Sec. 1: sites of the 4D periodic lattice).
 * dims = {Lx, Ly, Lz, Lt}, each >= 2; V = Lx*Ly*Lz*Lt must be < 2^31 / 12.
 * bc_t = +1 (periodic) or -1 (antiperiodic) in time.
 */
int wdt_lattice_create(const int32_t dims[4], int32_t bc_t, wdt_lattice *out);
int wdt_lattice_destroy(wdt_lattice lat);
int wdt_lattice_volume(wdt_lattice lat, int64_t *volume);
/* Bytes of one device spinor batch of n_rhs vectors in precision prec. */
int64_t wdt_spinor_bytes(wdt_lattice lat, int32_t n_rhs, int32_t prec);

/*
 * Gauge field.  Copies host links (layout above) to the device and derives
 * the lower-precision copies used by FP32 / FP16 operator applications.  The
 * links are stored without the time-boundary factor.
 */
int wdt_gauge_create(wdt_lattice lat, const double *host_links, wdt_gauge *out);
int wdt_gauge_destroy(wdt_gauge g);
/* Copies the FP64 links back to the host (same layout). */
int wdt_gauge_get(wdt_gauge g, double *host_links);

/*
 * Clover (Sheikholeslami-Wohlert) term for ensembles generated with the
 * O(a)-improved Wilson action; the paper's operator (Sec. 1) is the plain
 * Wilson one, which csw = 0 gives back.  With csw != 0 every later
 * application of D on this gauge (wdt_apply_D, wdt_solve, the batched solver
 * and the estimators built on them) adds to the site's own term
 *   C(x) = -(csw / 2) sum_{mu < nu} sigma_{mu nu} F_{mu nu}(x),
 * sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu] (DeGrand-Rossi basis) and
 * F = (Q - Q^dag) / (8i), Q_{mu nu}(x) the sum of the four plaquettes of the
 * (mu, nu) plane that start and end at x in the same sense (periodic in every
 * direction; the fermion time-boundary factor is not part of these loops; F
 * keeps its colour trace).  The sign is the one with which csw = 1 cancels
 * the Wilson term's O(a) shift at tree level.  C is Hermitian and commutes
 * with gamma5, so D^dag = gamma5 D gamma5 still holds.
 *
 * wdt_gauge_set_clover builds C from the FP64 links (FP64, plus an FP32 copy
 * for the FP32 / FP16 / BF16 operators: 72 * 12 bytes per site of device
 * memory, allocated on the first call).  csw = 0 frees it.  Synchronous.
 * Even-odd preconditioned solves then use the inverse blocks (4 + m0 + C)^-1
 * on the odd sites, computed on the solve's stream at the first solve with a
 * given m0 and kept with the gauge (another 72 * 12 bytes per site); solves
 * on one gauge with different m0 must therefore not run concurrently.  The
 * batched solver takes each gauge's term as it is at every wdt_batch_solve
 * (set, changed or removed after wdt_batch_create) and solves clover systems
 * without even-odd preconditioning.  wdt_force returns WDT_EINVAL while a
 * term is set (its derivative is not implemented).
 * WDT_EINVAL for a null handle or a non-finite csw; WDT_ENOMEM when the
 * device memory cannot be allocated (the gauge keeps its previous term; its
 * inverse blocks are recomputed at the next even-odd solve).
 *
 * wdt_gauge_get_clover copies C to host_packed (host, V * 72 doubles): per
 * site the two chiral 6 x 6 blocks (spins 0-1, then 2-3; index 3 * spin +
 * colour inside a block, C being zero between them), each as its 6 real
 * diagonal elements followed by the 15 elements above the diagonal, row by
 * row, as (re, im) pairs.  WDT_EINVAL when the gauge has no clover term.
 */
int wdt_gauge_set_clover(wdt_gauge g, double csw);
int wdt_gauge_get_clover(wdt_gauge g, double *host_packed);

/*
 * Torus colouring (Sec. 3, eq. coloring-formula): c(x) = sum_j sigma_j x_j
 * mod n_c, valid at distance d when distinct sites within periodic L1
 * distance d (wrap-around included) get different colours.  Exhaustive
 * search with n_c ascending from 2 and, for each n_c, sigma in lexicographic
 * order (sigma_1 most significant); the first valid sigma is returned.
 * dims: the nD extents coloured (nD = 3: a time slice; 4: the lattice).
 * Host only.  Returns WDT_ESEARCH if no n_c <= max_nc works.
 */
int wdt_colouring_search(const int32_t *dims, int32_t nD, int32_t d, int32_t max_nc,
                         int32_t *n_c, int32_t *sigma);
/* Returns 0 if the colouring (n_c, sigma) of dims is valid at distance d,
 * 1 if two sites within distance d share a colour, < 0 on bad arguments. */
int wdt_colouring_check(const int32_t *dims, int32_t nD, int32_t d, int32_t n_c,
                        const int32_t *sigma);

/*
 * Source vectors (Sec. 1 noise, Sec. 3 eq. "probing vectors" and dilution).
 * For RHS r the source is
 *   v(x, k) = eta_seed(12*x + k) * [c(x) == colour] * [k == component]
 *             * [t(x) == t0]
 * where eta_seed(g) = +1 if the top bit of SplitMix64 word number
 * seed*2^40 + g (the (seed*2^40 + g + 1)-th output from state 0) is clear,
 * else -1.  A field < 0 disables that mask: n_c <= 0 (no probing),
 * component < 0 (no spin-colour dilution), t0 < 0 (no time dilution).
 * sigma has 4 entries (x, y, z, t); a 3D colouring sets sigma[3] = 0.
 */
typedef struct {
    uint64_t seed;
    int32_t n_c;
    int32_t colour;
    int32_t sigma[4];
    int32_t component;
    int32_t t0;
} wdt_source_desc;

/* desc: host array of n_rhs descriptors; dev_out: spinor batch in prec. */
int wdt_sources(wdt_lattice lat, const wdt_source_desc *desc, int32_t n_rhs,
                void *dev_out, int32_t prec, void *stream);

/*
 * dev_out = D dev_in (dagger = 0) or D^dag dev_in (dagger = 1) for a batch
 * of n_rhs vectors in precision prec (FP64: FP64 links and arithmetic;
 * FP32: FP32 links and arithmetic; FP16: FP16 links, FP32 arithmetic).
 * dev_in and dev_out must not overlap.
 */
int wdt_apply_D(wdt_gauge g, double m0, const void *dev_in, void *dev_out,
                int32_t n_rhs, int32_t prec, int32_t dagger, void *stream);

/*
 * Batched solve D x_r = b_r, one BiCGStab recurrence per right-hand side
 * (Sec. 1: each sample needs the solution of a linear system with D).
 * prec selects the arithmetic:
 *   WDT_FP64 - BiCGStab in FP64 throughout;
 *   WDT_FP16 / WDT_FP32 - FP64 defect correction: r = b - D x in FP64, an
 *     inner BiCGStab on D e = r in FP32 arithmetic with vectors stored in
 *     FP16 (+ per-site-per-RHS scale) or FP32, then x += e in FP64.
 * On a lattice with every extent even both iterate on the even-odd (Schur)
 * system a x_e - H_eo H_oe x_e / (4a), a = 4 + m0, H the hop sum of D, and
 * rebuild the odd sites from b and x_e (see wdt_launch_shape.even_odd).
 * Every RHS stops when its true FP64 relative residual ||b - D x|| / ||b||
 * is <= tol.  dev_b, dev_x: FP64 batches; x starts from 0 unless
 * x0_is_guess.  stats (host, may be NULL): n_rhs records.  Uses two ints of
 * host-mapped memory per gauge handle (allocated on first use).
 * Returns WDT_WNOTCONVERGED if some RHS did not reach tol in max_iter, or if
 * its true residual is not finite (an input holding inf or NaN).
 */
typedef struct {
    double tol;          /* target true relative residual, e.g. 1e-10 */
    int32_t max_iter;    /* cap on (inner) BiCGStab iterations per RHS */
    int32_t prec;        /* WDT_FP64, WDT_FP32 or WDT_FP16 */
    double inner_tol;    /* relative residual reduction per inner solve
                            (<= 0: 0.003); the last solve of a RHS stops
                            earlier if that already meets tol.  An inner
                            solve also stops after 500 iterations, or for a
                            RHS whose recurrence residual grows 1e4 times past
                            its start; the FP64 correction continues from the
                            true residual.  BF16 storage needs >= 0.05 */
    int32_t max_outer;   /* cap on defect-correction steps */
    int32_t x0_is_guess; /* 1: dev_x holds a starting guess */
    int32_t check_every; /* wdt_batch_solve: iterations between convergence
                            checks on the host.  wdt_solve checks after every
                            iteration, one iteration behind the device (the
                            iteration queued past convergence does no work),
                            and ignores it */
} wdt_solve_params;

typedef struct {
    int32_t iterations;      /* BiCGStab iterations (summed over inner solves) */
    int32_t outer;           /* defect-correction steps (0 for FP64) */
    int32_t converged;       /* 1 if the true residual met tol */
    int32_t restarts;        /* breakdown restarts */
    double true_residual;    /* final ||b - D x|| / ||b|| in FP64 */
} wdt_rhs_stats;

int wdt_solve(wdt_gauge g, double m0, const void *dev_b, void *dev_x, int32_t n_rhs,
              const wdt_solve_params *params, wdt_rhs_stats *stats, void *stream);

/*
 * Many uneven systems solved together (FP64 BiCGStab, same recurrence and
 * stopping rule as wdt_solve): system i has its own lattice and links
 * (gauges[i]), mass m0[i] and n_rhs[i] right-hand sides.  Every phase of an
 * iteration is one launch over all systems, and one iteration is replayed
 * from a captured hipGraph on a stream the batch owns (ordered after and
 * before the caller's stream).  The gauge handles must outlive the batch.
 * wdt_batch_tune times candidate block budgets and RHS tiles for `iters`
 * iterations and keeps the fastest plan (*best_ms: time per iteration).
 * wdt_batch_solve: dev_b[i], dev_x[i] are FP64 batches of system i; stats
 * (may be NULL) receives sum(n_rhs) records, systems in order.
 */
typedef struct wdt_batch_s *wdt_batch;
int wdt_batch_create(const wdt_gauge *gauges, const double *m0, const int32_t *n_rhs,
                     int32_t n_sys, wdt_batch *out);
int wdt_batch_destroy(wdt_batch b);
int wdt_batch_tune(wdt_batch b, int32_t iters, double *best_ms);
int wdt_batch_solve(wdt_batch b, void *const *dev_b, void *const *dev_x,
                    const wdt_solve_params *params, wdt_rhs_stats *stats, void *stream);
/* Plan in use: total blocks per launch, block budget per CU, largest RHS tile. */
int wdt_batch_info(wdt_batch b, int32_t *total_blocks, int32_t *blocks_per_cu, int32_t *tile_cap);

/*
 * Contractions of a source batch v and a solution batch x (FP64 batches).
 * mode WDT_CONTRACT_DOT: host_out[r][t] (complex, 2 doubles) =
 *     sum_{x in slice t} sum_{s,s',c} conj(v_r(x,s,c)) B_{s s'} x_r(x,s',c)
 *   for every t = 0..Lt-1 (the per-slice pieces of v^dag B D^-1 v, Sec. 1
 *   and the disconnected loop O(t) = tr[Gamma5 D^-1(t,t)], Sec. 4).
 *   spin_B: host 4x4 complex matrix [s][s'][2] or NULL for the identity.
 * mode WDT_CONTRACT_NORM2: host_out[r][t] (real, 1 double) =
 *     sum_{x in slice t} ||x_r(x)||^2 (the connected correlator estimator,
 *     ||D^-1(t, t0)||_F^2 for time-diluted sources on t0, Sec. 4).
 * The sums are accumulated in FP64 in a fixed order (bit-reproducible).
 */
enum { WDT_CONTRACT_DOT = 0, WDT_CONTRACT_NORM2 = 1 };
int wdt_contract(wdt_lattice lat, const void *dev_src, const void *dev_sol, int32_t n_rhs,
                 const double *spin_B, int32_t mode, double *host_out, void *stream);

/*
 * Backward of f_r = eta_r^dag D^-1 eta_r given x_r = D^-1 eta_r and
 * y_r = D^-dag eta_r (FP64 batches, n_rhs each), and grad_out[r] = g_r
 * (host, complex [n_rhs][2]).  Writes
 *   dev_grad_U[x][mu][a][b] (complex double, device, [V][4][3][3]) =
 *     sum_r g_r conj(A_r) + conj(g_r) B_r,
 *   A_mu(x)_ab = 1/2 phi sum conj(y(x)_{s a}) (1 - gamma_mu)_{s s'} x(x+mu)_{s' b},
 *   B_mu(x)_ab = 1/2 phi sum conj(y(x+mu)_{s b}) (1 + gamma_mu)_{s s'} x(x)_{s' a},
 * (the derivatives of f with respect to U_mu(x)_ab and its conjugate, phi the
 * time-boundary factor of the hop; torch's complex-gradient convention) and
 *   *grad_m0 = sum_r Re(g_r conj(-y_r^dag x_r)).
 * Synchronises the stream (grad_m0 is a host value).
 */
int wdt_force(wdt_gauge g, const void *dev_x, const void *dev_y, int32_t n_rhs,
              const double *grad_out, void *dev_grad_U, double *grad_m0, void *stream);

/*
 * dev_out = gamma5 dev_in for an FP64 batch (gamma5 = diag(1, 1, -1, -1) on the
 * spin index).  With the Hermiticity of Gamma5 D (Sec. 2) this gives the
 * adjoint solution D^-dag eta = gamma5 D^-1 (gamma5 eta) from an ordinary
 * solve.  dev_in may equal dev_out.
 */
int wdt_gamma5(wdt_lattice lat, const void *dev_in, void *dev_out, int32_t n_rhs, void *stream);

/*
 * Block products for the low-mode subspace of the deflated estimator (Sec. 2,
 * eq. defl-split: the orthogonal projector V_k V_k^dag onto k low modes of
 * Q = Gamma5 D; the modes are found by subspace iteration with block solves
 * and Rayleigh-Ritz, which need the same two products).  FP64 batches in the
 * batch layout [V][12][n] (device); nx, ny in 1..64.
 *
 * wdt_block_dot: host_out[i*ny + j] (complex double, host, nx*ny entries) =
 *   sum over sites and spin-colour of conj(X_i) Y_j.  Sums in a fixed order
 *   (bit-reproducible).  Synchronises the stream.
 * wdt_block_combine: Y_j = beta Y_j + sum_i X_i W[i*ny + j] (W host, complex
 *   double [nx][ny]); beta = 0 overwrites Y without reading it.  dev_x and
 *   dev_y must not overlap (WDT_EINVAL).  Synchronises the stream.
 * Both use stream-ordered scratch (block_dot at most about 4.2M complex
 * doubles, 67 MB; block_combine nx * ny).
 */
int wdt_block_dot(wdt_lattice lat, const void *dev_x, int32_t nx, const void *dev_y, int32_t ny,
                  double *host_out, void *stream);
int wdt_block_combine(wdt_lattice lat, const void *dev_x, int32_t nx, const double *W, int32_t ny,
                      double beta, void *dev_y, void *stream);

/*
 * Layout bridge between the natural order [n_rhs][V][12] (complex double)
 * and the batch layout [V][12][n_rhs] used above (FP64 only).
 */
int wdt_pack_spinor(wdt_lattice lat, const void *dev_natural, void *dev_batch,
                    int32_t n_rhs, void *stream);
int wdt_unpack_spinor(wdt_lattice lat, const void *dev_batch, void *dev_natural,
                      int32_t n_rhs, void *stream);

/*
 * Kernel timing for benchmarks and tuning.  While enabled, every operator and
 * vector kernel the library launches is bracketed by HIP events on its own
 * stream; wdt_profile_read waits for the recorded events and returns, per
 * kernel class, the number of launches, the summed device time and the summed
 * algorithmic bytes (each input read once, each output written once, links
 * once per launch).  wdt_profile_enable(1) clears the counters; (0) stops
 * recording.  Host-side bookkeeping only; adds one event pair per launch.
 */
typedef struct {
    char name[48];
    int64_t calls;
    double ms;
    double bytes;
} wdt_prof_entry;

/*
 * Launch-shape overrides for the tuner (all kernels over (site, rhs)).
 * Zero in a field keeps the automatic choice, except where -1 is stated.
 *  rhs_tile         right-hand sides per tile (the batch is swept tile by tile)
 *  sites_per_block  sites (or columns, when marching) a block handles per step
 *  max_blocks       blocks per tile
 *  z_slab           thickness (a divisor of Lz) of the z-slabs of the site
 *                   order (t-neighbours are Lx*Ly*z_slab sites apart in it)
 *  serial_tiles     1: each operator block sweeps the RHS tiles one after
 *                   the other; 0: tiles side by side in the grid; -1 automatic
 *  t_chunk          > 0: the operator marches along t through columns in
 *                   chunks of t_chunk slices (a divisor of Lt); 0: site
 *                   sweep; -1 automatic
 *  brick            site sweep in brick order: bricks of brick[0] x brick[1]
 *                   x brick[2] columns (divisors of Lx, Ly, Lz) visited one
 *                   after the other, each through all of t; {0,0,0} automatic,
 *                   {-1,-1,-1} off
 *  wave_per_site    1: the operator gives each site one wavefront (its 64
 *                   lanes are the RHS; batches of 48 or 64); 0 off; -1 automatic
 *  even_odd         solvers: 1 or -1 (automatic) precondition even-odd on
 *                   lattices with every extent even, 0 solve the full system
 * Invalid combinations for a lattice fall back to the automatic choice.
 * Process-wide; not thread-safe.
 */
typedef struct {
    int32_t rhs_tile, sites_per_block, max_blocks, z_slab, serial_tiles, t_chunk;
    int32_t brick[3];
    int32_t wave_per_site;
    int32_t even_odd;
} wdt_launch_shape;
int wdt_set_launch_shape(const wdt_launch_shape *shape);

int wdt_profile_enable(int on);
/* Fills up to max entries; *n receives the number of kernel classes. */
int wdt_profile_read(wdt_prof_entry *out, int32_t max, int32_t *n);

#ifdef __cplusplus
}
#endif
#endif /* WDT_H */
