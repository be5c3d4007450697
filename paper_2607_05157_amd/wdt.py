"""ctypes binding of libwdt (include/wdt.h).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  PyTorch supplies
device memory (tensors' data_ptr) and the current HIP stream.

Raises if the built library is missing: there is no CPU fallback.
"""
import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# WDT_LIB selects another build of the library (A/B timing of build options)
LIB_PATH = os.environ.get("WDT_LIB") or os.path.join(HERE, "libwdt.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "wdt.h")

OK, WNOTCONVERGED, EINVAL, ENOMEM, EHIP, ESEARCH, ENODEVICE = 0, 1, -1, -2, -3, -4, -5
FP64, FP32, FP16, BF16 = 0, 1, 2, 3
CONTRACT_DOT, CONTRACT_NORM2 = 0, 1
PREC = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16, "mixed_fp16": FP16,
        "mixed_fp32": FP32, "mixed_bf16": BF16}


class SourceDesc(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_c", ctypes.c_int32), ("colour", ctypes.c_int32),
                ("sigma", ctypes.c_int32 * 4), ("component", ctypes.c_int32),
                ("t0", ctypes.c_int32)]


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("x0_is_guess", ctypes.c_int32), ("check_every", ctypes.c_int32)]


class RhsStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("true_residual", ctypes.c_double)]


class WdtError(RuntimeError):
    def __init__(self, code, fn, detail):
        super().__init__(f"{fn} failed with {code}: {detail}")
        self.code = code


_lib = None


def lib():
    """The loaded libwdt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with "
                               "`python -m paper_2607_05157_amd.build` (no CPU fallback exists)")
        # PyTorch first: the library's HIP runtime dependency (same soname)
        # then resolves to the runtime torch has loaded, so the process has
        # one runtime; loaded the other way round, two runtimes coexist and
        # torch sees no GPU.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "wdt_error_string": (ctypes.c_char_p, [ctypes.c_int]),
            "wdt_last_error_detail": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t]),
            "wdt_version": (ctypes.c_char_p, []),
            "wdt_init": (ctypes.c_int, [ctypes.c_int]),
            "wdt_lattice_create": (ctypes.c_int, [P(i32), i32, P(vp)]),
            "wdt_lattice_destroy": (ctypes.c_int, [vp]),
            "wdt_lattice_volume": (ctypes.c_int, [vp, P(i64)]),
            "wdt_spinor_bytes": (i64, [vp, i32, i32]),
            "wdt_gauge_create": (ctypes.c_int, [vp, P(dbl), P(vp)]),
            "wdt_gauge_destroy": (ctypes.c_int, [vp]),
            "wdt_gauge_get": (ctypes.c_int, [vp, P(dbl)]),
            "wdt_gauge_set_clover": (ctypes.c_int, [vp, dbl]),
            "wdt_gauge_get_clover": (ctypes.c_int, [vp, P(dbl)]),
            "wdt_colouring_search": (ctypes.c_int, [P(i32), i32, i32, i32, P(i32), P(i32)]),
            "wdt_colouring_check": (ctypes.c_int, [P(i32), i32, i32, i32, P(i32)]),
            "wdt_sources": (ctypes.c_int, [vp, P(SourceDesc), i32, vp, i32, vp]),
            "wdt_apply_D": (ctypes.c_int, [vp, dbl, vp, vp, i32, i32, i32, vp]),
            "wdt_solve": (ctypes.c_int, [vp, dbl, vp, vp, i32, P(SolveParams), P(RhsStats), vp]),
            "wdt_contract": (ctypes.c_int, [vp, vp, vp, i32, P(dbl), i32, P(dbl), vp]),
            "wdt_force": (ctypes.c_int, [vp, vp, vp, i32, P(dbl), vp, P(dbl), vp]),
            "wdt_pack_spinor": (ctypes.c_int, [vp, vp, vp, i32, vp]),
            "wdt_gamma5": (ctypes.c_int, [vp, vp, vp, i32, vp]),
            "wdt_block_dot": (ctypes.c_int, [vp, vp, i32, vp, i32, P(dbl), vp]),
            "wdt_block_combine": (ctypes.c_int, [vp, vp, i32, P(dbl), i32, dbl, vp, vp]),
            "wdt_unpack_spinor": (ctypes.c_int, [vp, vp, vp, i32, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions():
    """Names of the functions include/wdt.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wdt_[A-Za-z0-9_]+)\s*\(", txt)))


def _detail():
    buf = ctypes.create_string_buffer(512)
    lib().wdt_last_error_detail(buf, 512)
    return buf.value.decode()


def check(rc, fn, allow=(OK,)):
    if rc in allow:
        return rc
    raise WdtError(rc, fn, _detail())


def _i32(arr):
    a = (ctypes.c_int32 * len(arr))(*[int(v) for v in arr])
    return a


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def init(device=0):
    check(lib().wdt_init(device), "wdt_init")


def colouring_search(dims, d, max_nc=4096):
    nc = ctypes.c_int32(0)
    sig = (ctypes.c_int32 * 4)()
    check(lib().wdt_colouring_search(_i32(dims), len(dims), d, max_nc, ctypes.byref(nc), sig),
          "wdt_colouring_search")
    return nc.value, tuple(sig[i] for i in range(len(dims)))


def colouring_check(dims, d, n_c, sigma):
    rc = lib().wdt_colouring_check(_i32(dims), len(dims), d, n_c, _i32(list(sigma) + [0] * 4))
    if rc < 0:
        check(rc, "wdt_colouring_check")
    return rc == 0


class Lattice:
    """Lattice geometry handle (dims = (Lx, Ly, Lz, Lt), bc_t = +-1)."""

    def __init__(self, dims, bc_t=-1):
        self.dims = tuple(int(d) for d in dims)
        self.bc_t = bc_t
        h = ctypes.c_void_p()
        check(lib().wdt_lattice_create(_i32(self.dims), bc_t, ctypes.byref(h)),
              "wdt_lattice_create")
        self.h = h
        self.V = int(np.prod(self.dims))

    def spinor_bytes(self, n_rhs, prec=FP64):
        b = lib().wdt_spinor_bytes(self.h, n_rhs, prec)
        if b < 0:
            check(int(b), "wdt_spinor_bytes")
        return int(b)

    def new_batch(self, n_rhs, prec=FP64, device="cuda"):
        """Device spinor batch in the library layout ([V, 12, N] complex128 for FP64)."""
        import torch
        if prec == FP64:
            return torch.zeros((self.V, 12, n_rhs), dtype=torch.complex128, device=device)
        return torch.zeros(self.spinor_bytes(n_rhs, prec), dtype=torch.uint8, device=device)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.wdt_lattice_destroy(self.h)
            self.h = None


class Gauge:
    """Gauge field handle.  links: complex128 array [V, 4, 3, 3] (host)."""

    def __init__(self, lat, links):
        self.lat = lat
        U = np.ascontiguousarray(np.asarray(links, dtype=np.complex128))
        assert U.shape == (lat.V, 4, 3, 3), U.shape
        h = ctypes.c_void_p()
        check(lib().wdt_gauge_create(lat.h, U.view(np.float64).ctypes.data_as(
            ctypes.POINTER(ctypes.c_double)), ctypes.byref(h)), "wdt_gauge_create")
        self.h = h

    def get(self):
        out = np.empty((self.lat.V, 4, 3, 3), dtype=np.complex128)
        check(lib().wdt_gauge_get(self.h, out.view(np.float64).ctypes.data_as(
            ctypes.POINTER(ctypes.c_double))), "wdt_gauge_get")
        return out

    def set_clover(self, csw):
        """Adds the clover term with coefficient csw to every later operator
        application on this gauge (csw = 0 removes it)."""
        check(lib().wdt_gauge_set_clover(self.h, float(csw)), "wdt_gauge_set_clover")

    def clover_packed(self):
        """The clover term as stored: [V, 2, 36] (per chiral block its real
        diagonal, then the elements above it row by row as re, im)."""
        out = np.empty((self.lat.V, 2, 36), dtype=np.float64)
        check(lib().wdt_gauge_get_clover(self.h, out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_double))), "wdt_gauge_get_clover")
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.wdt_gauge_destroy(self.h)
            self.h = None


def source_descs(seeds, n_c=0, colour=0, sigma=(0, 0, 0, 0), component=None, t0=-1):
    """Array of descriptors; `component` may be a list (one per seed) or an int."""
    n = len(seeds)
    arr = (SourceDesc * n)()
    for i, s in enumerate(seeds):
        arr[i].seed = int(s)
        arr[i].n_c = int(n_c)
        arr[i].colour = int(colour[i] if isinstance(colour, (list, tuple)) else colour)
        sg = list(sigma) + [0] * (4 - len(sigma))
        for j in range(4):
            arr[i].sigma[j] = int(sg[j])
        comp = component[i] if isinstance(component, (list, tuple)) else component
        arr[i].component = -1 if comp is None else int(comp)
        arr[i].t0 = int(t0[i] if isinstance(t0, (list, tuple)) else t0)
    return arr


def sources(lat, descs, out, prec=FP64, stream=None):
    check(lib().wdt_sources(lat.h, descs, len(descs), ctypes.c_void_p(out.data_ptr()), prec,
                            _stream(stream)), "wdt_sources")
    return out


def apply_D(gauge, m0, x, out, n_rhs, prec=FP64, dagger=False, stream=None):
    check(lib().wdt_apply_D(gauge.h, float(m0), ctypes.c_void_p(x.data_ptr()),
                            ctypes.c_void_p(out.data_ptr()), n_rhs, prec, int(dagger),
                            _stream(stream)), "wdt_apply_D")
    return out


def solve(gauge, m0, b, x, n_rhs, tol=1e-10, prec=FP64, max_iter=10000, inner_tol=0.003,
          max_outer=40, x0_is_guess=False, check_every=5, stream=None, allow_unconverged=False):
    p = SolveParams(tol, max_iter, prec, inner_tol, max_outer, int(x0_is_guess), check_every)
    stats = (RhsStats * n_rhs)()
    allow = (OK, WNOTCONVERGED) if allow_unconverged else (OK,)
    rc = check(lib().wdt_solve(gauge.h, float(m0), ctypes.c_void_p(b.data_ptr()),
                               ctypes.c_void_p(x.data_ptr()), n_rhs, ctypes.byref(p), stats,
                               _stream(stream)), "wdt_solve", allow)
    return rc, [dict(iterations=s.iterations, outer=s.outer, converged=s.converged,
                     restarts=s.restarts, true_residual=s.true_residual) for s in stats]


def contract(lat, src, sol, n_rhs, spin=None, mode=CONTRACT_DOT, stream=None):
    """[n_rhs, Lt] complex (DOT) or float (NORM2) per-slice sums."""
    Lt = lat.dims[3]
    if mode == CONTRACT_DOT:
        out = np.zeros((n_rhs, Lt), dtype=np.complex128)
    else:
        out = np.zeros((n_rhs, Lt), dtype=np.float64)
    B = None
    if spin is not None:
        Bm = np.ascontiguousarray(np.asarray(spin, dtype=np.complex128))
        B = Bm.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    srcp = ctypes.c_void_p(src.data_ptr()) if src is not None else None
    check(lib().wdt_contract(lat.h, srcp, ctypes.c_void_p(sol.data_ptr()), n_rhs, B, mode,
                             out.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             _stream(stream)), "wdt_contract")
    return out


def force(gauge, x, y, n_rhs, grad_out, grad_U, stream=None):
    """grad_U (device complex128 [V,4,3,3]) and returns grad_m0 (float)."""
    g = np.ascontiguousarray(np.asarray(grad_out, dtype=np.complex128).reshape(n_rhs))
    gm = ctypes.c_double(0.0)
    check(lib().wdt_force(gauge.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                          n_rhs, g.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          ctypes.c_void_p(grad_U.data_ptr()), ctypes.byref(gm), _stream(stream)),
          "wdt_force")
    return gm.value


def gamma5(lat, x, out, n_rhs, stream=None):
    """out = gamma5 x for an FP64 batch (in place allowed)."""
    check(lib().wdt_gamma5(lat.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                           n_rhs, _stream(stream)), "wdt_gamma5")
    return out


def block_dot(lat, x, nx, y, ny, stream=None):
    """[nx, ny] complex: sum over sites and spin-colour of conj(x_i) y_j (FP64
    batches; nx, ny <= 64)."""
    out = np.zeros((nx, ny), dtype=np.complex128)
    check(lib().wdt_block_dot(lat.h, ctypes.c_void_p(x.data_ptr()), nx,
                              ctypes.c_void_p(y.data_ptr()), ny,
                              out.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              _stream(stream)), "wdt_block_dot")
    return out


def block_combine(lat, x, nx, W, y, ny, beta=0.0, stream=None):
    """y_j = beta y_j + sum_i x_i W[i, j] (FP64 batches; W host [nx, ny] complex)."""
    Wc = np.ascontiguousarray(np.asarray(W, dtype=np.complex128).reshape(nx, ny))
    check(lib().wdt_block_combine(lat.h, ctypes.c_void_p(x.data_ptr()), nx,
                                  Wc.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ny, float(beta), ctypes.c_void_p(y.data_ptr()), _stream(stream)),
          "wdt_block_combine")
    return y


def pack(lat, natural, batch, n_rhs, stream=None):
    check(lib().wdt_pack_spinor(lat.h, ctypes.c_void_p(natural.data_ptr()),
                                ctypes.c_void_p(batch.data_ptr()), n_rhs, _stream(stream)),
          "wdt_pack_spinor")
    return batch


def unpack(lat, batch, natural, n_rhs, stream=None):
    check(lib().wdt_unpack_spinor(lat.h, ctypes.c_void_p(batch.data_ptr()),
                                  ctypes.c_void_p(natural.data_ptr()), n_rhs, _stream(stream)),
          "wdt_unpack_spinor")
    return natural


class ProfEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("calls", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


def profile(on=True):
    """Start (clearing counters) or stop per-launch kernel timing in the library."""
    L = lib()
    L.wdt_profile_enable.restype = ctypes.c_int
    L.wdt_profile_enable.argtypes = [ctypes.c_int]
    check(L.wdt_profile_enable(1 if on else 0), "wdt_profile_enable")


def profile_read():
    """{kernel class: dict(calls, ms, bytes, gbps)} of the launches recorded so far."""
    L = lib()
    L.wdt_profile_read.restype = ctypes.c_int
    L.wdt_profile_read.argtypes = [ctypes.POINTER(ProfEntry), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)]
    buf = (ProfEntry * 64)()
    n = ctypes.c_int32(0)
    check(L.wdt_profile_read(buf, 64, ctypes.byref(n)), "wdt_profile_read")
    out = {}
    for i in range(min(n.value, 64)):
        e = buf[i]
        out[e.name.decode()] = dict(calls=int(e.calls), ms=e.ms, bytes=e.bytes,
                                    gbps=(e.bytes / (e.ms * 1e-3) / 1e9) if e.ms > 0 else 0.0)
    return out


class LaunchShape(ctypes.Structure):
    _fields_ = [("rhs_tile", ctypes.c_int32), ("sites_per_block", ctypes.c_int32),
                ("max_blocks", ctypes.c_int32), ("z_slab", ctypes.c_int32),
                ("serial_tiles", ctypes.c_int32), ("t_chunk", ctypes.c_int32),
                ("brick", ctypes.c_int32 * 3), ("wave_per_site", ctypes.c_int32),
                ("even_odd", ctypes.c_int32)]


def set_launch_shape(rhs_tile=0, sites_per_block=0, max_blocks=0, z_slab=0, serial_tiles=-1,
                     t_chunk=-1, brick=(0, 0, 0), wave_per_site=-1, even_odd=-1):
    """Override the launch shape of the (site, rhs) kernels (see wdt_launch_shape;
    the defaults restore the automatic choice)."""
    L = lib()
    L.wdt_set_launch_shape.restype = ctypes.c_int
    L.wdt_set_launch_shape.argtypes = [ctypes.POINTER(LaunchShape)]
    s = LaunchShape(rhs_tile, sites_per_block, max_blocks, z_slab, serial_tiles, t_chunk,
                    (ctypes.c_int32 * 3)(*brick), wave_per_site, even_odd)
    check(L.wdt_set_launch_shape(ctypes.byref(s)), "wdt_set_launch_shape")


class Batch:
    """Several uneven systems solved together (wdt_batch_*).  gauges: Gauge
    handles (kept alive by this object), m0s and n_rhs per system."""

    def __init__(self, gauges, m0s, n_rhs):
        L = lib()
        vp, i32, P = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER
        L.wdt_batch_create.restype = ctypes.c_int
        L.wdt_batch_create.argtypes = [P(vp), P(ctypes.c_double), P(i32), i32, P(vp)]
        L.wdt_batch_destroy.argtypes = [vp]
        L.wdt_batch_tune.restype = ctypes.c_int
        L.wdt_batch_tune.argtypes = [vp, i32, P(ctypes.c_double)]
        L.wdt_batch_solve.restype = ctypes.c_int
        L.wdt_batch_solve.argtypes = [vp, P(vp), P(vp), P(SolveParams), P(RhsStats), vp]
        L.wdt_batch_info.restype = ctypes.c_int
        L.wdt_batch_info.argtypes = [vp, P(i32), P(i32), P(i32)]
        self.gauges = list(gauges)
        self.n_rhs = [int(n) for n in n_rhs]
        n = len(self.gauges)
        gs = (vp * n)(*[g.h.value for g in self.gauges])
        ms = (ctypes.c_double * n)(*[float(m) for m in m0s])
        ns = (i32 * n)(*self.n_rhs)
        h = vp()
        check(L.wdt_batch_create(gs, ms, ns, n, ctypes.byref(h)), "wdt_batch_create")
        self.h = h

    def tune(self, iters=3):
        ms = ctypes.c_double(0)
        check(lib().wdt_batch_tune(self.h, iters, ctypes.byref(ms)), "wdt_batch_tune")
        return ms.value

    def info(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().wdt_batch_info(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "wdt_batch_info")
        return dict(total_blocks=a.value, blocks_per_cu=b.value, tile_cap=c.value)

    def solve(self, bs, xs, tol=1e-10, max_iter=10000, check_every=5, stream=None,
              allow_unconverged=False):
        n = len(self.gauges)
        vb = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
        vx = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        p = SolveParams(tol, max_iter, FP64, 0.0, 0, 0, check_every)
        stats = (RhsStats * sum(self.n_rhs))()
        allow = (OK, WNOTCONVERGED) if allow_unconverged else (OK,)
        rc = check(lib().wdt_batch_solve(self.h, vb, vx, ctypes.byref(p), stats, _stream(stream)),
                   "wdt_batch_solve", allow)
        return rc, [dict(iterations=s.iterations, converged=s.converged, restarts=s.restarts,
                         true_residual=s.true_residual) for s in stats]

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.wdt_batch_destroy(self.h)
            self.h = None
