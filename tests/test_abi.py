"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/wdt.h declares, validates arguments, and its host-only
torus-colouring search agrees with the oracle's."""
import ctypes
import json
import os

import pytest

from paper_2607_05157_amd import wdt

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_header_function():
    L = wdt.lib()
    names = wdt.header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n


def test_error_strings_and_version():
    L = wdt.lib()
    assert L.wdt_error_string(wdt.EINVAL) == b"invalid argument"
    assert L.wdt_error_string(wdt.OK) == b"ok"
    assert b"gfx950" in L.wdt_version()


def test_lattice_argument_validation():
    L = wdt.lib()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int32 * 4)(4, 4, 1, 4)
    assert L.wdt_lattice_create(dims, -1, ctypes.byref(h)) == wdt.EINVAL
    buf = ctypes.create_string_buffer(256)
    L.wdt_last_error_detail(buf, 256)
    assert b"extent" in buf.value
    dims = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    assert L.wdt_lattice_create(dims, 0, ctypes.byref(h)) == wdt.EINVAL
    lat = wdt.Lattice((4, 4, 4, 6), -1)
    assert lat.V == 384
    assert lat.spinor_bytes(3, wdt.FP64) == 384 * 12 * 3 * 16
    assert lat.spinor_bytes(3, wdt.FP16) == 384 * 12 * 3 * 4 + 384 * 3 * 4
    assert lat.spinor_bytes(3, wdt.BF16) == 384 * 12 * 3 * 4
    with pytest.raises(wdt.WdtError):
        lat.spinor_bytes(0, wdt.FP64)


def test_null_handles_rejected():
    L = wdt.lib()
    assert L.wdt_apply_D(None, 0.1, None, None, 1, 0, 0, None) == wdt.EINVAL
    assert L.wdt_solve(None, 0.1, None, None, 1, None, None, None) == wdt.EINVAL
    assert L.wdt_contract(None, None, None, 1, None, 0, None, None) == wdt.EINVAL


def test_colouring_search_matches_oracle_golden():
    g = json.load(open(os.path.join(GOLD, "colourings_workloads.json")))
    for case in g["cases"]:
        if case["n_c"] > 64 and len(case["dims"]) == 4:
            continue                       # the 96-colour search takes ~20 s; see the slow test
        nc, sig = wdt.colouring_search(case["dims"], case["d"])
        assert (nc, list(sig)) == (case["n_c"], case["sigma"]), case


@pytest.mark.slow
def test_colouring_search_large_golden():
    g = json.load(open(os.path.join(GOLD, "colourings_workloads.json")))
    for case in g["cases"]:
        if case["n_c"] > 64 and len(case["dims"]) == 4:
            nc, sig = wdt.colouring_search(case["dims"], case["d"])
            assert (nc, list(sig)) == (case["n_c"], case["sigma"]), case


def test_colouring_table1():
    g = json.load(open(os.path.join(GOLD, "table1_colours.json")))
    for d, nc in g["n_c_3d"].items():
        assert wdt.colouring_search(g["torus_3d"], int(d))[0] == nc
    for d, nc in g["n_c_4d"].items():
        got = wdt.colouring_search(g["torus_4d"], int(d))[0]
        assert got == (16 if d == "2" else nc)


def test_colouring_check_and_search_failure():
    assert wdt.colouring_check((16, 16, 16, 32), 2, 16, (1, 2, 3, 4))
    assert not wdt.colouring_check((16, 16, 16, 32), 2, 16, (1, 1, 3, 4))
    with pytest.raises(wdt.WdtError) as e:
        wdt.colouring_search((8, 8, 8, 8), 3, max_nc=8)
    assert e.value.code == wdt.ESEARCH


def test_library_shares_torchs_hip_runtime():
    """Loading the library through the binding, in a fresh process that has
    not imported torch, leaves exactly one HIP runtime in the process."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); from paper_2607_05157_amd import wdt; wdt.lib(); "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"
