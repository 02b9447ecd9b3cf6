"""Host-only checks of the C-ABI library: it loads, exports every symbol the header
declares, and validates parameters (no device work, runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1601_04640_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "gp.h")) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = B.load()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares exactly the header's functions
    assert sorted(B._SIGS) == names


def test_struct_layouts_match_header():
    assert ctypes.sizeof(B.gp_observables) == 10 * 8
    # int geom, 3 ints, 10 doubles, int prec (with padding)
    assert B.gp_params.dx.offset == 16
    assert B.gp_params.prec.offset == 16 + 10 * 8


def test_status_strings():
    lib = B.load()
    for s in (0, -1, -2, -3, -4, -5, -6, -7):
        assert len(lib.gp_status_string(s)) > 0


def ws(**kw):
    base = dict(geom="3d", nx=16, ny=16, nz=16, dx=0.2, dy=0.2, dz=0.2, dt=1e-3)
    base.update(kw)
    return B.gp_workspace_bytes(B.make_params(**base))


# below 4, or an FFT line past 64 KiB of LDS (FP64: 4096 points; for a length with a prime
# factor above 31, Bluestein's M >= 2N - 1: 2062 = 2 1031 needs M = 4125 -> 4200)
@pytest.mark.parametrize("n", [3, 2, 0, -8, 2062, 4098, 8192])
def test_unsupported_sizes_rejected(n):
    with pytest.raises(B.GPError) as e:
        ws(nx=n, prec="fp64")
    assert e.value.status == B.GP_E_SIZE
    with pytest.raises(B.GPError) as e:
        ws(nz=n, prec="fp64")
    assert e.value.status == B.GP_E_SIZE


def test_line_length_limit_depends_on_precision():
    assert ws(geom="2dxy", nx=8192, ny=8, prec="fp32") > 0
    assert ws(geom="2dxy", nx=2062, ny=8, prec="fp32") > 0   # Bluestein M = 4200
    assert B.gp_axis_kind(2062, "fp64") == 0 and B.gp_axis_kind(2039, "fp64") == 2
    assert B.gp_axis_kind(8192, "fp32") == 2 and B.gp_axis_kind(8192, "fp64") == 3
    # past one LDS line a 3D axis is refused ...
    for prec, n in (("fp64", 8192), ("fp32", 8194)):
        with pytest.raises(B.GPError) as e:
            ws(nx=n, prec=prec)
        assert e.value.status == B.GP_E_SIZE


# 2D axes longer than one LDS line (kind 3): a four-step split n = A B (both transforms
# within one line) and Crank-Nicolson segments; the paper's 2D grids 13000^2 and 15000^2
@pytest.mark.parametrize("prec,n", [("fp32", 8194), ("fp32", 9000), ("fp32", 13000),
                                    ("fp32", 15000), ("fp32", 8284), ("fp64", 4098),
                                    ("fp64", 8192), ("fp64", 15000), ("fp64", 4500)])
def test_long_2d_axes_accepted(prec, n):
    assert B.gp_axis_kind(n, prec) == 3
    for geom in ("2dxy", "2dxz"):
        assert ws(geom=geom, nx=n, ny=12, nz=12, prec=prec) > 0
        assert ws(geom=geom, nx=12, ny=n, nz=n, prec=prec) > 0
    assert ws(geom="2dxy", nx=n, ny=n, prec=prec) > 0


# no split: primes, and 2 p with p a prime whose line (by Bluestein's algorithm) is too
# long for two rows in LDS
@pytest.mark.parametrize("prec,n", [("fp32", 8209), ("fp32", 2 * 4099), ("fp64", 4099),
                                    ("fp64", 2 * 2053)])
def test_long_axes_without_split_rejected(prec, n):
    assert B.gp_axis_kind(n, prec) == 0
    with pytest.raises(B.GPError) as e:
        ws(geom="2dxy", nx=n, ny=12, prec=prec)
    assert e.value.status == B.GP_E_SIZE


# the specialised lengths, and lengths the run-time-length passes take (the paper's
# grids 50, 540, 600, 1000 among them; radices 7, 11, 13, 31; odd lengths)
@pytest.mark.parametrize("n", [8, 10, 12, 16, 20, 24, 30, 32, 40, 48, 60, 64, 80, 96, 120,
                               128, 160, 192, 240, 256, 320, 384, 480, 512,
                               4, 6, 14, 22, 26, 36, 50, 54, 62, 90, 100, 540, 600, 1000,
                               1024, 2048, 4096, 5, 7, 9, 15, 45, 49, 99, 625, 1001, 4095,
                               37, 74, 111, 106, 1009, 2039])
def test_supported_sizes_accepted(n):
    assert ws(nx=n, ny=8, nz=8, prec="fp64") > 0


def test_every_length_to_600_is_accepted():
    """Every length 4..600, even or odd, runs: kind 1 exactly for the specialised lengths
    (2^a 3^b 5^c, b, c <= 1, 8..512, even), kind 2 otherwise (prime factors up to 31 by
    Stockham stages, larger ones by Bluestein's algorithm); FP32 and FP64 agree."""
    spec = {8, 10, 12, 16, 20, 24, 30, 32, 40, 48, 60, 64, 80, 96, 120, 128, 160, 192, 240,
            256, 320, 384, 480, 512}
    for n in range(4, 601):
        for prec in ("fp32", "fp64"):
            assert B.gp_axis_kind(n, prec) == (1 if n in spec else 2), (n, prec)
        assert ws(geom="2dxy", nx=n, ny=8, prec="fp64") > 0


@pytest.mark.parametrize("kw", [dict(dt=0.0), dict(dt=-1e-3), dict(dx=0.0), dict(dy=-0.1),
                                dict(geom=7), dict(prec=5), dict(g=float("nan")),
                                dict(geom="2dxy", lam=0.0), dict(geom="2dxz", nu=-1.0)])
def test_bad_arguments_rejected(kw):
    with pytest.raises(B.GPError) as e:
        ws(**kw)
    assert e.value.status == B.GP_E_ARG


def test_2d_ignores_unused_axis():
    a = ws(geom="2dxy", nx=64, ny=32, nz=7)       # nz ignored in XY
    b = ws(geom="2dxz", nx=64, ny=3, nz=32)        # ny ignored in XZ
    assert a == b


def test_workspace_scales_with_precision_and_size():
    assert ws(prec="fp64") > ws(prec="fp32")
    assert ws(nx=32) > ws(nx=16)


def test_null_arguments_rejected():
    lib = B.load()
    n = ctypes.c_size_t(0)
    assert lib.gp_workspace_bytes(None, ctypes.byref(n)) == B.GP_E_ARG
    p = B.make_params("3d", 16, 16, 16)
    assert lib.gp_workspace_bytes(ctypes.byref(p), None) == B.GP_E_ARG
    ctx = ctypes.c_void_p()
    assert lib.gp_init(ctypes.byref(p), None, 0, None, ctypes.byref(ctx)) == B.GP_E_ARG
    for fn in ("gp_step_imag", "gp_step_real"):
        assert getattr(lib, fn)(None, 1) == B.GP_E_ARG
    assert lib.gp_destroy(None) == B.GP_E_ARG
    assert lib.gp_sync(None) == B.GP_E_ARG
    assert lib.gp_history_capacity() >= 1000


def test_host_resident_arrays_shrink_the_workspace():
    def align(n):
        return (n + 255) // 256 * 256
    for geom, kw in (("3d", {}), ("2dxz", dict(nx=40, ny=1, nz=48))):
        p = B.make_params(**{**dict(geom=geom, nx=24, ny=20, nz=16, dx=0.2, dy=0.2, dz=0.2,
                                    dt=1e-3, nu=4.0), **kw, "prec": "fp32"})
        full = B.gp_workspace_bytes(p)
        vb, kb = B.gp_host_bytes(p)
        assert B.gp_workspace_bytes_ex(p, 0) == full
        assert full - B.gp_workspace_bytes_ex(p, B.GP_HOST_V) == align(vb)
        assert full - B.gp_workspace_bytes_ex(p, B.GP_HOST_KTAB) == align(kb)
        assert full - B.gp_workspace_bytes_ex(p, B.GP_HOST_V | B.GP_HOST_KTAB) == align(vb) + align(kb)
    with pytest.raises(B.GPError) as e:
        B.gp_workspace_bytes_ex(p, 4)
    assert e.value.status == B.GP_E_ARG
