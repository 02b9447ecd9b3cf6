"""State files (the imaginary -> real-time hand-off): the library's readers against files
written here, independently, from the layout documented in include/gp.h; damaged files
are refused.  The readers also run in a host-only build with the address and
undefined-behaviour sanitizers.  No GPU: only the host-side readers are called."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_1601_04640_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fnv1a64(data: bytes) -> int:
    h = 0xcbf29ce484222325
    for b in data:
        h ^= b
        h = (h * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def write_state(path, kind, geom, nx, ny, nz, values, step=7, time=0.0035, prec=0,
                spacing=(0.3, 0.35, 0.4), checksum=None):
    """A state file byte for byte as the header comment of include/gp.h lays it out."""
    payload = np.ascontiguousarray(values).astype("<f8" if kind == 2 else "<c16").tobytes()
    npts = values.size
    head = bytearray(256)
    head[0:8] = b"GPDBECS1"
    struct.pack_into("<II", head, 8, 1, kind)
    struct.pack_into("<iiii", head, 16, geom, nx, ny, nz)
    struct.pack_into("<10d", head, 32, *spacing, 0.001, 1.0, 1.2, 2.0, 20.0, 6.0, 3.5)
    struct.pack_into("<i", head, 112, prec)
    struct.pack_into("<qd", head, 120, step, time)
    struct.pack_into("<QQ", head, 136, npts, fnv1a64(payload) if checksum is None else checksum)
    with open(path, "wb") as f:
        f.write(bytes(head) + payload)


@pytest.fixture(scope="module")
def lib():
    return B.load()


def test_reader_returns_header_and_values(lib, tmp_path):
    rng = np.random.default_rng(11)
    psi = rng.standard_normal((6, 5, 4)) + 1j * rng.standard_normal((6, 5, 4))
    path = str(tmp_path / "psi.gpd")
    write_state(path, 1, B.GP_3D, 4, 5, 6, psi, step=123, time=0.25, prec=1)
    head, vals = B.gp_state_read(path)
    assert head["kind"] == B.GP_STATE_PSI and head["step"] == 123 and head["time"] == 0.25
    p = head["params"]
    assert (p["geom"], p["nx"], p["ny"], p["nz"], p["prec"]) == ("3d", 4, 5, 6, "fp32")
    assert (p["dx"], p["dy"], p["dz"], p["g"], p["gdd"], p["R"]) == (0.3, 0.35, 0.4, 20.0, 6.0, 3.5)
    assert vals.dtype == np.complex128 and vals.shape == (6, 5, 4)
    assert np.array_equal(vals, psi)
    den = np.abs(psi[0]) ** 2                       # a 2D XZ density file (nz = 5 rows)
    path2 = str(tmp_path / "den.gpd")
    write_state(path2, 2, B.GP_2D_XZ, 4, 1, 5, den[:5, :4])
    head2, vals2 = B.gp_state_read(path2)
    assert head2["kind"] == B.GP_STATE_DENSITY and vals2.shape == (5, 4)
    assert np.array_equal(vals2, den[:5, :4])


def damaged_files(tmp_path):
    """(name, path) of files the readers must refuse with GP_E_IO."""
    rng = np.random.default_rng(12)
    psi = rng.standard_normal((4, 6)) + 1j * rng.standard_normal((4, 6))
    good = str(tmp_path / "good.gpd")
    write_state(good, 1, B.GP_2D_XY, 6, 4, 1, psi)
    raw = open(good, "rb").read()
    out = []

    def put(name, data):
        p = str(tmp_path / f"{name}.gpd")
        with open(p, "wb") as f:
            f.write(data)
        out.append((name, p))

    put("magic", b"GPDBECS2" + raw[8:])
    put("version", raw[:8] + struct.pack("<I", 2) + raw[12:])
    put("kind", raw[:12] + struct.pack("<I", 3) + raw[16:])
    put("short_header", raw[:100])
    put("short_payload", raw[:-8])
    put("trailing", raw + b"\0")
    flipped = bytearray(raw)
    flipped[300] ^= 1
    put("checksum", bytes(flipped))
    put("npoints", raw[:136] + struct.pack("<Q", 25) + raw[144:])
    put("geom", raw[:16] + struct.pack("<i", 7) + raw[20:])
    return good, out


def test_damaged_files_are_refused(lib, tmp_path):
    good, bad = damaged_files(tmp_path)
    B.gp_state_read(good)
    for name, path in bad:
        with pytest.raises(B.GPError) as e:
            B.gp_state_read(path)
        assert e.value.status == B.GP_E_IO, name
    with pytest.raises(B.GPError) as e:
        B.gp_state_read_info(str(tmp_path / "missing.gpd"))
    assert e.value.status == B.GP_E_IO


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_readers_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "state_reader")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "paper_1601_04640_amd", "csrc", "gp_state.cpp"),
           os.path.join(ROOT, "tests", "host", "state_reader_main.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    good, bad = damaged_files(tmp_path)
    # the environment is passed through as it is; the runtime's link-order check is off
    # so that a library preloaded by the environment does not stop the run
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, good] + [p for _, p in bad], capture_output=True, text=True,
                       env=env)
    assert r.returncode == 0, r.stderr
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    lines = r.stdout.split("\n")
    assert lines[0] == "0 1 24"
    for (name, _), line in zip(bad, lines[1:]):
        assert line.split()[0] == str(B.GP_E_IO), (name, line)
