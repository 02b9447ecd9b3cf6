"""Thin ctypes binding of libgpdbec (include/gp.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch supplies the device workspace and the HIP stream.  If the shared library is
missing this module raises; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree library; GPDBEC_LIB selects another build of the same sources
LIB_PATH = os.environ.get("GPDBEC_LIB", os.path.join(_PKG, "libgpdbec.so"))

GP_OK = 0
GP_E_ARG = -1
GP_E_SIZE = -2
GP_E_DEVICE = -3
GP_E_NONFINITE = -4
GP_E_STATE = -5
GP_E_NOMEM = -6
GP_E_IO = -7
GP_STATE_PSI, GP_STATE_DENSITY = 1, 2
GP_HOST_V, GP_HOST_KTAB = 1, 2

GP_3D, GP_2D_XY, GP_2D_XZ = 0, 1, 2
GP_FP64, GP_FP32_MIXED = 0, 1
GEOM = {"3d": GP_3D, "2dxy": GP_2D_XY, "2dxz": GP_2D_XZ}
PREC = {"fp64": GP_FP64, "fp32": GP_FP32_MIXED}


class gp_params(ctypes.Structure):
    _fields_ = [
        ("geom", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("gamma", ctypes.c_double), ("nu", ctypes.c_double), ("lambda_", ctypes.c_double),
        ("g", ctypes.c_double), ("gdd", ctypes.c_double),
        ("cutoff_R", ctypes.c_double),
        ("prec", ctypes.c_int),
    ]


class gp_observables(ctypes.Structure):
    _fields_ = [
        ("norm", ctypes.c_double), ("mu", ctypes.c_double), ("energy", ctypes.c_double),
        ("e_kin", ctypes.c_double), ("e_pot", ctypes.c_double), ("e_int", ctypes.c_double),
        ("e_dd", ctypes.c_double), ("rms", ctypes.c_double * 3),
    ]

    def as_dict(self):
        return {"norm": self.norm, "mu": self.mu, "energy": self.energy,
                "e_kin": self.e_kin, "e_pot": self.e_pot, "e_int": self.e_int,
                "e_dd": self.e_dd, "rms": tuple(self.rms)}


class gp_state_info(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int), ("params", gp_params), ("step", ctypes.c_longlong),
        ("time", ctypes.c_double), ("npoints", ctypes.c_ulonglong),
        ("checksum", ctypes.c_ulonglong),
    ]


# name -> (restype, argtypes), mirroring include/gp.h
_P = ctypes.c_void_p
# int (*gp_output_fn)(void* user, gp_ctx* ctx, int step, const gp_observables* obs)
GP_OUTPUT_FN = ctypes.CFUNCTYPE(ctypes.c_int, _P, _P, ctypes.c_int,
                                ctypes.POINTER(gp_observables))
_SIGS = {
    "gp_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(gp_params), ctypes.POINTER(ctypes.c_size_t)]),
    "gp_init": (ctypes.c_int, [ctypes.POINTER(gp_params), _P, ctypes.c_size_t, _P,
                               ctypes.POINTER(_P)]),
    "gp_destroy": (ctypes.c_int, [_P]),
    "gp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gp_set_psi": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "gp_get_psi": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "gp_set_potential": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "gp_set_couplings": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double]),
    "gp_step_imag": (ctypes.c_int, [_P, ctypes.c_int]),
    "gp_step_real": (ctypes.c_int, [_P, ctypes.c_int]),
    "gp_energy": (ctypes.c_int, [_P, ctypes.POINTER(gp_observables)]),
    "gp_dipolar_potential": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "gp_history": (ctypes.c_int, [_P, ctypes.POINTER(gp_observables), ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int)]),
    "gp_history_capacity": (ctypes.c_int, []),
    "gp_sync": (ctypes.c_int, [_P]),
    "gp_last_error": (ctypes.c_char_p, []),
    "gp_use_graphs": (ctypes.c_int, [_P, ctypes.c_int]),
    "gp_timing_span": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int)]),
    "gp_timing_burst": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double)]),
    "gp_batch_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(gp_params), ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "gp_batch_init": (ctypes.c_int, [ctypes.POINTER(gp_params), ctypes.c_int, _P, ctypes.c_size_t,
                                     _P, ctypes.POINTER(_P)]),
    "gp_batch_destroy": (ctypes.c_int, [_P]),
    "gp_batch_context": (_P, [_P, ctypes.c_int]),
    "gp_batch_step_imag": (ctypes.c_int, [_P, ctypes.c_int]),
    "gp_batch_step_real": (ctypes.c_int, [_P, ctypes.c_int]),
    "gp_batch_energy": (ctypes.c_int, [_P, ctypes.POINTER(gp_observables)]),
    "gp_batch_plan": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "gp_batch_set_blocks": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "gp_batch_use_graphs": (ctypes.c_int, [_P, ctypes.c_int]),
    "gp_batch_set_shape": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "gp_batch_shapes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int)]),
    "gp_step_real_adjoint": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "gp_batch_set_psi": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_int]),
    "gp_batch_get_psi": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_int]),
    "gp_batch_use_streams": (ctypes.c_int, [_P, ctypes.c_int]),
    "gp_dipolar_potential_noalloc": (ctypes.c_int, [ctypes.POINTER(gp_params), _P, _P, _P]),
    "gp_timing_enable": (ctypes.c_int, [_P, ctypes.c_uint]),
    "gp_get_params": (ctypes.c_int, [_P, ctypes.POINTER(gp_params)]),
    "gp_axis_kind": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "gp_workspace_bytes_ex": (ctypes.c_int, [ctypes.POINTER(gp_params), ctypes.c_uint,
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "gp_host_bytes": (ctypes.c_int, [ctypes.POINTER(gp_params), ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "gp_init_ex": (ctypes.c_int, [ctypes.POINTER(gp_params), ctypes.c_uint, _P, ctypes.c_size_t,
                                  _P, _P, _P, ctypes.POINTER(_P)]),
    "gp_save_state": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_longlong, ctypes.c_double]),
    "gp_save_density": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_longlong, ctypes.c_double]),
    "gp_load_state": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.POINTER(gp_state_info)]),
    "gp_state_read_info": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(gp_state_info)]),
    "gp_state_read": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(gp_state_info), _P,
                                     ctypes.c_size_t]),
    "gp_evolve": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, GP_OUTPUT_FN, _P,
                                 ctypes.POINTER(ctypes.c_int)]),
    "gp_timing_read": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int)]),
}

PASS_NAMES = ("r2c_x", "fft_y_fwd", "conv_z", "fft_y_inv", "conv_y", "c2r_nl_cnx", "cn_y",
              "cn_z", "finalize")

_lib = None


def load(path: str = LIB_PATH):
    """Load libgpdbec.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgpdbec.so not found at {path}: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    # torch ships its own HIP runtime with the same soname as the system one; loading
    # torch first makes the library bind to that runtime, so device pointers and
    # streams created by torch are valid in the library (one runtime per process).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class GPError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        lib = load()
        msg = lib.gp_status_string(status).decode()
        detail = lib.gp_last_error().decode() if status in (GP_E_DEVICE, GP_E_SIZE) else ""
        if detail:
            msg += ": " + detail
        super().__init__(f"{where}: {msg} ({status})")


def _check(status, where):
    if status != GP_OK:
        raise GPError(status, where)


def make_params(geom, nx, ny=1, nz=1, dx=0.1, dy=0.1, dz=0.1, dt=1e-3, gamma=1.0, nu=1.0,
                lam=1.0, g=0.0, gdd=0.0, R=0.0, prec="fp64", **_ignored):
    p = gp_params()
    p.geom = GEOM[geom] if isinstance(geom, str) else int(geom)
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.dx, p.dy, p.dz = float(dx), float(dy), float(dz)
    p.dt = float(dt)
    p.gamma, p.nu, p.lambda_ = float(gamma), float(nu), float(lam)
    p.g, p.gdd = float(g), float(gdd)
    p.cutoff_R = float(R)
    p.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    return p


# ------------------------------------------------------- same-name thin wrappers
def gp_workspace_bytes(params: gp_params) -> int:
    n = ctypes.c_size_t(0)
    _check(load().gp_workspace_bytes(ctypes.byref(params), ctypes.byref(n)), "gp_workspace_bytes")
    return n.value


def gp_init(params: gp_params, workspace_ptr: int, ws_bytes: int, stream_ptr: int) -> int:
    ctx = _P()
    _check(load().gp_init(ctypes.byref(params), _P(workspace_ptr), ws_bytes, _P(stream_ptr),
                          ctypes.byref(ctx)), "gp_init")
    return ctx.value


def gp_workspace_bytes_ex(params: gp_params, host: int) -> int:
    n = ctypes.c_size_t(0)
    _check(load().gp_workspace_bytes_ex(ctypes.byref(params), host, ctypes.byref(n)),
           "gp_workspace_bytes_ex")
    return n.value


def gp_host_bytes(params: gp_params) -> tuple:
    v = ctypes.c_size_t(0)
    k = ctypes.c_size_t(0)
    _check(load().gp_host_bytes(ctypes.byref(params), ctypes.byref(v), ctypes.byref(k)),
           "gp_host_bytes")
    return v.value, k.value


def gp_init_ex(params: gp_params, host: int, workspace_ptr: int, ws_bytes: int, host_v: int,
               host_ktab: int, stream_ptr: int) -> int:
    ctx = _P()
    _check(load().gp_init_ex(ctypes.byref(params), host, _P(workspace_ptr), ws_bytes,
                             _P(host_v), _P(host_ktab), _P(stream_ptr), ctypes.byref(ctx)),
           "gp_init_ex")
    return ctx.value


def gp_destroy(ctx: int):
    _check(load().gp_destroy(_P(ctx)), "gp_destroy")


def gp_set_psi(ctx: int, ptr: int, on_device: int):
    _check(load().gp_set_psi(_P(ctx), _P(ptr), on_device), "gp_set_psi")


def gp_get_psi(ctx: int, ptr: int, on_device: int):
    _check(load().gp_get_psi(_P(ctx), _P(ptr), on_device), "gp_get_psi")


def gp_set_potential(ctx: int, ptr: int, on_device: int):
    _check(load().gp_set_potential(_P(ctx), _P(ptr), on_device), "gp_set_potential")


def gp_set_couplings(ctx: int, g: float, gdd: float):
    _check(load().gp_set_couplings(_P(ctx), g, gdd), "gp_set_couplings")


def gp_step_imag(ctx: int, nsteps: int):
    _check(load().gp_step_imag(_P(ctx), nsteps), "gp_step_imag")


def gp_step_real(ctx: int, nsteps: int):
    _check(load().gp_step_real(_P(ctx), nsteps), "gp_step_real")


def gp_step_real_adjoint(ctx: int, psi_n: int, lam: int, gradV: int, grad_g: int,
                         grad_gdd: int):
    _check(load().gp_step_real_adjoint(_P(ctx), _P(psi_n), _P(lam), _P(gradV), _P(grad_g),
                                       _P(grad_gdd)), "gp_step_real_adjoint")


def gp_energy(ctx: int) -> dict:
    ob = gp_observables()
    _check(load().gp_energy(_P(ctx), ctypes.byref(ob)), "gp_energy")
    return ob.as_dict()


def gp_dipolar_potential(ctx: int, ptr: int, on_device: int):
    _check(load().gp_dipolar_potential(_P(ctx), _P(ptr), on_device), "gp_dipolar_potential")


def gp_dipolar_potential_noalloc(params: gp_params, psi_ptr: int, phi_ptr: int,
                                 stream_ptr: int):
    _check(load().gp_dipolar_potential_noalloc(ctypes.byref(params), _P(psi_ptr), _P(phi_ptr),
                                               _P(stream_ptr)), "gp_dipolar_potential_noalloc")


def gp_history(ctx: int, max_records: int) -> list:
    arr = (gp_observables * max(1, max_records))()
    cnt = ctypes.c_int(0)
    _check(load().gp_history(_P(ctx), arr, max_records, ctypes.byref(cnt)), "gp_history")
    return [arr[i].as_dict() for i in range(cnt.value)]


def gp_sync(ctx: int):
    _check(load().gp_sync(_P(ctx)), "gp_sync")


def gp_use_graphs(ctx: int, enable: bool):
    _check(load().gp_use_graphs(_P(ctx), int(bool(enable))), "gp_use_graphs")


def gp_timing_enable(ctx: int, mask: int):
    _check(load().gp_timing_enable(_P(ctx), mask), "gp_timing_enable")


def gp_timing_read(ctx: int) -> dict:
    n = len(PASS_NAMES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int * n)()
    _check(load().gp_timing_read(_P(ctx), ms, cnt), "gp_timing_read")
    return {PASS_NAMES[i]: (ms[i], cnt[i]) for i in range(n)}


def gp_timing_span(ctx: int, pass_name: str) -> tuple:
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int(0)
    _check(load().gp_timing_span(_P(ctx), PASS_NAMES.index(pass_name), ctypes.byref(ms),
                                 ctypes.byref(n)), "gp_timing_span")
    return ms.value, n.value


def gp_timing_burst(ctx: int, pass_name: str, reps: int) -> float:
    ms = ctypes.c_double(0.0)
    _check(load().gp_timing_burst(_P(ctx), PASS_NAMES.index(pass_name), reps, ctypes.byref(ms)),
           "gp_timing_burst")
    return ms.value


def _info_dict(info: gp_state_info) -> dict:
    p = info.params
    geom = {v: k for k, v in GEOM.items()}[p.geom]
    return {"kind": info.kind, "step": info.step, "time": info.time, "npoints": info.npoints,
            "params": {"geom": geom, "nx": p.nx, "ny": p.ny, "nz": p.nz, "dx": p.dx,
                       "dy": p.dy, "dz": p.dz, "dt": p.dt, "gamma": p.gamma, "nu": p.nu,
                       "lam": p.lambda_, "g": p.g, "gdd": p.gdd, "R": p.cutoff_R,
                       "prec": "fp64" if p.prec == GP_FP64 else "fp32"}}


def gp_get_params(ctx: int) -> gp_params:
    p = gp_params()
    _check(load().gp_get_params(_P(ctx), ctypes.byref(p)), "gp_get_params")
    return p


def gp_save_state(ctx: int, path: str, step: int = 0, time: float = 0.0):
    _check(load().gp_save_state(_P(ctx), os.fsencode(path), step, time), "gp_save_state")


def gp_save_density(ctx: int, path: str, step: int = 0, time: float = 0.0):
    _check(load().gp_save_density(_P(ctx), os.fsencode(path), step, time), "gp_save_density")


def gp_load_state(ctx: int, path: str) -> dict:
    info = gp_state_info()
    _check(load().gp_load_state(_P(ctx), os.fsencode(path), ctypes.byref(info)), "gp_load_state")
    return _info_dict(info)


def gp_state_read_info(path: str) -> dict:
    info = gp_state_info()
    _check(load().gp_state_read_info(os.fsencode(path), ctypes.byref(info)), "gp_state_read_info")
    return _info_dict(info)


def gp_state_read(path: str):
    """(header dict, values): complex128 for a wave-function file, float64 for a density
    file, in the grid's shape."""
    head = gp_state_read_info(path)
    k = 2 if head["kind"] == GP_STATE_PSI else 1
    buf = np.empty(head["npoints"] * k, dtype=np.float64)
    info = gp_state_info()
    _check(load().gp_state_read(os.fsencode(path), ctypes.byref(info), _P(buf.ctypes.data),
                                buf.size), "gp_state_read")
    vals = buf.view(np.complex128) if k == 2 else buf
    return head, vals.reshape(_shape(head["params"]))


def gp_evolve(ctx: int, imag: bool, nsteps: int, every: int, fn=None) -> int:
    """nsteps steps in runs of `every`; fn(step, observables dict) is called after 0, every,
    ... and nsteps steps (return True to stop).  Returns the steps taken."""
    done = ctypes.c_int(0)
    errors = []

    def tramp(_user, _ctx, step, obs):
        try:
            return 1 if fn(step, obs.contents.as_dict()) else 0
        except Exception as e:  # noqa: BLE001 - re-raised below, after the C loop returns
            errors.append(e)
            return 1

    cb = GP_OUTPUT_FN(tramp) if fn is not None else GP_OUTPUT_FN()
    st = load().gp_evolve(_P(ctx), int(bool(imag)), nsteps, every, cb, None, ctypes.byref(done))
    if errors:
        raise errors[0]
    _check(st, "gp_evolve")
    return done.value


def gp_axis_kind(n: int, prec: str = "fp64") -> int:
    """1: specialised passes, 2: run-time-length passes, 3: a 2D axis longer than one LDS
    line (four-step transforms, segmented sweeps), 0: unsupported."""
    return load().gp_axis_kind(n, PREC[prec])


def supported_sizes(limit: int = 16384, prec: str = "fp64", kind=None) -> list:
    """Axis lengths gp_init accepts (kind 1, 2 or, in 2D grids, 3; or only the given
    kind)."""
    out = []
    for n in range(2, limit + 1):
        k = gp_axis_kind(n, prec)
        if k and (kind is None or k == kind):
            out.append(n)
    return out


# ------------------------------------------------------------ convenience class
class Solver:
    """One context on one device: owns a torch workspace tensor and uses a torch stream.

    params: dict with the keys of `make_params` (geom, nx, ny, nz, dx, dy, dz, dt, gamma,
    nu, lam, g, gdd, R); prec: "fp64" or "fp32" (FP32 bulk, FP64 reductions)."""

    def __init__(self, params: dict, prec: str = "fp64", device: str = "cuda:0", stream=None,
                 host=()):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.params = dict(params)
        self.prec = prec
        self.p = make_params(**{**params, "prec": prec})
        self.shape = _shape(params)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # host: "V" and/or "ktab" kept in pinned host memory (gp_init_ex)
        flags = (GP_HOST_V if "V" in host else 0) | (GP_HOST_KTAB if "ktab" in host else 0)
        self.host_flags = flags
        self.ws_bytes = gp_workspace_bytes_ex(self.p, flags)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.host_v = self.host_ktab = None
        if flags:
            vb, kb = gp_host_bytes(self.p)
            if flags & GP_HOST_V:
                self.host_v = torch.empty(vb, dtype=torch.uint8, pin_memory=True)
            if flags & GP_HOST_KTAB:
                self.host_ktab = torch.empty(kb, dtype=torch.uint8, pin_memory=True)
        self.ctx = gp_init_ex(self.p, flags, self._ws_ptr, self.ws_bytes,
                              self.host_v.data_ptr() if self.host_v is not None else 0,
                              self.host_ktab.data_ptr() if self.host_ktab is not None else 0,
                              self.stream.cuda_stream)
        self.cdtype = torch.complex128 if prec == "fp64" else torch.complex64
        self.rdtype = torch.float64 if prec == "fp64" else torch.float32

    def close(self):
        if self.ctx:
            gp_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- state
    def set_psi(self, psi):
        if isinstance(psi, np.ndarray):
            a = np.ascontiguousarray(psi, dtype=np.complex128)
            assert a.shape == self.shape, (a.shape, self.shape)
            gp_set_psi(self.ctx, a.ctypes.data, 0)
        else:
            t = psi.to(device=self.device, dtype=self.cdtype).contiguous()
            assert tuple(t.shape) == self.shape
            gp_set_psi(self.ctx, t.data_ptr(), 1)
            self.stream.synchronize()

    def get_psi(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.complex128)
        gp_get_psi(self.ctx, out.ctypes.data, 0)
        return out

    def get_psi_device(self):
        t = self.torch.empty(self.shape, dtype=self.cdtype, device=self.device)
        gp_get_psi(self.ctx, t.data_ptr(), 1)
        return t

    def set_potential(self, V):
        if isinstance(V, np.ndarray):
            a = np.ascontiguousarray(V, dtype=np.float64)
            assert a.shape == self.shape
            gp_set_potential(self.ctx, a.ctypes.data, 0)
        else:
            t = V.to(device=self.device, dtype=self.rdtype).contiguous()
            gp_set_potential(self.ctx, t.data_ptr(), 1)
            self.stream.synchronize()

    def set_couplings(self, g, gdd):
        gp_set_couplings(self.ctx, g, gdd)

    # --- method
    def step_imag(self, n: int):
        gp_step_imag(self.ctx, n)

    def step_real(self, n: int):
        gp_step_real(self.ctx, n)

    def energy(self) -> dict:
        return gp_energy(self.ctx)

    def dipolar_potential(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float64)
        gp_dipolar_potential(self.ctx, out.ctypes.data, 0)
        return out

    def dipolar_potential_device(self):
        """Phi of the current psi (without g_dd) as a device tensor of the context
        precision (asynchronous on the solver's stream)."""
        t = self.torch.empty(self.shape, dtype=self.rdtype, device=self.device)
        gp_dipolar_potential(self.ctx, t.data_ptr(), 1)
        return t

    def history(self, n: int) -> list:
        return gp_history(self.ctx, n)

    def sync(self):
        gp_sync(self.ctx)

    def use_graphs(self, enable: bool):
        gp_use_graphs(self.ctx, enable)

    def timing_enable(self, passes=()):
        mask = 0
        for p in passes:
            mask |= 1 << PASS_NAMES.index(p)
        gp_timing_enable(self.ctx, mask)

    def timing_read(self) -> dict:
        return gp_timing_read(self.ctx)

    def timing_span(self, pass_name: str = "c2r_nl_cnx") -> tuple:
        """(summed in-kernel spans in ms, launches) since timing_enable."""
        return gp_timing_span(self.ctx, pass_name)

    # --- saved states and output cadence
    def save_state(self, path: str, step: int = 0, time: float = 0.0):
        gp_save_state(self.ctx, path, step, time)

    def save_density(self, path: str, step: int = 0, time: float = 0.0):
        gp_save_density(self.ctx, path, step, time)

    def load_state(self, path: str) -> dict:
        return gp_load_state(self.ctx, path)

    def evolve(self, imag: bool, nsteps: int, every: int = 0, fn=None) -> int:
        return gp_evolve(self.ctx, imag, nsteps, every, fn)

    def timing_burst(self, pass_name: str, reps: int = 64) -> float:
        """ms per launch of one pass replayed back to back (advances the state)."""
        return gp_timing_burst(self.ctx, pass_name, reps)


def _shape(params):
    g = params["geom"]
    if g == "3d":
        return (params["nz"], params["ny"], params["nx"])
    if g == "2dxy":
        return (params["ny"], params["nx"])
    return (params["nz"], params["nx"])


# ------------------------------------------------------------------ batched ensemble
BATCH_PASSES = ("r2c_x", "conv_y", "c2r_nl_cnx", "cn_y")
BATCH_CLASSES = 2


class Batch:
    """Many independent quasi-2D instances stepped together (gp_batch_*): one persistent
    launch per pass and size class.  params_list: dicts as for Solver (geom 2dxy/2dxz)."""

    def __init__(self, params_list, prec="fp32", device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.prec = prec
        self.count = len(params_list)
        arr = (gp_params * self.count)()
        for i, p in enumerate(params_list):
            arr[i] = make_params(**{**p, "prec": prec})
        self._arr = arr
        self.shapes = [_shape(p) for p in params_list]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        lib = load()
        n = ctypes.c_size_t(0)
        _check(lib.gp_batch_workspace_bytes(arr, self.count, ctypes.byref(n)),
               "gp_batch_workspace_bytes")
        self.ws_bytes = n.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) & ~255
        h = _P()
        _check(lib.gp_batch_init(arr, self.count, _P(ptr), self.ws_bytes,
                                 _P(self.stream.cuda_stream), ctypes.byref(h)), "gp_batch_init")
        self.handle = h.value
        self.ctxs = [lib.gp_batch_context(_P(self.handle), i) for i in range(self.count)]

    def close(self):
        if self.handle:
            _check(load().gp_batch_destroy(_P(self.handle)), "gp_batch_destroy")
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shape_of(self, idx):
        # an index out of range is passed through: the library answers GP_E_ARG
        return self.shapes[idx] if 0 <= idx < self.count else (1,)

    def set_psi(self, idx, psi):
        """psi: a host array (converted from FP64), or a device tensor of the batch
        precision (copied on the device)."""
        if isinstance(psi, np.ndarray):
            a = np.ascontiguousarray(psi, dtype=np.complex128)
            assert not 0 <= idx < self.count or a.shape == self.shapes[idx]
            _check(load().gp_batch_set_psi(_P(self.handle), idx, _P(a.ctypes.data), 0),
                   "gp_batch_set_psi")
            return
        cd = self.torch.complex128 if self.prec == "fp64" else self.torch.complex64
        t = psi.to(device=self.device, dtype=cd).contiguous()
        assert not 0 <= idx < self.count or tuple(t.shape) == self.shapes[idx]
        _check(load().gp_batch_set_psi(_P(self.handle), idx, _P(t.data_ptr()), 1),
               "gp_batch_set_psi")
        self.stream.synchronize()

    def get_psi(self, idx):
        out = np.empty(self._shape_of(idx), dtype=np.complex128)
        _check(load().gp_batch_get_psi(_P(self.handle), idx, _P(out.ctypes.data), 0),
               "gp_batch_get_psi")
        return out

    def use_streams(self, enable):
        _check(load().gp_batch_use_streams(_P(self.handle), int(bool(enable))),
               "gp_batch_use_streams")

    def step_imag(self, n):
        _check(load().gp_batch_step_imag(_P(self.handle), n), "gp_batch_step_imag")

    def step_real(self, n):
        _check(load().gp_batch_step_real(_P(self.handle), n), "gp_batch_step_real")

    def energy(self):
        arr = (gp_observables * self.count)()
        _check(load().gp_batch_energy(_P(self.handle), arr), "gp_batch_energy")
        return [arr[i].as_dict() for i in range(self.count)]

    def history(self, idx, n):
        return gp_history(self.ctxs[idx], n)

    def plan(self):
        k = len(BATCH_PASSES) * BATCH_CLASSES
        items = (ctypes.c_int * k)()
        blocks = (ctypes.c_int * k)()
        _check(load().gp_batch_plan(_P(self.handle), items, blocks), "gp_batch_plan")
        return {(BATCH_PASSES[i // BATCH_CLASSES], i % BATCH_CLASSES): (items[i], blocks[i])
                for i in range(k)}

    def set_blocks(self, pass_name, size_class, blocks):
        _check(load().gp_batch_set_blocks(_P(self.handle), BATCH_PASSES.index(pass_name),
                                          size_class, blocks), "gp_batch_set_blocks")

    def set_shape(self, pass_name, size_class, shape):
        _check(load().gp_batch_set_shape(_P(self.handle), BATCH_PASSES.index(pass_name),
                                         size_class, shape), "gp_batch_set_shape")

    def tile_shapes(self):
        k = len(BATCH_PASSES) * BATCH_CLASSES
        out = (ctypes.c_int * k)()
        _check(load().gp_batch_shapes(_P(self.handle), out), "gp_batch_shapes")
        return {(BATCH_PASSES[i // BATCH_CLASSES], i % BATCH_CLASSES): out[i] for i in range(k)}

    def use_graphs(self, enable):
        _check(load().gp_batch_use_graphs(_P(self.handle), int(bool(enable))), "gp_batch_use_graphs")

    def points(self):
        return int(sum(int(np.prod(s)) for s in self.shapes))
