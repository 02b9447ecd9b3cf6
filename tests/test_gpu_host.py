"""Host-resident trap potential and kernel table (gp_init_ex with GP_HOST_V /
GP_HOST_KTAB; the paper's POTMEM choice, Fig. 1): the kernels read the arrays from pinned
host memory through its device mapping, and every result is bit for bit that of a
context with the arrays in the device workspace; and against the FP64 oracle."""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1601_04640_amd import binding as B
from paper_1601_04640_amd import inputs as I
from tests.gpu_util import FP32_PSI_TOL, FP64_PSI_TOL, assert_psi_close, banner, oparams

pytestmark = pytest.mark.gpu

CASES = {
    "3d_24x20x16": dict(geom="3d", nx=24, ny=20, nz=16, dx=0.35, dy=0.4, dz=0.45, dt=0.002,
                        gamma=1.0, nu=1.3, lam=2.0, g=25.0, gdd=8.0, R=2.8),
    "2dxy_48x40": dict(geom="2dxy", nx=48, ny=40, nz=1, dx=0.25, dy=0.3, dz=1.0, dt=0.002,
                       gamma=1.0, nu=1.5, lam=4.0, g=30.0, gdd=10.0, R=0.0),
    # run-time-length axes
    "3d_50x54x36": dict(geom="3d", nx=50, ny=54, nz=36, dx=0.3, dy=0.28, dz=0.4, dt=0.002,
                        gamma=1.0, nu=1.2, lam=2.0, g=25.0, gdd=8.0, R=4.0),
    # 2D axes past one LDS line (four-step transforms, segmented sweeps): the kernel table
    # in the spectrum's slot order, read from host memory
    "2dxy_9000x12": dict(geom="2dxy", nx=9000, ny=12, nz=1, dx=25.6 / 9000, dy=0.5, dz=1.0,
                         dt=0.0005, gamma=1.0, nu=1.0, lam=4.0, g=10.0, gdd=5.0, R=0.0),
    "2dxz_10x8400": dict(geom="2dxz", nx=10, ny=1, nz=8400, dx=0.5, dy=1.0, dz=25.6 / 8400,
                         dt=0.0005, gamma=1.0, nu=4.0, lam=1.0, g=10.0, gdd=5.0, R=0.0),
}


def run(w, prec, host, psi0, V=None):
    from paper_1601_04640_amd.binding import Solver
    s = Solver(w, prec=prec, host=host)
    if V is not None:
        s.set_potential(V)
    s.set_psi(psi0)
    s.step_imag(9)
    s.step_real(10)
    out = (s.get_psi(), s.history(19), s.energy(), s.dipolar_potential())
    return s, out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_host_arrays_equal_resident_ones(name, prec, gpu_lib):
    w = CASES[name]
    banner("host-resident V and kernel table", name, prec)
    p = oparams(w)
    psi0 = I.random_complex(p.shape(), 701, p.dV())
    s0, ref = run(w, prec, (), psi0)
    for host in (("V",), ("ktab",), ("V", "ktab")):
        s1, got = run(w, prec, host, psi0)
        assert np.array_equal(got[0], ref[0]), host
        assert got[1] == ref[1] and got[2] == ref[2], host
        assert np.array_equal(got[3], ref[3]), host
        if "V" in host:   # the pinned buffer holds the harmonic trap in the context precision
            dt = np.float64 if prec == "fp64" else np.float32
            Vh = s1.host_v.numpy().view(dt).reshape(s1.shape).astype(np.float64)
            Vo = O.harmonic_potential(p)
            # the device evaluates the same FP64 formula in another order, then rounds to T
            assert np.max(np.abs(Vh - Vo)) <= float(np.finfo(dt).eps) * np.max(np.abs(Vo))
        s1.close()
    s0.close()
    # and against the oracle (imaginary then real time)
    ref_psi = O.run(O.run(psi0, p, True, 9), p, False, 10)
    assert_psi_close(ref[0], ref_psi, FP64_PSI_TOL if prec == "fp64" else FP32_PSI_TOL)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_set_potential_writes_the_host_array(prec, gpu_lib):
    import torch
    w = CASES["3d_24x20x16"]
    banner("host-resident V: set_potential", prec)
    p = oparams(w)
    psi0 = I.random_complex(p.shape(), 702, p.dV())
    V = O.harmonic_potential(p) + 0.3 * I.smooth_random_field(p.shape(), p.spacings(), 1.0, 703)
    s0, ref = run(w, prec, (), psi0, V)
    s1, got = run(w, prec, ("V",), psi0, V)
    assert np.array_equal(got[0], ref[0])
    dt = np.float64 if prec == "fp64" else np.float32
    assert np.array_equal(s1.host_v.numpy().view(dt).reshape(s1.shape), V.astype(dt))
    # a device potential is copied into the pinned buffer as well
    s1.set_potential(torch.from_numpy(2.0 * V).to("cuda:0"))
    assert np.array_equal(s1.host_v.numpy().view(dt).reshape(s1.shape), (2.0 * V).astype(dt))
    s0.close()
    s1.close()


def test_unpinned_host_arrays_are_refused(gpu_lib):
    import torch
    w = CASES["3d_24x20x16"]
    banner("host-resident V: refusals")
    prm = B.make_params(**{**w, "prec": "fp64"})
    nbytes = B.gp_workspace_bytes_ex(prm, B.GP_HOST_V)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:0")
    ptr = (ws.data_ptr() + 255) & ~255
    vb, _ = B.gp_host_bytes(prm)
    pageable = np.zeros(vb // 8, dtype=np.float64)         # ordinary (pageable) memory
    st = torch.cuda.current_stream().cuda_stream
    for hv in (0, pageable.ctypes.data):
        with pytest.raises(B.GPError) as e:
            B.gp_init_ex(prm, B.GP_HOST_V, ptr, nbytes, hv, 0, st)
        assert e.value.status == B.GP_E_ARG
    pinned = torch.empty(vb, dtype=torch.uint8, pin_memory=True)
    with pytest.raises(B.GPError) as e:                       # misaligned
        B.gp_init_ex(prm, B.GP_HOST_V, ptr, nbytes, pinned.data_ptr() + 8, 0, st)
    assert e.value.status == B.GP_E_ARG
    ctx = B.gp_init_ex(prm, B.GP_HOST_V, ptr, nbytes, pinned.data_ptr(), 0, st)
    B.gp_destroy(ctx)


def test_adjoint_with_host_potential(gpu_lib):
    import torch
    from paper_1601_04640_amd.binding import Solver
    w = CASES["2dxy_48x40"]
    banner("host-resident V: adjoint step")
    p = oparams(w)
    psi = I.random_complex(p.shape(), 704, p.dV())
    lam0 = I.random_complex(p.shape(), 705, p.dV())
    outs = []
    for host in ((), ("V", "ktab")):
        s = Solver(w, prec="fp64", host=host)
        s.set_psi(psi)
        pd = torch.from_numpy(psi).to("cuda:0")
        lam = torch.from_numpy(lam0).to("cuda:0")
        gv = torch.zeros(s.shape, dtype=torch.float64, device="cuda:0")
        gg = torch.zeros(2, dtype=torch.float64, device="cuda:0")
        B.gp_step_real_adjoint(s.ctx, pd.data_ptr(), lam.data_ptr(), gv.data_ptr(),
                               gg.data_ptr(), gg.data_ptr() + 8)
        torch.cuda.synchronize()
        outs.append((lam.cpu().numpy(), gv.cpu().numpy(), gg.cpu().numpy()))
        s.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
