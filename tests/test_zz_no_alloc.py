"""The allocation-free entry point gp_dipolar_potential_noalloc against gp_dipolar_potential
(the context entry point it mirrors) and the FP64 oracle, through the C ABI: two calls in
a row on one device, the second with a smaller grid, in both precisions; and a grid past
the scratch limit rejected on the host."""
import numpy as np
import pytest

import oracle as O
from paper_1601_04640_amd import binding as B
from paper_1601_04640_amd import inputs as I
from tests.gpu_util import banner, oparams, rel_l2

pytestmark = pytest.mark.gpu

BIG = dict(geom="3d", nx=40, ny=30, nz=48, dx=0.3, dy=0.35, dz=0.25, dt=0.001, gamma=1.0,
           nu=1.1, lam=1.8, g=30.0, gdd=12.0, R=5.0)
SMALL = dict(geom="2dxz", nx=30, ny=1, nz=64, dx=0.4, dy=1.0, dz=0.2, dt=0.001, gamma=1.0,
             nu=4.0, lam=2.5, g=20.0, gdd=15.0, R=0.0)


def noalloc_phi(w, prec, psi_dev, torch):
    s_shape = B._shape(w)
    rdt = torch.float64 if prec == "fp64" else torch.float32
    phi = torch.full(s_shape, float("nan"), dtype=rdt, device="cuda:0")
    st = torch.cuda.current_stream()
    B.gp_dipolar_potential_noalloc(B.make_params(**{**w, "prec": prec}), psi_dev.data_ptr(),
                                   phi.data_ptr(), st.cuda_stream)
    st.synchronize()
    return phi.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_context_call(prec, gpu_lib):
    import torch
    from paper_1601_04640_amd.binding import Solver
    for k, w in enumerate((BIG, SMALL)):       # the second call is smaller
        banner("dipolar_potential_noalloc", w["geom"], w["nx"], w["ny"], w["nz"], prec)
        p = oparams(w)
        psi = I.random_complex(p.shape(), 300 + k, p.dV())
        s = Solver(w, prec=prec)
        s.set_psi(psi)
        ref_ctx = s.dipolar_potential()
        psi_dev = torch.from_numpy(psi).to("cuda:0", s.cdtype)
        got = noalloc_phi(w, prec, psi_dev, torch)
        s.close()
        # same kernels on the same input: equal to the context call
        assert np.all(np.isfinite(got))
        assert rel_l2(got, ref_ctx) <= (1e-15 if prec == "fp64" else 1e-7), rel_l2(got, ref_ctx)
        # and to the oracle at the dipolar-potential bars of the parity tests (the FP32 input
        # is psi rounded to float, which the oracle sees in FP64)
        psi_in = psi if prec == "fp64" else psi.astype(np.complex64).astype(np.complex128)
        ref = O.dipolar_potential(np.abs(psi_in) ** 2, p)
        assert rel_l2(got, ref) <= (1e-12 if prec == "fp64" else 2e-6), rel_l2(got, ref)


def test_noalloc_rejects_grid_past_scratch(gpu_lib):
    import torch
    w = dict(BIG, nx=256, ny=256, nz=256, dx=0.1, dy=0.1, dz=0.1)
    x = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    with pytest.raises(B.GPError) as e:
        B.gp_dipolar_potential_noalloc(B.make_params(**{**w, "prec": "fp64"}), x.data_ptr(),
                                       x.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert e.value.status == B.GP_E_SIZE
    assert "scratch" in str(e.value)
