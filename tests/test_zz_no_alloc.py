"""nlse_mass_energy_noalloc (the entry point that allocates nothing) against
nlse_mass_energy of a grid on the same field: the same bits, on two calls in a
row with the second on a smaller field, and against the FP64 oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1203_1263_amd import workloads as wl
from gpu_util import to_dev, pot_dev

pytestmark = pytest.mark.gpu

ORDER = {"cd2": 2, "2shoc": 4}


def _field(shape, index, with_v):
    u = 1.5 + 0.4 * wl.random_field(shape, index, smooth=2.0)
    V = 0.3 * wl.random_field(shape, index, stream=1, smooth=3.0).real if with_v else None
    return u, V


def _both(u, V, dtype, h, a, s, order, bc):
    """(no-alloc result, grid result) on one device field."""
    import torch
    from paper_1203_1263_amd import nlse
    from paper_1203_1263_amd.nlse import Grid
    psi, Vd = to_dev(u, dtype), pot_dev(V, dtype)
    dims = list(reversed(u.shape)) + [1] * (3 - u.ndim)
    st = torch.cuda.current_stream()
    got = nlse.nlse_mass_energy_noalloc(u.ndim, dims, h, a, s, nlse.NLSE_F32 if dtype == "f32" else nlse.NLSE_F64,
                                        order, nlse.BC[bc], psi.data_ptr(),
                                        Vd.data_ptr() if Vd is not None else None, st.cuda_stream)
    g = Grid(psi, h, a, s, V=Vd)
    ref = g.mass_energy(order, bc)
    g.close()
    return got, ref


PAIRS = [((9, 40, 70), (7, 5, 66)), ((150, 137), (37, 150)), ((5000,), (600,)), ((256, 256, 256), (21, 13, 70))]


@pytest.mark.parametrize("big,small", PAIRS, ids=["x".join(map(str, p[0])) for p in PAIRS])
@pytest.mark.parametrize("scheme,bc", [("cd2", "dirichlet"), ("2shoc", "msd"), ("2shoc", "dirichlet"),
                                       ("2shoc", "l0")])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_equals_grid_mass_energy(big, small, scheme, bc, dtype):
    if big == (256, 256, 256) and (dtype == "f64" or bc != "msd"):
        pytest.skip("one full-size case (FP32, 2SHOC + MSD) is enough")
    h, a, s = 0.3, 0.7, -0.9
    order = ORDER[scheme]
    for k, shape in enumerate((big, small)):
        u, V = _field(shape, 70 + k, with_v=(k == 0))
        (Mn, En), (Mg, Eg) = _both(u, V, dtype, h, a, s, order, bc)
        print(f"{dtype} {scheme}+{bc} {shape}: noalloc ({Mn!r}, {En!r}) grid ({Mg!r}, {Eg!r})")
        assert (Mn, En) == (Mg, Eg)
        if np.prod(shape) <= 200_000:
            uu = u.astype(np.complex64).astype(np.complex128) if dtype == "f32" else u
            VV = None if V is None else (V.astype(np.float32).astype(np.float64) if dtype == "f32" else V)
            Mr, Er = oracle.mass_energy(uu, h, a, s, V=VV, order=order, bc=bc)
            assert Mn == pytest.approx(Mr, rel=1e-12)
            assert En == pytest.approx(Er, rel=1e-11, abs=1e-11 * abs(Mr))


def test_noalloc_rejects_a_field_beyond_the_scratch():
    import torch
    from paper_1203_1263_amd import nlse
    psi = torch.zeros(16, dtype=torch.complex64, device="cuda")
    with pytest.raises(nlse.NLSEError) as e:
        nlse.nlse_mass_energy_noalloc(3, [1024, 1024, 257], 0.1, 1.0, 1.0, nlse.NLSE_F32, 2, nlse.NLSE_BC_DIRICHLET,
                                      psi.data_ptr(), None, None)
    assert e.value.code == nlse.NLSE_EINVAL
    assert "static scratch" in str(e.value)
