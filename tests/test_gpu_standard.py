"""GPU parity of the standard lattice Boltzmann comparator (mode "standard", Sec. I, Eq. 4)
against the oracle, through the C ABI.

Bars: FP64 storage <= 1e-12 and FP32 <= 1e-5 relative L2 on the populations and on rho, u;
16-bit deviation storage within the code's rounding (rel. L2 1e-3 for binary16, 1e-2 for
bfloat16 after 20 steps).  The prescribed temperature is a non-uniform field (kept per site),
or uniform (kept as one constant).
"""
import numpy as np
import pytest

import oracle
from paper_2501_00620_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def lbm():
    from paper_2501_00620_amd import lbm as m
    return m


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def run_pair(dims, storage, steps, uniform_T=False, tau=0.7, seed=5):
    nx, ny, nz = dims
    rho, u, T = wl.fourier_fields(nx, ny, nz, seed=seed, u_max=0.2)
    if uniform_T:
        T = np.full_like(T, 0.3)
    g = lbm().Lattice(nx, ny, nz, tau, storage=storage, mode="standard")
    g.set_fields(rho, u, T)
    o = oracle.OracleLattice(nx, ny, nz, tau, mode="standard")
    o.init(rho, u, T)
    g.step(steps)
    o.step(steps)
    F, _ = g.get_state()
    r, uu, TT = g.moments()
    ro, uo, To = o.moments()
    errs = {"F": rel_l2(F.cpu().numpy(), o.F), "rho": rel_l2(r.cpu().numpy(), ro),
            "u": rel_l2(uu.cpu().numpy(), uo), "T": rel_l2(TT.cpu().numpy(), To)}
    print(dims, storage, steps, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    return errs


@pytest.mark.parametrize("dims", [(17, 9, 5), (32, 32, 1), (8, 6, 2), (65, 3, 4)])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_standard_parity(dims, storage, tol):
    errs = run_pair(dims, storage, 30)
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_standard_parity_uniform_temperature(storage, tol):
    errs = run_pair((24, 20, 6), storage, 40, uniform_T=True)
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("storage,tol", [("f16dev", 1e-3), ("bf16dev", 1e-2)])
def test_standard_16bit_storage(storage, tol):
    errs = run_pair((24, 20, 6), storage, 20)
    assert max(errs.values()) <= tol, errs


def test_standard_conserves_mass_and_momentum():
    dims = (16, 12, 10)
    rho, u, T = wl.fourier_fields(*dims, seed=8, u_max=0.2)
    g = lbm().Lattice(*dims, 0.6, storage="f64", mode="standard")
    g.set_fields(rho, u, T)
    i0 = g.invariants()
    g.step(200)
    i1 = g.invariants()
    assert abs(i1[0] / i0[0] - 1) < 1e-13
    assert np.abs(i1[1:4] - i0[1:4]).max() < 1e-13 * i0[0]
