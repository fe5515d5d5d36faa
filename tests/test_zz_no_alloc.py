"""lbm_invariants_noalloc (include/lbm.h): the invariants of lbm_invariants with no device
allocation, its partial sums in a static scratch array per GPU.  Checked through the C ABI
against lbm_invariants on the same lattice, to the bit, with the device and the host output, on
two calls in a row, the second on a smaller lattice (the shared scratch keeps the first call's
partials, which the second must not pick up)."""
import ctypes as C

import numpy as np
import pytest

from paper_2501_00620_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def lbm():
    from paper_2501_00620_amd import lbm as m
    return m


def _lattice(dims, storage, steps, seed):
    g = lbm().Lattice(*dims, 0.7, storage=storage)
    rho, u, T = wl.fourier_fields(*dims, seed=seed, u_max=0.2)
    g.set_fields(rho, u + np.array([0.03, -0.02, 0.01]).reshape(3, 1, 1, 1), T)
    g.step(steps)
    return g


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
def test_noalloc_invariants_equal_lbm_invariants(storage):
    lib = lbm().load_library()
    # the larger lattice fills all 1024 partial slots; the smaller uses 9 of them
    for dims, steps, seed in (((96, 80, 40), 6, 1), ((17, 11, 12), 3, 2)):
        g = _lattice(dims, storage, steps, seed)
        ref = g.invariants()
        out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
        rc = lib.lbm_invariants_noalloc(g.handle, C.c_void_p(out.data_ptr()), 1)
        assert rc == 0, lib.lbm_last_error()
        g.sync()
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
        host = (C.c_double * 5)(*([float("nan")] * 5))
        rc = lib.lbm_invariants_noalloc(g.handle, C.cast(host, C.c_void_p), 0)
        assert rc == 0, lib.lbm_last_error()
        np.testing.assert_array_equal(np.array(host[:]), ref)
        np.testing.assert_array_equal(g.invariants_noalloc(), ref)
        g.close()


def test_noalloc_argument_errors():
    lib = lbm().load_library()
    g = lbm().Lattice(8, 8, 8, 0.7, storage="f32")
    host = (C.c_double * 5)()
    assert lib.lbm_invariants_noalloc(g.handle, C.cast(host, C.c_void_p), 0) == -7  # STATE: no fields yet
    assert lib.lbm_invariants_noalloc(g.handle, None, 0) == -1
    g.close()
