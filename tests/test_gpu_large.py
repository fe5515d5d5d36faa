"""GPU parity at the largest workload: 512^3 random smooth fields (rho = 1 +- 0.05, |u| <= 0.3,
T in [0.9, 1.1] T_ref; tau = 0.6), stepped by the fused sweep in the launch configuration the
bench times, in FP32 and FP16-deviation storage.

At this size a plane offset inside a buffer group reaches 2^31 bytes, so these cases cover the
sweep's unsigned offset arithmetic.  The oracle cannot run the lattice, so single steps are
checked on sampled sites, as in the full-size checks of test_gpu_parity: the oracle steps a
5x5x5 periodic copy of each site's neighbourhood cut out of the GPU state.  The samples include
the last plane, the box corners and the middle plane.
"""
import functools

import numpy as np
import pytest

from paper_2501_00620_amd import workloads as wl
from test_gpu_parity import _check_stored_bound, lbm, rel_l2, sampled_one_step

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 512
TAU = 0.6


@functools.lru_cache(maxsize=1)
def fields():
    return wl.fourier_fields(N, N, N, seed=5)


def sample_sites():
    rng = np.random.default_rng(3)
    sites = rng.integers(0, N ** 3, size=48)
    n2 = N * N
    corners = [0, N - 1, n2 - N, n2 - 1, (N - 1) * n2, (N - 1) * n2 + N - 1, N ** 3 - N, N ** 3 - 1]
    sites[:8] = corners
    sites[8:16] = (N - 1) * n2 + rng.integers(0, n2, size=8)  # the last plane
    sites[16:20] = (N // 2) * n2 + rng.integers(0, n2, size=4)  # the middle plane
    return sites


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_512_cubed_sampled_steps(storage):
    rho, u, T = fields()
    print(f"512^3 {storage}: set_fields", flush=True)
    g = lbm().Lattice(N, N, N, TAU, storage=storage)  # kernel choice as the bench runs it
    g.set_fields(rho, u, T)
    g.step(4)
    if storage == "f32":
        scales, refs = np.ones(25), np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12 + [0.0] * 6)
    else:
        scales, refs = g.codec()
    print(f"512^3 {storage}: sampled step", flush=True)
    Fg, bg, Fo, bo, bsg, bso = sampled_one_step(g, TAU, "thermal", sample_sites())
    if storage == "f32":
        assert rel_l2(Fg, Fo) <= 1e-6, rel_l2(Fg, Fo)
        assert rel_l2(bsg, bso) <= 1e-5, rel_l2(bsg, bso)
    _check_stored_bound(storage, Fg, Fo, bsg, bso, scales, refs)
    assert g.health()[:2] == (0, 0)
    g.close()
    torch.cuda.empty_cache()
