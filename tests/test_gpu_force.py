"""GPU parity of the body force (lbm_set_body_force) against the oracle, through the C ABI.

Bars: FP64 storage <= 1e-12 and FP32 <= 1e-5 relative L2 on the state and the moments; exact
momentum growth under a uniform force; the Kolmogorov-flow amplitude A / (T tau k^2) within 0.5%.
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


def force_field(dims, seed, amp=2e-4):
    _, a, _ = wl.fourier_fields(*dims, seed=seed, u_max=1.0)
    return amp * a


@pytest.mark.parametrize("kernel", ["auto", "two_pass"])
@pytest.mark.parametrize("dims", [(17, 9, 5), (32, 16, 1), (8, 6, 7)])
@pytest.mark.parametrize("mode", ["thermal", "iso", "standard"])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_body_force_parity(dims, mode, storage, tol, kernel):
    # kernel "auto" steps a periodic lattice with the fused sweep (STANDARD: its own kernel)
    tau, steps = 0.7, 30
    fields = wl.fourier_fields(*dims, seed=23, u_max=0.2)
    accel = force_field(dims, 24)
    g = lbm().Lattice(*dims, tau, storage=storage, mode=mode, kernel=kernel)
    g.set_fields(*fields)
    g.set_body_force(accel)
    o = oracle.OracleLattice(*dims, tau, mode=mode)
    o.init(*fields)
    o.set_body_force(accel)
    g.step(steps)
    o.step(steps)
    F, b = g.get_state()
    r, u, T = g.moments()
    ro, uo, To = o.moments()
    errs = {"F": rel_l2(F.cpu().numpy(), o.F), "b": rel_l2(b.cpu().numpy(), o.b),
            "rho": rel_l2(r.cpu().numpy(), ro), "u": rel_l2(u.cpu().numpy(), uo), "T": rel_l2(T.cpu().numpy(), To)}
    assert max(errs.values()) <= tol, errs


def test_uniform_force_momentum_on_gpu():
    dims = (12, 10, 8)
    g = lbm().Lattice(*dims, 0.7, storage="f64")
    g.set_fields(*wl.fourier_fields(*dims, seed=6, u_max=0.1))
    a = np.array([1e-4, -2e-4, 3e-5])
    g.set_body_force(a)
    i0 = g.invariants()
    g.step(100)
    i1 = g.invariants()
    np.testing.assert_allclose(i1[1:4] - i0[1:4], 100 * i0[0] * a, rtol=0, atol=1e-11)
    assert abs(i1[0] / i0[0] - 1) < 1e-14


def test_kolmogorov_flow_on_gpu():
    N, tau, T0, A = 64, 0.6, 0.2, 1e-6
    k = 2 * np.pi / N
    x = np.arange(N)
    g = lbm().Lattice(N, 1, 1, tau, storage="f64", mode="iso")
    g.set_fields(np.ones((1, 1, N)), np.zeros((3, 1, 1, N)), np.full((1, 1, N), T0))
    accel = np.zeros((3, 1, 1, N))
    accel[1, 0, 0] = A * np.sin(k * x)
    g.set_body_force(accel)
    g.step(8000)
    uy = g.moments()[1][1].cpu().numpy().reshape(N)
    amp = 2.0 / N * np.sum(uy * np.sin(k * x))
    assert abs(amp / (A / (T0 * tau * k * k)) - 1) < 0.005


def test_removing_the_force_restores_the_fused_step():
    dims = (20, 9, 6)
    fields = wl.fourier_fields(*dims, seed=3, u_max=0.2)
    out = []
    for with_force in (False, True):
        g = lbm().Lattice(*dims, 0.7, storage="f64")
        g.set_fields(*fields)
        if with_force:
            g.set_body_force(force_field(dims, 5))
            g.set_body_force(None)
        g.step(10)
        out.append(g.get_state()[0].cpu().numpy())
    np.testing.assert_array_equal(out[0], out[1])


@pytest.mark.parametrize("dims", [(70, 9, 11), (70, 33, 1), (45, 20, 2), (70, 9, 37)])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "bf16dev"])
def test_fused_equals_two_pass_with_force(storage, dims):
    # the fused sweep adds the force where the two-pass collision does: equal up to the order of
    # the gradient sums, as without a force
    fields = wl.fourier_fields(*dims, seed=12, u_max=0.25)
    accel = force_field(dims, 13)
    out = []
    kernels = ("fused", "two_pass") + (("fused_pc",) if storage != "f64" and dims[2] >= 3 else ())
    for kernel in kernels:
        g = lbm().Lattice(*dims, 0.65, storage=storage, kernel=kernel)
        g.set_fields(*fields)
        g.set_body_force(accel)
        g.step(7)
        F, b = g.get_state()
        out.append((F.cpu().numpy(), b.cpu().numpy()))
    tol = {"f64": 1e-14, "f32": 1e-6, "f16dev": 1e-3, "bf16dev": 1e-2}[storage]
    for k in (0, 2)[:len(out) - 1]:
        assert rel_l2(out[k][0], out[1][0]) <= tol, kernels[k]
        assert rel_l2(out[k][1], out[1][1]) <= tol, kernels[k]
    # and the force changes the result by far more than the bar (the comparison is not vacuous;
    # over 7 steps the force moves the state by ~1e-4, under the 16-bit bars, so checked where
    # the bar is tight)
    if storage in ("f64", "f32"):
        g = lbm().Lattice(*dims, 0.65, storage=storage, kernel="fused")
        g.set_fields(*fields)
        g.step(7)
        assert rel_l2(g.get_state()[0].cpu().numpy(), out[0][0]) > 10 * tol


def test_body_force_argument_errors():
    L = lbm()
    g = L.Lattice(8, 8, 1, 0.7, storage="f32")
    g.set_projection(2)
    with pytest.raises(L.LBMError):
        g.set_body_force([1e-4, 0, 0])
    # the fused sweep takes a force, and a force does not prevent choosing it
    g = L.Lattice(8, 8, 8, 0.7, storage="f32", kernel="fused")
    g.set_body_force([1e-4, 0, 0])
    g.set_kernel("fused")


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("kernel", ["fused", "fused_pc", "two_pass"])
@pytest.mark.parametrize("mode", ["thermal", "iso", "standard"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
def test_uniform_force_equals_the_same_field(kernel, mode, storage, walls):
    # lbm_set_body_force_uniform: the forcing of a field holding the vector at every site, bit for
    # bit, in every kernel that takes a force (and the readout of the moments); with walls the
    # split sweep's interior planes and the wall kernel's wall planes
    if kernel == "fused_pc" and (storage == "f64" or mode == "standard"):
        pytest.skip("the split sweep has no double-precision instantiation; STANDARD steps its own kernel")
    if kernel == "fused" and (mode == "standard" or walls):
        pytest.skip("STANDARD steps its own kernel; the single-role sweep is periodic")
    dims = (19, 10, 6)
    fields = wl.fourier_fields(*dims, seed=51, u_max=0.15)
    a = [2e-4, -1e-4, 3e-4]
    out = []
    for field in (False, True):
        g = lbm().Lattice(*dims, 0.7, storage=storage, mode=mode, kernel=kernel)
        g.set_fields(*fields)
        if walls:
            g.set_walls([0.01, 0.0, 0.0], [0.0, -0.02, 0.0])
        g.set_body_force(a, field=field)
        g.step(7)
        F, b = g.get_state()
        r, u, T = g.moments()
        out.append([q.cpu().numpy() for q in (F, b, r, u, T)])
    for x, y in zip(*out):
        np.testing.assert_array_equal(x, y)


def test_uniform_force_replaces_and_is_replaced():
    L = lbm()
    dims = (12, 10, 8)
    fields = wl.fourier_fields(*dims, seed=52, u_max=0.1)

    def run(setup):
        g = L.Lattice(*dims, 0.7, storage="f32")
        g.set_fields(*fields)
        setup(g)
        g.step(5)
        return g.get_state()[0].cpu().numpy()

    plain = run(lambda g: None)
    # set, then removed: the force-free step
    np.testing.assert_array_equal(run(lambda g: (g.set_body_force([1e-4, 0, 0]), g.set_body_force(None))), plain)
    # a field replaces the uniform force, and the uniform force a field
    field = run(lambda g: g.set_body_force([0, 2e-4, 0], field=True))
    np.testing.assert_array_equal(run(lambda g: (g.set_body_force([1e-4, 0, 0]), g.set_body_force([0, 2e-4, 0], field=True))), field)
    np.testing.assert_array_equal(run(lambda g: (g.set_body_force(np.full((3,) + dims[::-1], 1e-3)), g.set_body_force([0, 2e-4, 0]))), field)
    p = L.Lattice(8, 8, 1, 0.7, storage="f32")
    p.set_projection(2)
    with pytest.raises(L.LBMError):
        p.set_body_force([1e-4, 0, 0])
    q = L.Lattice(8, 8, 8, 0.7, storage="f32")
    with pytest.raises(L.LBMError):
        q.set_body_force([float("nan"), 0, 0])
