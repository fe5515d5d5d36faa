"""GPU parity of the walls (lbm_set_walls: half-way bounce-back with moving walls, the channels
of Sec. III A and C) against the oracle, through the C ABI, in the bump scheme and the standard
comparator, with and without a body force; the split fused sweep with walls (interior planes in
the sweep, the wall planes with the two-pass wall kernel) against the two-pass step.

Bars: FP64 storage <= 1e-12 and FP32 <= 1e-5 relative L2 on the state and the moments; exact
mass conservation and the steady linear Couette profile on the GPU; the Poiseuille viscosity.
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


UB, UT = [0.02, -0.01, 0.0], [-0.015, 0.03, 0.0]


@pytest.mark.parametrize("dims", [(17, 9, 5), (32, 16, 3), (8, 6, 7)])
@pytest.mark.parametrize("mode", ["thermal", "iso", "standard"])
@pytest.mark.parametrize("force", [False, True])
@pytest.mark.parametrize("storage,tol,kernel", [("f64", 1e-12, "auto"), ("f32", 1e-5, "auto"),
                                                ("f32", 1e-5, "two_pass")])
def test_walls_parity(dims, mode, force, storage, tol, kernel):
    # "auto": FP64 steps two-pass; FP32 steps its interior planes in the split fused sweep (from
    # the second step on) and its wall planes with the wall kernel
    tau, steps = 0.7, 30
    fields = wl.fourier_fields(*dims, seed=31, u_max=0.2)
    g = lbm().Lattice(*dims, tau, storage=storage, mode=mode, kernel=kernel)
    g.set_fields(*fields)
    g.set_walls(UB, UT)
    o = oracle.OracleLattice(*dims, tau, mode=mode)
    o.init(*fields)
    o.set_walls(UB, UT)
    if force:
        _, a, _ = wl.fourier_fields(*dims, seed=32, u_max=1.0)
        a = 2e-4 * a + np.array([0.0, 0.0, -1e-3]).reshape(3, 1, 1, 1)
        g.set_body_force(a)
        o.set_body_force(a)
    g.step(steps)
    o.step(steps)
    F, b = g.get_state()
    r, u, T = g.moments()
    ro, uo, To = o.moments()
    errs = {"F": rel_l2(F.cpu().numpy(), o.F), "rho": rel_l2(r.cpu().numpy(), ro), "u": rel_l2(u.cpu().numpy(), uo)}
    if mode != "standard":
        errs["b"] = rel_l2(b.cpu().numpy(), o.b)
        errs["T"] = rel_l2(T.cpu().numpy(), To)
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_walls_with_16bit_storage(storage):
    # the bounced population is encoded with the codec scale of the slot it lands in; 16-bit
    # storage stays within its rounding of the FP32 run and keeps the mass
    dims = (24, 12, 10)
    fields = wl.fourier_fields(*dims, seed=34, u_max=0.1)
    out = {}
    for st in ("f32", storage):
        g = lbm().Lattice(*dims, 0.7, storage=st)
        g.set_fields(*fields)
        g.set_walls(UB, UT)
        g.set_body_force([0.0, 1e-4, -1e-4])
        m0 = g.get_state()[0].sum().item()
        g.step(40)
        out[st] = [q.cpu().numpy() for q in g.moments()]
        out[st + "_mass"] = abs(g.get_state()[0].sum().item() / m0 - 1)
    # bars in units of the code's unit roundoff r (2^-11 FP16, 2^-8 BF16); measured: rho 1.5e-6 /
    # 1.3e-5, u 1.0e-4 / 8.4e-4, as for the periodic lattice.  A bounced population decoded with
    # another slot's scale would be off by a power of two.
    r = 2.0 ** -11 if storage == "f16dev" else 2.0 ** -8
    assert rel_l2(out[storage][0], out["f32"][0]) < 0.2 * r
    assert rel_l2(out[storage][1], out["f32"][1]) < 4 * r
    assert out[storage + "_mass"] < 1e-5


def test_walls_with_ghost_relaxation():
    dims = (12, 7, 6)
    fields = wl.fourier_fields(*dims, seed=33, u_max=0.2)
    g = lbm().Lattice(*dims, 0.65, storage="f64")
    g.set_ghost_relaxation(0.5)
    g.set_fields(*fields)
    g.set_walls(UB, UT)
    o = oracle.OracleLattice(*dims, 0.65, tau_ghost=0.5)
    o.init(*fields)
    o.set_walls(UB, UT)
    g.step(25)
    o.step(25)
    assert rel_l2(g.get_state()[0].cpu().numpy(), o.F) <= 1e-12


@pytest.mark.parametrize("mode", ["thermal", "iso", "standard"])
def test_mass_is_conserved_on_gpu(mode):
    dims = (16, 12, 10)
    g = lbm().Lattice(*dims, 0.7, storage="f64", mode=mode)
    g.set_fields(*wl.fourier_fields(*dims, seed=5, u_max=0.1))
    g.set_walls(UB, UT)
    g.set_body_force([1e-4, 0.0, -1e-3])
    m0 = g.get_state()[0].sum().item()
    g.step(100)
    assert abs(g.get_state()[0].sum().item() / m0 - 1) < 1e-13


def test_couette_is_linear_on_gpu():
    nz, tau, T0, U = 16, 0.8, 0.25, 0.02
    zp = np.arange(nz) + 0.5
    u = np.zeros((3, nz, 1, 1))
    u[1, :, 0, 0] = 2 * U * zp / nz
    g = lbm().Lattice(1, 1, nz, tau, storage="f64", mode="iso")
    g.set_fields(np.ones((nz, 1, 1)), u, np.full((nz, 1, 1), T0))
    g.set_walls(None, [0, 2 * U, 0])
    g.step(2000)
    uy = g.moments()[1][1].cpu().numpy().reshape(nz)
    np.testing.assert_allclose(uy, 2 * U * zp / nz, rtol=0, atol=1e-12)


def test_poiseuille_viscosity_on_gpu():
    nz, tau, T0, a = 21, 0.5, 0.2, 1e-5
    nu = T0 * tau
    zp = np.arange(nz) + 0.5
    u = np.zeros((3, nz, 1, 1))
    u[1, :, 0, 0] = a / (2 * nu) * zp * (nz - zp)
    g = lbm().Lattice(1, 1, nz, tau, storage="f64", mode="iso")
    g.set_fields(np.ones((nz, 1, 1)), u, np.full((nz, 1, 1), T0))
    g.set_walls()
    g.set_body_force([0.0, a, 0.0])
    g.step(int(3 * nz * nz / nu))
    r, u, _ = g.moments()
    eta = r.mean().item() * a * nz ** 2 / (8 * u[1].max().item())
    assert abs(eta / (r.mean().item() * T0 * tau) - 1) < 5e-3


def test_walls_off_restores_the_periodic_fused_step():
    dims = (20, 9, 6)
    fields = wl.fourier_fields(*dims, seed=3, u_max=0.2)
    out = []
    for with_walls in (False, True):
        g = lbm().Lattice(*dims, 0.7, storage="f64")
        g.set_fields(*fields)
        if with_walls:
            g.set_walls(UB, UT)
            g.set_walls(on=False)
        g.step(10)
        out.append(g.get_state()[0].cpu().numpy())
    np.testing.assert_array_equal(out[0], out[1])


def test_wall_argument_errors():
    L = lbm()
    g = L.Lattice(8, 8, 2, 0.7, storage="f32")
    with pytest.raises(L.LBMError):
        g.set_walls()  # nz < 3
    g = L.Lattice(8, 8, 8, 0.7, storage="f32")
    with pytest.raises(L.LBMError):
        g.set_walls([0, 0, 0.01], None)  # normal wall velocity
    with pytest.raises(L.LBMError):
        g.set_walls([float("nan"), 0, 0], None)
    g.set_walls()
    with pytest.raises(L.LBMError):
        g.set_kernel("fused")  # the single-role sweep is periodic
    g.set_kernel("fused_pc")  # the split sweep takes walls
    f = L.Lattice(8, 8, 8, 0.7, storage="f32", kernel="fused")
    with pytest.raises(L.LBMError):
        f.set_walls()
    d = L.Lattice(8, 8, 8, 0.7, storage="f64")
    d.set_walls()
    with pytest.raises(L.LBMError):
        d.set_kernel("fused_pc")  # double precision steps two-pass


@pytest.mark.parametrize("dims", [(17, 9, 5), (32, 16, 3), (70, 13, 37)])
@pytest.mark.parametrize("tau_g", [None, 0.5])
@pytest.mark.parametrize("storage,tol", [("f32", 1e-6), ("f16dev", 1e-3), ("bf16dev", 1e-2)])
def test_split_sweep_with_walls_equals_two_pass(dims, tau_g, storage, tol):
    # Moving walls, a body force and (or not) a ghost rate: the split sweep over the interior
    # planes (the wall planes with the wall kernel) against the two-pass step, in every storage it
    # takes.  The same arithmetic up to the order of the gradient sums (the bars of the periodic
    # comparison).  nz = 37 sweeps the 35 interior planes in two z chunks; nz = 3 leaves one
    # interior plane, nz = 5 three.
    fields = wl.fourier_fields(*dims, seed=41, u_max=0.2)
    _, a, _ = wl.fourier_fields(*dims, seed=42, u_max=1.0)
    a = 2e-4 * a + np.array([0.0, 0.0, -1e-3]).reshape(3, 1, 1, 1)
    out = []
    for kernel in ("two_pass", "fused_pc"):
        g = lbm().Lattice(*dims, 0.7, storage=storage, kernel=kernel)
        g.set_fields(*fields)
        g.set_walls(UB, UT)
        g.set_body_force(a)
        if tau_g is not None:
            g.set_ghost_relaxation(tau_g)
        g.step(9)
        assert g.health()[:2] == (0, 0)
        F, b = g.get_state()
        out.append((F.cpu().numpy(), b.cpu().numpy()))
    assert rel_l2(out[1][0], out[0][0]) <= tol, rel_l2(out[1][0], out[0][0])
    assert rel_l2(out[1][1], out[0][1]) <= tol, rel_l2(out[1][1], out[0][1])


def test_split_sweep_wall_channel_mass_and_couette():
    # FP32 Couette channel in the split sweep: exact mass conservation with walls at rest, and the
    # steady linear profile between a wall at rest and one moving at U (the two-pass bar)
    L = lbm()
    nz, U, T0 = 12, 0.02, 0.25
    g = L.Lattice(4, 4, nz, 0.8, storage="f32", mode="iso", kernel="fused_pc")
    g.set_fields(np.ones((nz, 4, 4)), np.zeros((3, nz, 4, 4)), np.full((nz, 4, 4), T0))
    g.set_walls([0, 0, 0], [U, 0, 0])
    m0 = g.get_state()[0].sum().item()
    g.step(6000)
    assert abs(g.get_state()[0].sum().item() / m0 - 1) < 1e-6
    u = g.moments()[1][0].cpu().numpy().mean(axis=(1, 2))
    z = np.arange(nz) + 0.5
    assert np.abs(u - U * z / nz).max() <= 1e-3 * U, u - U * z / nz


@pytest.mark.parametrize("mode", ["thermal", "iso"])
def test_f32_channel_long_horizon(mode):
    # The FP32 path with walls over a long run: a 32 x 16 x 24 channel between walls moving in
    # different directions, under a uniform acceleration with a component along the wall normal
    # (a hydrostatic layer), 1000 steps; the split sweep (interior planes, wall planes with the
    # wall kernel) and the two-pass step against one oracle run.  The flow keeps the walls'
    # shear, so u does not decay to round-off.  Measured: u within 2e-7, F within 1e-8.
    dims, tau, steps = (32, 16, 24), 0.6, 1000
    acc = [1e-5, 2e-5, -1e-4]
    fields = wl.fourier_fields(*dims, seed=61, u_max=0.1)
    o = oracle.OracleLattice(*dims, tau, mode=mode)
    o.init(*fields)
    o.set_walls(UB, UT)
    o.set_body_force(np.broadcast_to(np.array(acc).reshape(3, 1, 1, 1), (3,) + dims[::-1]).copy())
    o.step(steps)
    ro, uo, To = o.moments()
    for kernel in ("auto", "two_pass"):
        g = lbm().Lattice(*dims, tau, storage="f32", mode=mode, kernel=kernel)
        g.set_fields(*fields)
        g.set_walls(UB, UT)
        g.set_body_force(acc)
        g.step(steps)
        F, b = g.get_state()
        r, u, T = g.moments()
        errs = {"F": rel_l2(F.cpu().numpy(), o.F), "rho": rel_l2(r.cpu().numpy(), ro),
                "u": rel_l2(u.cpu().numpy(), uo), "T": rel_l2(T.cpu().numpy(), To),
                "b_on_T_scale": float(np.linalg.norm(b.cpu().numpy() - o.b) / np.linalg.norm(To))}
        assert max(errs.values()) <= 1e-5, (kernel, errs)
        g.close()
