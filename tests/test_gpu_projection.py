"""GPU parity of the projected lattices (lbm_set_projection: D2Q9 for nx x ny x 1, D1Q3 for
nx x 1 x 1, held as class sums) against the D3Q19 oracle on the same lattice, through the C ABI.

Bars: FP64 storage <= 1e-12 and FP32 <= 1e-5 relative L2 on the moments and on the state
contracted to classes (oracle.project); the projected GPU step equals the D3Q19 GPU step on the
same lattice to 1e-13 (FP64); the Sod shock tube (400 x 1 x 1, 1000 steps) as D1Q3 against the
oracle.
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


def planar_fields(nx, ny, seed, u_max=0.2):
    rho, u, T = wl.fourier_fields(nx, ny, 1, seed=seed, u_max=u_max)
    u = u.copy()
    u[2] = 0.0
    if ny == 1:
        u[1] = 0.0
    return rho, u, T


CASES = [(2, (70, 33)), (2, (17, 9)), (1, (300, 1)), (1, (7, 1))]


@pytest.mark.parametrize("dims,shape", CASES)
@pytest.mark.parametrize("mode", ["thermal", "iso"])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_projection_parity(dims, shape, mode, storage, tol):
    nx, ny = shape
    tau, steps = 0.7, 40
    fields = planar_fields(nx, ny, seed=41)
    g = lbm().Lattice(nx, ny, 1, tau, storage=storage, mode=mode)
    g.set_projection(dims)
    g.set_fields(*fields)
    o = oracle.OracleLattice(nx, ny, 1, tau, mode=mode)
    o.init(*fields)
    g.step(steps)
    o.step(steps)
    F, b = g.get_state()
    Fo, bo = oracle.project(o.F, o.b, dims, mode == "thermal")
    r, u, T = g.moments()
    ro, uo, To = o.moments()
    errs = {"F": rel_l2(F.cpu().numpy(), Fo), "b": rel_l2(b.cpu().numpy(), bo), "rho": rel_l2(r.cpu().numpy(), ro),
            "u": rel_l2(u.cpu().numpy(), uo), "T": rel_l2(T.cpu().numpy(), To)}
    assert max(errs.values()) <= tol, errs
    assert g.projection() == (dims, F.shape[0], b.shape[0])


@pytest.mark.parametrize("dims,shape", [(2, (64, 48)), (1, (256, 1))])
@pytest.mark.parametrize("mode", ["thermal", "iso"])
def test_projection_equals_the_d3q19_step_on_gpu(dims, shape, mode):
    nx, ny = shape
    fields = planar_fields(nx, ny, seed=42)
    out = []
    for proj in (3, dims):
        g = lbm().Lattice(nx, ny, 1, 0.6, storage="f64", mode=mode)
        g.set_projection(proj)
        g.set_fields(*fields)
        g.step(100)
        out.append([q.cpu().numpy() for q in g.moments()])
    for a, b in zip(*out):
        assert rel_l2(a, b) <= 1e-13


@pytest.mark.parametrize("dims,shape", [(2, (70, 33)), (2, (5, 3)), (1, (300, 1)), (1, (3, 1))])
@pytest.mark.parametrize("mode", ["thermal", "iso"])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-14), ("f32", 1e-6)])
def test_one_launch_step_equals_the_two_pass_step(dims, shape, mode, storage, tol):
    # tiles with a ragged edge, and lattices smaller than one tile (the ring wraps more than once)
    nx, ny = shape
    fields = planar_fields(nx, ny, seed=43)
    out = []
    for kernel in ("auto", "two_pass"):
        g = lbm().Lattice(nx, ny, 1, 0.7, storage=storage, mode=mode, kernel=kernel)
        g.set_projection(dims)
        g.set_fields(*fields)
        g.step(25)
        out.append([q.cpu().numpy() for q in g.get_state()])
    for a, b in zip(*out):
        assert rel_l2(a, b) <= tol


@pytest.mark.parametrize("dims,shape", [(2, (70, 33)), (1, (300, 1))])
@pytest.mark.parametrize("mode", ["thermal", "iso"])
@pytest.mark.parametrize("storage", ["bf16dev", "f16dev"])
def test_16bit_projection_stays_within_its_rounding(dims, shape, mode, storage):
    # BF16 deviation codes hold the deviation itself; FP16 ones a deviation scaled per plane.
    # Bars in units of the code's unit roundoff r (2^-8 BF16, 2^-11 FP16) against the FP32
    # projected run, as for 16-bit D3Q19 storage.  The stored class sums carry the mass, and each
    # rounds a deviation up to nine populations large, so the mass moves at the density's own bar
    # (measured: 8e-5 for BF16 D1Q3 THERMAL; BF16 D3Q19, rounding single populations, ~1e-6).
    nx, ny = shape
    fields = planar_fields(nx, ny, seed=44, u_max=0.1)
    out = {}
    for st in ("f32", storage):
        g = lbm().Lattice(nx, ny, 1, 0.7, storage=st, mode=mode)
        g.set_projection(dims)
        g.set_fields(*fields)
        m0 = g.get_state()[0][:(9 if dims == 2 else 3)].sum().item()  # the class sums F_c
        g.step(40)
        out[st] = [q.cpu().numpy() for q in g.moments()]
        out[st + "_m"] = abs(g.get_state()[0][:(9 if dims == 2 else 3)].sum().item() / m0 - 1)
    r = 2.0 ** -8 if storage == "bf16dev" else 2.0 ** -11
    errs = (rel_l2(out[storage][0], out["f32"][0]), rel_l2(out[storage][1], out["f32"][1]), out[storage + "_m"])
    assert errs[0] < 0.2 * r and errs[1] < 4 * r and errs[2] < 0.2 * r, errs


def test_sod_tube_as_d1q3():
    # the Sod configuration of the D3Q19 tests: 400 x 1 x 1, 1000 steps, FP64
    rho, u, T = wl.sod(400)
    g = lbm().Lattice(400, 1, 1, 0.8, storage="f64")
    g.set_projection(1)
    g.set_fields(rho, u, T)
    o = oracle.OracleLattice(400, 1, 1, 0.8)
    o.init(rho, u, T)
    g.step(1000)
    o.step(1000)
    r, uu, TT = g.moments()
    ro, uo, To = o.moments()
    assert max(rel_l2(r.cpu().numpy(), ro), rel_l2(uu.cpu().numpy(), uo), rel_l2(TT.cpu().numpy(), To)) <= 1e-12


def test_projection_argument_errors():
    L = lbm()
    with pytest.raises(L.LBMError):
        L.Lattice(8, 8, 2, 0.7, storage="f32").set_projection(2)  # nz != 1
    with pytest.raises(L.LBMError):
        L.Lattice(8, 2, 1, 0.7, storage="f32").set_projection(1)  # ny != 1
    with pytest.raises(L.LBMError):
        L.Lattice(8, 8, 1, 0.7, storage="f32", mode="standard").set_projection(2)
    g = L.Lattice(8, 8, 1, 0.7, storage="f32")
    g.set_projection(2)
    u = np.zeros((3, 1, 8, 8))
    u[2] = 0.01
    with pytest.raises(L.LBMError):
        g.set_fields(np.ones((1, 8, 8)), u, np.full((1, 8, 8), 1 / 3))  # transverse velocity
    g.set_fields(np.ones((1, 8, 8)), np.zeros((3, 1, 8, 8)), np.full((1, 8, 8), 1 / 3))
    for call in (lambda: g.invariants(), lambda: g.set_body_force([1e-4, 0, 0]), lambda: g.set_kernel("fused")):
        with pytest.raises(L.LBMError):
            call()
    g.set_projection(3)  # back to D3Q19: state freed, set_fields again
    g.set_fields(np.ones((1, 8, 8)), np.zeros((3, 1, 8, 8)), np.full((1, 8, 8), 1 / 3))
    g.step(2)
    assert g.projection() == (3, 19, 6)
