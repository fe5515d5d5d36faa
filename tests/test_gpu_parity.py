"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars (relative L2, per field, over the whole lattice):
  F64 storage / F64 math      <= 1e-12   (state fbar, bbar and moments rho, u, T)
  F32 storage / F32 math      <= 1e-5
  16-bit deviation storage    one-step checks against the oracle run from the decoded state,
                              with a per-element bound from the code's rounding (see below).
At full workload sizes, where the oracle cannot run the whole lattice, single steps are checked
on sampled sites: the oracle steps a 5x5x5 periodic copy of each site's neighbourhood (all a
site's update depends on) cut out of the GPU state.
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


def pair(dims, tau, fields, mode="thermal", storage="f64", kernel="auto"):
    nx, ny, nz = dims
    rho, u, T = fields
    g = lbm().Lattice(nx, ny, nz, tau, storage=storage, mode=mode, kernel=kernel)
    g.set_fields(rho, u, T)
    o = oracle.OracleLattice(nx, ny, nz, tau, mode=mode)
    o.init(rho, u, T)
    return g, o


def compare(g, o, tol, what=""):
    F, b = g.get_state()
    errs = {"F": rel_l2(F.cpu().numpy(), o.F), "b": rel_l2(b.cpu().numpy(), o.b)}
    r, u, T = g.moments()
    ro, uo, To = o.moments()
    errs["rho"] = rel_l2(r.cpu().numpy(), ro)
    un = np.linalg.norm(uo)
    errs["u"] = np.linalg.norm(u.cpu().numpy() - uo) / max(un, 1e-12 * np.linalg.norm(ro))
    errs["T"] = rel_l2(T.cpu().numpy(), To)
    print(what, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (what, k, v)
    return errs


ODD_DIMS = [(17, 9, 5), (8, 6, 5), (1, 1, 1), (2, 1, 1), (1, 1, 7), (3, 1, 4), (5, 4, 2), (65, 3, 2)]


KERNELS = ["fused", "two_pass"]
# float and 16-bit storage also step with the producer/consumer sweep (auto picks it from the
# second step on); double precision has no such instantiation
KERNELS_FLOAT = ["fused", "fused_pc", "two_pass"]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dims", ODD_DIMS)
@pytest.mark.parametrize("mode", ["thermal", "iso"])
def test_f64_parity_odd_sizes(dims, mode, kernel):
    fields = wl.fourier_fields(*dims, seed=sum(dims), u_max=0.2)
    g, o = pair(dims, 0.7, fields, mode=mode, kernel=kernel)
    compare(g, o, 1e-12, f"f64 {mode} {dims} step 0")
    # boxes this small damp their modes within tens of steps (k^2 nu ~ 0.4 per step); after 10
    # steps the velocity is still far above the level where it is only round-off of O(0.1)
    # populations, so its relative error stays a meaningful measure
    g.step(10)
    o.step(10)
    compare(g, o, 1e-12, f"f64 {mode} {dims} step 10")


@pytest.mark.parametrize("kernel", KERNELS)
def test_f64_parity_24_cubed(kernel):
    dims = (24, 24, 24)
    g, o = pair(dims, 0.6, wl.fourier_fields(*dims, seed=3, u_max=0.3), kernel=kernel)
    g.step(40)
    o.step(40)
    compare(g, o, 1e-12, "f64 24^3 step 40")


def test_f64_sod_full_config():
    # 400 x 1 x 1, FP64, tau = 0.8, 1000 steps (the full shock-tube workload)
    g, o = pair((400, 1, 1), 0.8, wl.sod(400))
    g.step(1000)
    o.step(1000)
    compare(g, o, 1e-12, "sod f64 1000 steps")


@pytest.mark.parametrize("kernel", KERNELS_FLOAT)
@pytest.mark.parametrize("mode", ["thermal", "iso"])
def test_f32_parity(mode, kernel):
    # short runs in the small boxes, whose modes damp within tens of steps; longer ones where
    # the flow lives longer
    for dims, steps in [((17, 9, 5), 30), ((32, 32, 1), 100), ((12, 10, 8), 30), ((33, 17, 9), 60)]:
        if kernel == "fused_pc" and dims[2] < 3:
            continue  # the split sweep marches in z
        g, o = pair(dims, 0.6, wl.fourier_fields(*dims, seed=7, u_max=0.25), mode=mode, storage="f32",
                    kernel=kernel)
        g.step(steps)
        o.step(steps)
        compare(g, o, 1e-5, f"f32 {mode} {dims} step {steps}")


def test_f32_acoustic_pulse_full_grid():
    # 256 x 256 x 1 acoustic pulse, FP32, tau = 0.6; 100 steps of the 5000 (oracle time-bound)
    g, o = pair((256, 256, 1), 0.6, wl.acoustic_pulse(256), storage="f32")
    g.step(100)
    o.step(100)
    compare(g, o, 1e-5, "acoustic f32 256^2 step 100")


@pytest.mark.parametrize("dims", [(70, 9, 11), (70, 33, 1), (45, 20, 2), (70, 9, 37)])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "bf16dev"])
def test_fused_equals_two_pass(storage, dims):
    # same arithmetic in a different schedule: equal up to the order of the gradient sums (for
    # one z plane the fused sweep also regroups the gather and the gradient in-plane).  nz = 37
    # runs as two z chunks of 19 planes: a chunk starting at an odd plane, for the populations
    # the sweep carries in LDS slots chosen by plane parity
    fields = wl.fourier_fields(*dims, seed=12, u_max=0.25)
    out = []
    kernels = ["two_pass", "fused"] + (["fused_pc"] if storage != "f64" and dims[2] >= 3 else [])
    for kernel in kernels:
        g = lbm().Lattice(*dims, 0.65, storage=storage, kernel=kernel)
        g.set_fields(*fields)
        g.step(7)
        F, b = g.get_state()
        out.append((F.cpu().numpy(), b.cpu().numpy()))
    tol = {"f64": 1e-14, "f32": 1e-6, "f16dev": 1e-3, "bf16dev": 1e-2}[storage]
    for k in range(1, len(out)):
        assert rel_l2(out[k][0], out[0][0]) <= tol, (kernels[k], rel_l2(out[k][0], out[0][0]))
        assert rel_l2(out[k][1], out[0][1]) <= tol, (kernels[k], rel_l2(out[k][1], out[0][1]))


def test_conservation_on_gpu():
    for storage, tol in (("f64", 1e-13), ("f32", 2e-6)):
        dims = (16, 12, 10)
        g = lbm().Lattice(*dims, 0.7, storage=storage)
        g.set_fields(*wl.fourier_fields(*dims, seed=4, u_max=0.2))
        i0 = g.invariants()
        g.step(200)
        i1 = g.invariants()
        scale = np.array([i0[0]] * 4 + [i0[4]])
        assert np.abs((i1 - i0) / scale).max() <= tol, (storage, (i1 - i0) / scale)


def test_deterministic_bitwise_and_restart():
    dims = (20, 9, 7)
    fields = wl.fourier_fields(*dims, seed=5, u_max=0.2)
    for storage in ("f64", "f32"):
        a = lbm().Lattice(*dims, 0.7, storage=storage)
        a.set_fields(*fields)
        a.step(30)
        b = lbm().Lattice(*dims, 0.7, storage=storage)
        b.set_fields(*fields)
        b.step(30)
        Fa, ba = a.get_state()
        Fb, bb = b.get_state()
        assert torch.equal(Fa, Fb) and torch.equal(ba, bb)
        # restart: 12 steps, checkpoint, restore into a fresh lattice, 18 more
        c = lbm().Lattice(*dims, 0.7, storage=storage)
        c.set_fields(*fields)
        c.step(12)
        Fc, bc = c.get_state()
        d = lbm().Lattice(*dims, 0.7, storage=storage)
        d.set_state(Fc, bc)
        d.step(18)
        Fd, bd = d.get_state()
        # a checkpoint holds bbar gathered; the continued run gathers the same sums, so the
        # restart equals the uninterrupted run to the last bit only up to that re-association
        assert rel_l2(Fd.cpu().numpy(), Fa.cpu().numpy()) <= (1e-15 if storage == "f64" else 1e-6)
        assert rel_l2(bd.cpu().numpy(), ba.cpu().numpy()) <= (1e-15 if storage == "f64" else 1e-6)


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_deviation_codec_is_bit_exact(storage):
    from oracle import codec
    dims = (9, 7, 5)
    rho, u, T = wl.fourier_fields(*dims, seed=6, u_max=0.3)
    o = oracle.OracleLattice(*dims, 0.7)
    o.init(rho, u, T)
    o.step(3)
    g = lbm().Lattice(*dims, 0.7, storage=storage)
    g.set_state(o.F, o.b)
    scales, refs = g.codec()
    Fc, bc = g.raw_codes()
    enc = codec.encode_f16 if storage == "f16dev" else codec.encode_bf16
    for i in range(19):
        np.testing.assert_array_equal(Fc[i], enc(o.F[i], refs[i], scales[i]))
    for c in range(6):
        np.testing.assert_array_equal(bc[c], enc(o.b[c], refs[19 + c], scales[19 + c]))
    # scales are powers of two, one per stored array (the populations; bbar): the sweep reads
    # each array's first entry for all of its planes
    assert np.all(np.log2(scales) == np.round(np.log2(scales)))
    assert np.all(scales[:19] == scales[0]) and np.all(scales[19:] == scales[19])


def test_argument_errors():
    L = lbm()
    with pytest.raises(L.LBMError) as e:
        L.Lattice(4, 4, 4, -1.0)
    assert e.value.name == "ARG"
    with pytest.raises(L.LBMError) as e:
        L.Lattice(0, 4, 4, 0.7)
    assert e.value.name == "ARG"
    g = L.Lattice(4, 4, 4, 0.7)
    with pytest.raises(L.LBMError) as e:
        g.step(1)
    assert e.value.name == "STATE"
    rho, u, T = wl.uniform(4, 4, 4)
    rho[0, 0, 0] = -1.0
    with pytest.raises(L.LBMError) as e:
        g.set_fields(rho, u, T)
    assert e.value.name == "ARG"
    rho[0, 0, 0] = np.nan
    with pytest.raises(L.LBMError) as e:
        g.set_fields(rho, u, T)
    assert e.value.name == "ARG"


def test_health_flags_divergence():
    L = lbm()
    dims = (6, 5, 4)
    rho, u, T = wl.fourier_fields(*dims, seed=2, u_max=0.2)
    g = L.Lattice(*dims, 0.7, storage="f32")
    g.set_fields(rho, u, T)
    assert g.health()[:2] == (0, 0)
    # far beyond the positivity bound |u| <= 0.5 at a cold temperature and tau near 0: the
    # run blows up within a few hundred steps, and the health check reports it
    bad = L.Lattice(*dims, 0.01, storage="f32")
    uu = np.zeros_like(u)
    uu[0] = 0.9 * np.sign(np.sin(np.arange(dims[0]) + 0.5))[None, None, :]
    bad.set_fields(rho, uu, T * 0.1)
    bad.step(300)
    n_bad, n_neg, _ = bad.health()
    assert n_bad > 0 or n_neg > 0


# ---------------------------------------------------------------------------------------------
# full-size sampled checks
# ---------------------------------------------------------------------------------------------
def _boxes(t, sites, shape, planes):
    """(m, planes, 5, 5, 5) neighbourhoods (periodic) of flat `sites` from a CUDA tensor."""
    nz, ny, nx = shape
    s = torch.as_tensor(sites, device=t.device)
    x, y, z = s % nx, (s // nx) % ny, s // (nx * ny)
    d = torch.arange(-2, 3, device=t.device)
    zz = (z[:, None] + d[None, :]) % nz
    yy = (y[:, None] + d[None, :]) % ny
    xx = (x[:, None] + d[None, :]) % nx
    idx = (zz[:, :, None, None] * ny * nx + yy[:, None, :, None] * nx + xx[:, None, None, :]).reshape(len(sites), -1)
    flat = t.reshape(planes, -1)
    return flat[:, idx].permute(1, 0, 2).reshape(len(sites), planes, 5, 5, 5)


def sampled_one_step(g, tau, mode, sites, Tfield=None):
    """One step at `sites`, by the oracle from the GPU's current state and by the GPU.

    Returns (F_gpu, b_gpu, F_oracle, b_oracle, bstar_gpu, bstar_oracle): the post-stream state
    after the step at the sites (gathered bbar), plus the stored post-collision bbar* at the
    sites (what the GPU holds before carrying it along), each (m, 19) / (m, 6)."""
    F0, b0 = g.get_state()
    Fb = _boxes(F0, sites, g.shape, 19).cpu().numpy()
    bb = _boxes(b0, sites, g.shape, 6).cpu().numpy()
    Tb = None
    if Tfield is not None:
        Tb = _boxes(torch.as_tensor(Tfield, device="cuda").reshape(1, -1), sites, g.shape, 1).cpu().numpy()
    del F0, b0
    g.step(1)
    s = torch.as_tensor(sites, device="cuda")
    F1, b1 = g.get_state()
    Fg = F1.reshape(19, -1)[:, s].T.cpu().numpy()
    bg = b1.reshape(6, -1)[:, s].T.cpu().numpy()
    del F1, b1
    F1s, b1s, gathered = g.get_stored()
    assert not gathered
    bsg = b1s.reshape(6, -1)[:, s].T.cpu().numpy()
    assert np.array_equal(F1s.reshape(19, -1)[:, s].T.cpu().numpy(), Fg)
    del F1s, b1s
    Fo = np.zeros_like(Fg)
    bo = np.zeros_like(bg)
    bso = np.zeros_like(bg)
    centre = 2 * 25 + 2 * 5 + 2
    for m in range(len(sites)):
        o = oracle.OracleLattice(5, 5, 5, tau, mode=mode, T_field=None if Tb is None else Tb[m, 0])
        fo, bo_, bs_ = o.step_sites([centre], Fb[m], bb[m], with_bstar=True)
        Fo[m], bo[m], bso[m] = fo[0], bo_[0], bs_[0]
    return Fg, bg, Fo, bo, bsg, bso


def test_tgv_256_cubed_f32_sampled_steps():
    # 3-D compressible Taylor-Green vortex, 256^3, Ma 0.5, tau = 0.55, FP32 storage
    n = 256
    rho, u, T = wl.taylor_green(n)
    g = lbm().Lattice(n, n, n, 0.55, storage="f32")
    g.set_fields(rho, u, T)
    g.step(20)
    rng = np.random.default_rng(0)
    sites = rng.integers(0, n ** 3, size=64)
    sites[:4] = [0, n - 1, n * n * n - 1, n * n * (n - 1)]  # seams of the periodic box
    Fg, bg, Fo, bo, bsg, bso = sampled_one_step(g, 0.55, "thermal", sites)
    assert rel_l2(Fg, Fo) <= 1e-6, rel_l2(Fg, Fo)
    assert rel_l2(bg, bo) <= 1e-5, rel_l2(bg, bo)
    assert rel_l2(bsg, bso) <= 1e-5, rel_l2(bsg, bso)


HALF_ULP = {"f32": 0.0, "f16dev": 2.0 ** -11, "bf16dev": 2.0 ** -8}


def _check_stored_bound(storage, Fg, Fo, bsg, bso, scales, refs):
    """Per element: the code's rounding (half a unit in the last place of h = deviation/scale,
    plus the smallest subnormal step for fp16) and FP32 arithmetic (a few 1e-7 of the terms)."""
    half = HALF_ULP[storage]
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    for vals_g, vals_o, off, floor in ((Fg, Fo, 0, w), (bsg, bso, 19, np.full(6, 1e-2))):
        for k in range(vals_g.shape[1]):
            dev = np.abs(vals_o[:, k] - refs[off + k])
            code = half * dev + (scales[off + k] * 2.0 ** -24 if storage == "f16dev" else 0.0)
            arith = 5e-7 * np.maximum(dev, floor[k])
            bad = np.abs(vals_g[:, k] - vals_o[:, k]) > code + arith
            assert not bad.any(), (storage, off + k, np.abs(vals_g[:, k] - vals_o[:, k])[bad], (code + arith)[bad])


@pytest.mark.parametrize("storage", ["f32", "f16dev", "bf16dev"])
def test_stored_state_one_step_bound(storage):
    # One step from the decoded state: the oracle's FP64 step against the GPU's FP32-arithmetic
    # step, compared on what the GPU stores (post-stream populations, post-collision bbar*).
    n = 64
    rho, u, T = wl.fourier_fields(n, n, n, seed=11)
    g = lbm().Lattice(n, n, n, 0.6, storage=storage)
    g.set_fields(rho, u, T)
    g.step(5)
    if storage == "f32":
        scales, refs = np.ones(25), np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12 + [0.0] * 6)
    else:
        scales, refs = g.codec()
    rng = np.random.default_rng(1)
    sites = rng.integers(0, n ** 3, size=48)
    Fg, bg, Fo, bo, bsg, bso = sampled_one_step(g, 0.6, "thermal", sites)
    _check_stored_bound(storage, Fg, Fo, bsg, bso, scales, refs)


# ---------------------------------------------------------------------------------------------
# long horizon, invariants, reference-shifted deviation variables, range flag
# ---------------------------------------------------------------------------------------------
def test_f32_tgv_long_horizon():
    # The FP32 path held to its bar over a long run: 48^3 Taylor-Green vortex, Mach 0.5, tau 0.55,
    # 1000 steps, both kernels against one oracle run.  In a box this small the vortex decays by
    # e^-9 over the run, and the relative error of a vanishing u (or of b, which then holds only
    # T - 1/3) measures nothing; a uniform drift velocity keeps a reference that does not decay.
    # A bias of a few 1e-8 per step in the momentum the collision hands on (a rounded-constant
    # split of omega j + F, or 1 - omega and omega rounded apart) compounds to about 3e-5 on the
    # drift here; unbiased rounding stays near 1e-6.
    n, tau, steps = 48, 0.55, 1000
    rho, u, T = wl.taylor_green(n)
    fields = (rho, u + np.array([0.05, -0.04, 0.03]).reshape(3, 1, 1, 1), T)
    o = oracle.OracleLattice(n, n, n, tau)
    o.init(*fields)
    o.step(steps)
    ro, uo, To = o.moments()
    for kernel in KERNELS_FLOAT:
        g = lbm().Lattice(n, n, n, tau, storage="f32", kernel=kernel)
        g.set_fields(*fields)
        g.step(steps)
        F, b = g.get_state()
        r, u, T = g.moments()
        # bbar is the bumps' variance relative to c^2/3: it vanishes as T -> 1/3, so its own
        # relative L2 only echoes the absolute error of T; it is held to the bar on the scale of
        # the temperature it carries
        errs = {"F": rel_l2(F.cpu().numpy(), o.F), "rho": rel_l2(r.cpu().numpy(), ro),
                "u": rel_l2(u.cpu().numpy(), uo), "T": rel_l2(T.cpu().numpy(), To),
                "b_on_T_scale": float(np.linalg.norm(b.cpu().numpy() - o.b) / np.linalg.norm(To))}
        print(f"f32 tgv 48^3 {steps} steps {kernel}", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        assert max(errs.values()) <= 1e-5, errs
        g.close()


def _invariant_scale(o):
    # mass and energy against themselves; each momentum component against sum rho |u|, so that a
    # component near zero is still held to the same absolute accuracy
    ro, uo, _ = o.moments()
    inv = o.invariants()
    mom = float(np.sum(ro * np.sqrt((uo ** 2).sum(0))))
    return inv, np.array([inv[0], mom, mom, mom, inv[4]])


@pytest.mark.parametrize("kernel", KERNELS_FLOAT)
@pytest.mark.parametrize("storage,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_invariants_match_oracle(storage, tol, kernel):
    if storage == "f64" and kernel == "fused_pc":
        pytest.skip("the producer/consumer sweep has no double-precision instantiation")
    # the GPU's FP64 reductions of mass, momentum and energy (Sec. II C's conserved sums) against
    # the oracle's on the same state: right after set_fields (bbar gathered) and after steps
    # (bbar* held before the gather); a drift velocity makes every momentum component distinct
    dims = (19, 14, 11)
    rho, u, T = wl.fourier_fields(*dims, seed=21, u_max=0.2)
    u = u + np.array([0.05, -0.03, 0.02]).reshape(3, 1, 1, 1)
    g, o = pair(dims, 0.65, (rho, u, T), storage=storage, kernel=kernel)
    for steps in (0, 37):
        if steps:
            g.step(steps)
            o.step(steps)
        gi = g.invariants()
        oi, scale = _invariant_scale(o)
        err = np.abs(gi - oi) / scale
        print(storage, kernel, steps, err, flush=True)
        assert err.max() <= tol, (steps, err)


def shifted_pair(dims, tau, fields, mode, storage, kernel, rho_ref, T_ref):
    nx, ny, nz = dims
    g = lbm().Lattice(nx, ny, nz, tau, storage=storage, mode=mode, kernel=kernel, rho_ref=rho_ref, T_ref=T_ref)
    g.set_fields(*fields)
    o = oracle.OracleLattice(nx, ny, nz, tau, mode=mode)
    o.init(*fields)
    return g, o


@pytest.mark.parametrize("kernel", KERNELS_FLOAT)
@pytest.mark.parametrize("mode", ["thermal", "iso"])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_reference_shifted_parity(storage, tol, mode, kernel):
    if storage == "f64" and kernel == "fused_pc":
        pytest.skip("the producer/consumer sweep has no double-precision instantiation")
    # Deviation variables about rho_ref != 1 and T_ref != 1/3 (the served lattices' references):
    # the constant rho_ref (T_ref - 1/3) enters the second-moment source (Eq. 61) and the
    # predictor's density offset.  A change of variables only, so the oracle's result holds.
    dims = (17, 9, 6)
    rho, u, T = wl.fourier_fields(*dims, seed=23, u_max=0.2, T0=0.25)
    rho = 0.6 * rho
    rho_ref, T_ref = lbm().codec_reference(rho, T)
    assert abs(rho_ref - 1.0) > 0.3 and abs(T_ref - 1.0 / 3.0) > 0.05
    g, o = shifted_pair(dims, 0.7, (rho, u, T), mode, storage, kernel, rho_ref, T_ref)
    compare(g, o, tol, f"shifted {storage} {mode} {kernel} step 0")
    g.step(25)
    o.step(25)
    compare(g, o, tol, f"shifted {storage} {mode} {kernel} step 25")


@pytest.mark.parametrize("layout", ["fused", "two_pass", "projected"])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_reference_shifted_four_quadrant(storage, tol, layout):
    # A served request's shape and references: a four-quadrant Riemann problem on n x n x 1 with
    # the codec centred on its mean density and temperature, stepped by the one-plane fused sweep,
    # the two-pass kernel and the projected D2Q9 kernel
    n, tau, steps = 40, 0.8, 60
    fields = wl.riemann2d_request(np.random.default_rng(31), n=n)
    rho_ref, T_ref = lbm().codec_reference(fields[0], fields[2])
    kernel = "auto" if layout == "projected" else layout
    g, o = shifted_pair((n, n, 1), tau, fields, "thermal", storage, kernel, rho_ref, T_ref)
    if layout == "projected":
        g.set_projection(2)
        g.set_fields(*fields)
    g.step(steps)
    o.step(steps)
    r, u, T = g.moments()
    ro, uo, To = o.moments()
    errs = {"rho": rel_l2(r.cpu().numpy(), ro), "u": rel_l2(u.cpu().numpy(), uo), "T": rel_l2(T.cpu().numpy(), To)}
    F, b = g.get_state()
    if layout == "projected":
        Fo, bo = oracle.project(o.F, o.b, 2, True)
    else:
        Fo, bo = o.F, o.b
    errs["F"] = rel_l2(F.cpu().numpy(), Fo)
    errs["b"] = rel_l2(b.cpu().numpy(), bo)
    print(storage, layout, errs, flush=True)
    assert max(errs.values()) <= tol, errs


def _near_empty_site_state(dims, site):
    # rest state at T = 1/3, except one site whose populations carry a momentum of (2, 2, 0) at a
    # density of 0.05 (populations +1 along +x and +y, -1 + 0.025 along -x and -y): its velocity
    # of 40 per component puts rho ux^2 uy^2 near 8e5 into the next collision's equilibrium, far
    # beyond 1024 times the largest initial deviation (about 1), the headroom of the fp16 codec
    # scale; the density stays well above the codes' rounding (about 2e-3 at that scale)
    _, w = oracle.velocity_set()
    nx, ny, nz = dims
    F = np.broadcast_to(w.reshape(19, 1, 1, 1), (19, nz, ny, nx)).copy()
    b = np.zeros((6, nz, ny, nx))
    z, y, x = site
    F[:, z, y, x] = 0.0
    F[1, z, y, x] = F[2, z, y, x] = 1.0
    F[3, z, y, x] = F[4, z, y, x] = -1.0 + 0.025
    return F, b


@pytest.mark.parametrize("kernel", KERNELS_FLOAT)
def test_fp16_overflow_is_reported_as_range(kernel):
    # Numerical overflow of the 16-bit code (not a device fault): the step stores +-inf, and the
    # next health check reports RANGE once and clears the flag; the non-finite values are then
    # reported as a divergence.  Setting new fields afterwards starts from a clear flag.
    L = lbm()
    dims = (12, 10, 8)
    g = L.Lattice(*dims, 0.7, storage="f16dev", kernel=kernel)
    F, b = _near_empty_site_state(dims, (4, 5, 6))
    g.set_state(F, b)
    assert g.health()[:2] == (0, 0)
    g.step(1)
    with pytest.raises(L.LBMError) as e:
        g.health()
    assert e.value.name == "RANGE"
    n_bad, _, _ = g.health()
    assert n_bad > 0
    g.set_fields(*wl.fourier_fields(*dims, seed=2, u_max=0.2))
    assert g.health()[:2] == (0, 0)
    g.step(3)
    assert g.health()[:2] == (0, 0)


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("dims", [(5, 3, 3), (64, 8, 3), (65, 9, 4), (130, 17, 5)])
@pytest.mark.parametrize("mode", ["thermal", "iso"])
def test_split_sweep_all_terms_against_oracle(dims, mode, walls):
    # The split sweep with every term at once, FP32 against the oracle (<= 1e-5): references
    # shifted off rho = 1, T = 1/3 (the K e_i terms), a body-force field and a ghost rate, and
    # (or not) moving walls, whose planes the wall kernel steps.  The shapes take one plane per z
    # chunk past the warm-up (nz = 3, 4, 5; with walls one to three interior planes), lattices
    # narrower than the 64 x 8 tile (its lanes wrap onto the same sites and store nothing), one
    # exact tile, and ragged tiles in x and y.
    tau, tau_g, steps = 0.7, 0.55, 12
    rho, u, T = wl.fourier_fields(*dims, seed=47, u_max=0.2, T0=0.3)
    rho = 0.8 * rho
    rho_ref, T_ref = lbm().codec_reference(rho, T)
    _, a, _ = wl.fourier_fields(*dims, seed=48, u_max=1.0)
    a = 3e-4 * a
    nx, ny, nz = dims
    g = lbm().Lattice(nx, ny, nz, tau, storage="f32", mode=mode, kernel="fused_pc", rho_ref=rho_ref, T_ref=T_ref)
    g.set_ghost_relaxation(tau_g)
    g.set_fields(rho, u, T)
    g.set_body_force(a)
    o = oracle.OracleLattice(nx, ny, nz, tau, mode=mode, tau_ghost=tau_g)
    o.init(rho, u, T)
    o.set_body_force(a)
    if walls:
        ub, ut = [0.02, -0.01, 0.0], [-0.015, 0.03, 0.0]
        g.set_walls(ub, ut)
        o.set_walls(ub, ut)
    g.step(steps)
    o.step(steps)
    compare(g, o, 1e-5, f"split sweep, all terms, {dims} {mode}, walls {walls}")
