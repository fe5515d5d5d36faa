"""Serving: many independent lattices batched on one GPU (lbm_server_* in include/lbm.h).

- each request's result in the mix equals the same request stepped alone (bitwise: the
  per-site arithmetic does not depend on what else is resident), also when a small memory
  budget forces requests to queue and be admitted while others run;
- a request that cannot start (non-finite input) or that diverges is reported FAILED without
  disturbing the others;
- the memory budget is enforced at submission for a lattice that could never fit;
- 16-bit deviation storage is served the same way.
"""
import time

import numpy as np
import pytest

from paper_2501_00620_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def lbm():
    from paper_2501_00620_amd import lbm as m
    return m


def alone(fields, tau, steps, storage, mode="thermal"):
    rho, u, T = fields
    nz, ny, nx = rho.shape
    rho_ref, T_ref = lbm().codec_reference(rho, T)  # the server's default reference
    # the server holds a one-plane lattice without transverse velocity as a projected D2Q9
    # lattice; alone, the same projection steps it
    projected = nz == 1 and not np.any(np.asarray(u)[2])
    g = lbm().Lattice(nx, ny, nz, tau, storage=storage, mode=mode, kernel="auto" if projected else "fused",
                      rho_ref=rho_ref, T_ref=T_ref)
    if projected:
        g.set_projection(2)
    g.set_fields(rho, u, T)
    g.step(steps)
    r, uu, TT = g.moments()
    return r.cpu().numpy(), uu.cpu().numpy(), TT.cpu().numpy()


def requests(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        if k % 3 == 2:
            d = int(rng.integers(12, 24))
            f = wl.fourier_fields(d + 3, d, d - 2, seed=int(rng.integers(1 << 30)), u_max=0.2)
        else:
            f = wl.riemann2d_request(rng, n=int(rng.integers(40, 140)))
        steps = int(rng.integers(5, 130))
        tau = float(rng.uniform(0.6, 1.0))
        out.append((f, tau, steps))
    return out


@pytest.mark.parametrize("storage", ["f32", "bf16dev", "f16dev"])
def test_mix_equals_alone_with_queueing(storage):
    L = lbm()
    reqs = requests(7, 9)
    biggest = max(L.lattice_bytes(*f[0].shape[::-1], storage=storage) for f, _, _ in reqs)
    # room for about two lattices: the rest must wait and be admitted as others finish
    with L.Server(budget_bytes=int(2.2 * biggest), bundle_steps=16, storage=storage) as srv:
        ids = []
        for f, tau, steps in reqs:
            ids.append(srv.submit(*f, tau=tau, steps=steps))
            time.sleep(0.002)
        for rid in ids:
            assert srv.wait(rid, timeout=120) == "done", srv.error(rid)
        st = srv.stats()
        assert st["done"] == len(reqs) and st["failed"] == 0 and st["resident_bytes"] == 0
        admits = sorted(srv.poll(r)[2] for r in ids)
        dones = sorted(srv.poll(r)[3] for r in ids)
        assert admits[-1] > dones[0]  # some request was admitted after another had finished
        for rid, (f, tau, steps) in zip(ids, reqs):
            got = srv.fetch(rid)
            ref = alone(f, tau, steps, storage)
            for a, b in zip(got, ref):
                np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_failures_are_isolated(storage):
    # a diverging request is reported as such; in FP16 deviations the diverging values may
    # overflow the code first, which the health check reports as saturation (RANGE)
    L = lbm()
    good = wl.riemann2d_request(np.random.default_rng(1), n=64)
    nan = wl.riemann2d_request(np.random.default_rng(2), n=48)
    nan[0][0, 3, 5] = np.nan
    rho, u, T = wl.fourier_fields(20, 18, 1, seed=3, u_max=0.2)
    u = u.copy()
    u[0] = 0.9  # beyond the positivity bound: diverges
    with L.Server(budget_bytes=1 << 30, bundle_steps=10, storage=storage) as srv:
        rg = srv.submit(*good, tau=0.8, steps=60)
        rn = srv.submit(*nan, tau=0.8, steps=60)
        rb = srv.submit(rho, u, T * 0.1, tau=0.01, steps=300)
        assert srv.wait(rg) == "done"
        assert srv.wait(rn) == "failed" and "admission" in srv.error(rn)
        assert srv.wait(rb) == "failed"
        reason = srv.error(rb)
        kinds = ("diverged", "16-bit encode saturated") if storage == "f16dev" else ("diverged",)
        assert reason.startswith(kinds), reason
        for a, b in zip(srv.fetch(rg), alone(good, 0.8, 60, storage)):
            np.testing.assert_array_equal(a, b)
        with pytest.raises(L.LBMError):
            srv.fetch(rn)


def test_budget_is_enforced_at_submission():
    L = lbm()
    f = wl.riemann2d_request(np.random.default_rng(4), n=128)
    need = L.lattice_bytes(128, 128, 1, storage="f32")
    with L.Server(budget_bytes=need // 2, bundle_steps=8, storage="f32") as srv:
        with pytest.raises(L.LBMError) as e:
            srv.submit(*f, tau=0.8, steps=10)
        assert e.value.name == "ARG"


def test_iso_mode_and_single_step_requests():
    L = lbm()
    rho, u, T = wl.fourier_fields(33, 17, 5, seed=9, u_max=0.2)
    with L.Server(budget_bytes=1 << 30, bundle_steps=7, storage="f32") as srv:
        r1 = srv.submit(rho, u, T, tau=0.7, steps=1)
        r2 = srv.submit(rho, u, T, tau=0.7, steps=23, mode="iso")
        assert srv.wait(r1) == "done" and srv.wait(r2) == "done"
        for a, b in zip(srv.fetch(r1), alone((rho, u, T), 0.7, 1, "f32")):
            np.testing.assert_array_equal(a, b)
        for a, b in zip(srv.fetch(r2), alone((rho, u, T), 0.7, 23, "f32", mode="iso")):
            np.testing.assert_array_equal(a, b)


def test_projected_and_d3q19_one_plane_requests_side_by_side():
    # FP32 one-plane requests without transverse velocity are served projected (THERMAL and ISO);
    # one with a transverse velocity stays D3Q19.  Each equals its alone run to the bit.
    L = lbm()
    a = wl.riemann2d_request(np.random.default_rng(11), n=96)
    rho, u, T = wl.fourier_fields(70, 45, 1, seed=12, u_max=0.15)
    flat = (rho, np.concatenate([u[:2], np.zeros_like(u[2:])]), T)
    with L.Server(budget_bytes=1 << 30, bundle_steps=9, storage="f32") as srv:
        r1 = srv.submit(*a, tau=0.8, steps=50)
        r2 = srv.submit(*flat, tau=0.7, steps=41, mode="iso")
        r3 = srv.submit(rho, u, T, tau=0.7, steps=33)  # u_z != 0: D3Q19
        for r in (r1, r2, r3):
            assert srv.wait(r) == "done", srv.error(r)
        for rid, ref in ((r1, alone(a, 0.8, 50, "f32")), (r2, alone(flat, 0.7, 41, "f32", mode="iso")),
                         (r3, alone((rho, u, T), 0.7, 33, "f32"))):
            for x, y in zip(srv.fetch(rid), ref):
                np.testing.assert_array_equal(x, y)


def test_smallest_served_requests_match_the_oracle():
    # The three smallest requests of the served batch (512 four-quadrant Riemann problems,
    # 2000 steps, tau = 0.8; FP32 storage), served as the batch serves them: projected D2Q9
    # lattices with the codec centred on each request's mean density and temperature.  Each
    # result is checked against the oracle's D3Q19 run of the same request: <= 1e-5 relative L2
    # on rho, u and T; a request the GPU reports failed must diverge in the oracle as well.
    import oracle
    L = lbm()
    steps, tau = 2000, 0.8
    _, sizes, seeds = wl.served_batch()
    order = np.argsort(sizes, kind="stable")[:3]
    reqs = [wl.served_request(sizes[k], seeds[k]) for k in order]
    with L.Server(budget_bytes=1 << 30, bundle_steps=50, storage="f32", health_every=10) as srv:
        ids = [srv.submit(*f, tau=tau, steps=steps) for f in reqs]
        status = [srv.wait(r, timeout=100) for r in ids]
        got = [srv.fetch(r) if s == "done" else None for r, s in zip(ids, status)]
    for k, f, st, res in zip(order, reqs, status, got):
        n = f[0].shape[-1]
        o = oracle.OracleLattice(n, n, 1, tau)
        o.init(*f)
        o.step(steps)
        ro, uo, To = o.moments()
        healthy = bool(np.all(np.isfinite(o.F)) and np.all(ro > 0))
        print(f"request {k} n={n}: server {st}, oracle {'finite' if healthy else 'diverged'}", flush=True)
        if st != "done":
            assert not healthy, (k, n, st)
            continue
        errs = [np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(res, (ro, uo, To))]
        print(f"  rel L2 rho {errs[0]:.2e} u {errs[1]:.2e} T {errs[2]:.2e}", flush=True)
        assert max(errs) <= 1e-5, (k, n, errs)
