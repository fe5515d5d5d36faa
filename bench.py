"""Benchmark of the fused collide-and-stream sweep on one MI355X.

Timed workload (one "step" = one full pass of the sweep over the lattice): the 3-D compressible
Taylor-Green vortex on a 256^3 periodic D3Q19 lattice, Mach 0.5, tau = 0.55, FP32 storage and
arithmetic, inputs resident in HBM.  W untimed warm-up steps, then exactly K timed steps in five
consecutive windows, each between HIP events recorded on the lattice's stream (synchronize on
both sides); the headline is the median window's rate.

Also reported on the same JSON line:
  roofline      algorithmic bytes per step (2 x 25 values x 4 B per site) over the measured
                average step duration, against the 8 TB/s HBM peak; `traffic` from the committed
                rocprofv3 FETCH_SIZE / WRITE_SIZE counters when they match the current kernel
                sources, else null; `copy_ceiling`, the GB/s of a plain 1 GiB device copy
                measured in the same run, and the achieved rate as a fraction of it;
  variants      the 2000-step run in FP64, FP32, FP16- and BF16-deviation storage: MLUPS and the
                relative L2 error of rho, u, T against the FP64-storage run, kinetic-energy decay;
  served        the served batch: 512 independent four-quadrant Riemann problems (n x n x 1,
                n uniform in [64, 512], 2000 steps each) arriving as a Poisson stream at 50/s,
                admitted by a 4 GiB device-memory budget, in FP32 and FP16/BF16-deviation
                storage; p50/p99 time-to-result (per run and over the requests every storage
                completed), aggregate MLUPS, failed requests with their reasons (strong
                four-quadrant problems leave the scheme's stability region and diverge);
  configs       the other workloads: the Sod tube (400 x 1 x 1, FP64) against the exact Riemann
                solution at t = 75 and its invariants over 1000 steps; the 256^2 acoustic pulse
                (FP32, 5000 steps), sound speeds of four Fourier modes against sqrt(5T/3) and
                sqrt(T); 512^3 random smooth fields in FP16-deviation vs FP32 storage (500
                steps): MLUPS, GB/s, relative L2;
  comparator    the standard lattice Boltzmann comparator (Sec. I, Eq. 4) timed on the same
                input, the Galilean-invariance contrast measured on the GPU (shear-wave
                viscosity in a moving frame, bump vs standard scheme), the MRT step's
                throughput beside the single-rate two-pass step, the body force (fused and two-pass
                throughput; Kolmogorov-flow amplitude against A / (T tau k^2)), and the walls
                (channel throughput in the split fused sweep and two-pass, beside the periodic
                sweep; the gravity Couette flow of Sec. III C in two frames, bump vs standard,
                against its closed form);
  cpu_baseline  the FP64 CPU oracle timed on this host on a bounded sample (a 48^3 Taylor-Green
                vortex for ~10 s) with OpenMP on all allowed threads, and again on one core;
                the CPU model.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--quick]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline, FP32 vs FP16-storage at stated L2 err; served p99"
HBM_PEAK_GBS = 8000.0
BYTES_PER_VALUE = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}
VALUES_PER_LUP = 2 * (19 + 6)


# The sources that define the fused sweep kernel and its compile flags: PMC counters taken on
# other sources do not describe the kernel being timed.
KERNEL_SOURCES = ("paper_2501_00620_amd/csrc/lbm_device.hpp", "paper_2501_00620_amd/csrc/lbm_fused.hpp",
                  "paper_2501_00620_amd/csrc/lbm_sweep.hip",
                  "paper_2501_00620_amd/csrc/lbm_fused_pc.hpp",
                  "paper_2501_00620_amd/build.py")


def source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, workload, launch_sites):
    """HBM bytes per launch from committed PMC counters, if taken on the current sources."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def valu_busy_from_profiles(kernel, workload):
    """Share of a SIMD's cycles that issue VALU work in the profiled kernel (wave64 instructions
    at 4 cycles each over the 1,024 SIMDs, against GRBM_GUI_ACTIVE summed over the 8 XCDs), from
    committed SQ counters taken on the current sources; else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sq = rec.get("sq") or {}
    if rec.get("source_hash") != source_hash() or not sq.get("GRBM_GUI_ACTIVE"):
        return None
    return sq["SQ_INSTS_VALU"] * 4 / 1024 / (sq["GRBM_GUI_ACTIVE"] / 8)


def step_kernel(kernel, storage, nz):
    """The kernel that times the steady-state steps of an n^3 lattice (lbm_set_kernel's choice)."""
    if kernel == "two_pass":
        return "k_two_pass"
    if kernel == "fused_pc" or (kernel == "auto" and storage != "f64" and nz >= 3):
        return "k_fused_pc"
    return "k_fused"


def timed_windows(lat, steps, warmup, windows=5):
    """W warm-up steps, then exactly `steps` timed steps split into `windows` consecutive
    windows, each between HIP events on the lattice's stream.  Returns the per-step seconds of
    each window."""
    import torch
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    windows = max(1, min(windows, steps))
    sizes = [steps // windows] * windows
    sizes[-1] += steps - sum(sizes)
    stream = lat.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(windows + 1)]
    ev[0].record(stream)
    for w, k in enumerate(sizes):
        lat.step(k)
        ev[w + 1].record(stream)
    ev[-1].synchronize()
    torch.cuda.synchronize()
    return [ev[w].elapsed_time(ev[w + 1]) / 1e3 / k for w, k in enumerate(sizes)]


def timed_steps(lat, steps, warmup):
    import torch
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    stream = lat.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3  # seconds


def rel_l2(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def run_variants(n, steps, tau, mach, every=500):
    """FP64 / FP32 / FP16dev / BF16dev storage over the full run; errors against FP64."""
    import torch
    from paper_2501_00620_amd import lbm, workloads
    rho0, u0, T0 = workloads.taylor_green(n, mach=mach)
    out = {}
    ref = None
    for storage in ("f64", "f32", "f16dev", "bf16dev"):
        lat = lbm.Lattice(n, n, n, tau, storage=storage)
        lat.set_fields(rho0, u0, T0)
        ke = []
        t_total = 0.0
        done = 0
        while done < steps:
            k = min(every, steps - done)
            t_total += timed_steps(lat, k, 0)
            done += k
            r, u, T = lat.moments()
            ke.append(float((0.5 * r * (u * u).sum(0)).sum() / r.sum()))
        r, u, T = lat.moments()
        bad = lat.health()
        mlups = n ** 3 * steps / t_total / 1e6
        gbs = mlups * VALUES_PER_LUP * BYTES_PER_VALUE[storage] / 1e3
        rec = {"mlups": mlups, "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS, "kinetic_energy": ke,
               "nonfinite_sites": bad[0]}
        if n == 256:
            busy = valu_busy_from_profiles(step_kernel("auto", storage, n), "tgv256_" + storage)
            if busy is not None:
                rec["valu_issue_busy"] = busy
        if ref is None:
            ref = (r, u, T)
        else:
            rec["rel_l2_vs_f64"] = {"rho": rel_l2(r, ref[0]), "u": rel_l2(u, ref[1]), "T": rel_l2(T, ref[2])}
        out[storage] = rec
        print(f"[bench] variant {storage}: {rec['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        del lat
        torch.cuda.empty_cache()
    return out


def run_serving(storage, n_requests=512, rate=50.0, steps=2000, budget=4 << 30, bundle=50, seed=2024, tau=0.8):
    """Served batch: independent n x n x 1 four-quadrant Riemann problems, n uniform in
    [64, 512], Poisson arrivals at `rate` per second, admitted by a device-memory budget.
    Returns p50/p99 time-to-result, aggregate MLUPS over the whole run, and per-request
    outcomes (latency, or the reason a request failed)."""
    import numpy as np
    from paper_2501_00620_amd import lbm, workloads
    arrivals, sizes, field_seeds = workloads.served_batch(n_requests, rate, seed)
    ids = []
    with lbm.Server(budget_bytes=budget, bundle_steps=bundle, storage=storage, health_every=10) as srv:
        t0 = time.perf_counter()
        for k in range(n_requests):
            while time.perf_counter() - t0 < arrivals[k]:
                time.sleep(min(0.002, max(0.0, arrivals[k] - (time.perf_counter() - t0))))
            f = workloads.served_request(sizes[k], field_seeds[k])
            ids.append(srv.submit(*f, tau=tau, steps=steps))
        status = [srv.wait(r, timeout=600) for r in ids]
        times = np.array([srv.poll(r)[1:] for r in ids])
        errors = [srv.error(r) if s_ != "done" else "" for r, s_ in zip(ids, status)]
        st = srv.stats()
        # results of every 8th request, fetched after the timed run, for the storages' comparison
        sample = {}
        for k, (r, s_) in enumerate(zip(ids, status)):
            if s_ == "done" and k % 8 == 0:
                sample[k] = tuple(np.asarray(a, np.float32) for a in srv.fetch(r))
    ok = np.array([s_ == "done" for s_ in status])
    print(f"[bench] served {storage}: {int(ok.sum())}/{n_requests} done", file=sys.stderr, flush=True)
    latency = times[:, 2] - times[:, 0]
    wait = times[ok, 1] - times[ok, 0]
    span = times[ok, 2].max() - times[:, 0].min()
    lups = float((sizes[ok].astype(np.float64) ** 2).sum() * steps)
    reasons = {}
    for e in errors:
        if e:
            key = e.split(":")[0]
            reasons[key] = reasons.get(key, 0) + 1
    rec = {"requests": n_requests, "done": int(ok.sum()), "failed": int((~ok).sum()),
           "failure_reasons": reasons,
           "p50_s": float(np.percentile(latency[ok], 50)), "p99_s": float(np.percentile(latency[ok], 99)),
           "p50_queue_wait_s": float(np.percentile(wait, 50)), "p99_queue_wait_s": float(np.percentile(wait, 99)),
           "aggregate_mlups": lups / span / 1e6, "span_s": float(span),
           "bundle_busy_mlups": st["lattice_updates"] / max(st["busy_s"], 1e-9) / 1e6,
           "workload": f"{n_requests} four-quadrant Riemann problems n x n x 1, n ~ U[64,512], tau {tau}, "
                       f"{steps} steps, Poisson {rate}/s, budget {budget / 2**30:.0f} GiB, bundle {bundle} steps"}
    return rec, ok, latency, sample


def run_served_comparison(storages=("f32", "f16dev", "bf16dev"), **kw):
    """The served batch once per storage.  Requests that diverge are reported failed, and which
    ones do depends on the storage precision, so beside each run's own percentiles the latency is
    also given over the requests that completed under every storage."""
    import numpy as np
    out, oks, lats, samples = {}, [], [], []
    for st in storages:
        rec, ok, lat, sample = run_serving(st, **kw)
        out[st] = rec
        oks.append(ok)
        lats.append(lat)
        samples.append(sample)
    common = np.logical_and.reduce(oks)
    for st, ok, lat, sample in zip(storages, oks, lats, samples):
        out[st]["failed_also_in_" + storages[0]] = int((~ok & ~oks[0]).sum())
        out[st]["common_requests"] = int(common.sum())
        out[st]["p50_s_common"] = float(np.percentile(lat[common], 50))
        out[st]["p99_s_common"] = float(np.percentile(lat[common], 99))
        if st == storages[0]:
            continue
        # the served results against the first storage's, request by request (every 8th request
        # that both completed): the error a lower-precision storage adds to what it serves
        keys = sorted(set(sample) & set(samples[0]))
        errs = {f: [] for f in ("rho", "u", "T")}
        for k in keys:
            for f, a, b in zip(("rho", "u", "T"), sample[k], samples[0][k]):
                a64, b64 = a.astype(np.float64), b.astype(np.float64)
                errs[f].append(float(np.linalg.norm(a64 - b64) / np.linalg.norm(b64)))
        if keys:
            out[st]["rel_l2_vs_" + storages[0]] = {
                "sampled_requests": len(keys),
                **{f: {"median": float(np.median(v)), "max": float(np.max(v))} for f, v in errs.items()}}
    return out


def _test_helpers():
    """The tests' exact Riemann solution and damped-cosine fit (analysis, not the method)."""
    path = os.path.join(ROOT, "tests")
    if path not in sys.path:
        sys.path.insert(0, path)
    import fitting
    import riemann
    return fitting, riemann


def run_sod(n=400, t_exact=75, steps=1000, tau=0.8):
    """Shock tube on an n x 1 x 1 periodic D3Q19 lattice, FP64: the density at t = 75 (before the
    periodic images interact) against the exact Riemann solution (gamma = 5/3), the invariants'
    drift over the full 1000 steps, and the step rate."""
    import numpy as np
    from paper_2501_00620_amd import lbm, workloads
    _, riemann = _test_helpers()
    rho, u, T = workloads.sod(n, x0=n // 2)
    lat = lbm.Lattice(n, 1, 1, tau, storage="f64")
    lat.set_fields(rho, u, T)
    i0 = lat.invariants()
    lat.step(t_exact)
    r = lat.moments()[0].cpu().numpy().reshape(n)
    ex = riemann.RiemannSolution(1.0, 0.0, 1 / 3, 0.125, 0.0, 0.125 * 0.8 / 3, workloads.GAMMA)
    x = np.arange(n, dtype=float)
    re, _, _ = ex.profile(x, n / 2 - 0.5, float(t_exact))
    win = (x >= 110) & (x < 320)
    sp = ex.wave_speeds()
    xc, xs = n / 2 - 0.5 + sp["contact"] * t_exact, n / 2 - 0.5 + sp["right_shock"] * t_exact
    plateau_l = r[int(n / 2 - 0.5 + sp["left_tail"] * t_exact) + 4:int(xc) - 4].mean()
    plateau_r = r[int(xc) + 5:int(xs) - 5].mean()
    secs = timed_steps(lat, steps - t_exact, 0)
    i1 = lat.invariants()
    drift = np.abs((i1 - i0) / np.array([i0[0]] * 4 + [i0[4]])).max()
    out = {"l1_rel_density_t75": float(np.abs(r - re)[win].mean() / re[win].mean()),
           "plateau_left_rel_err": float(plateau_l / ex.rho_starL - 1),
           "plateau_right_rel_err": float(plateau_r / ex.rho_starR - 1),
           "invariant_drift_1000_steps": float(drift), "mlups": n * (steps - t_exact) / secs / 1e6,
           "workload": f"Sod tube {n} x 1 x 1, FP64, tau {tau}, rho 1 | 0.125, T 1/3 | 0.8/3"}
    print(f"[bench] Sod: L1 {out['l1_rel_density_t75']:.4f}, drift {drift:.1e}", file=sys.stderr, flush=True)
    return out


def run_acoustic(n=256, steps=5000, tau=0.6, every=4):
    """Gaussian pulse on an n x n x 1 lattice, FP32: the sound speed of Fourier modes
    k = 2 pi m / n (m = 1..4) fitted from the density's (m, 0) coefficient, against
    sqrt(5 T / 3) (energy-conserving mode) and sqrt(T) (prescribed temperature)."""
    import numpy as np
    import torch
    from paper_2501_00620_amd import lbm, workloads
    fitting, _ = _test_helpers()
    rho, u, T = workloads.acoustic_pulse(n)
    T0 = float(T.flat[0])
    out = {"workload": f"acoustic pulse {n}^2 x 1, FP32, tau {tau}, {steps} steps"}
    for mode, c2 in (("thermal", 5.0 / 3.0 * T0), ("iso", T0)):
        lat = lbm.Lattice(n, n, 1, tau, storage="f32", mode=mode)
        lat.set_fields(rho, u, T)
        ts, amps = [], []
        for t in range(0, steps + 1, every):
            if t:
                lat.step(every)
            r = lat.moments()[0].reshape(n, n).double()
            amps.append(torch.fft.rfft(r.mean(dim=0) - 1.0)[1:5].real.cpu().numpy())
            ts.append(t)
        amps = np.array(amps)
        ratios = []
        for m in range(1, 5):
            k = 2 * np.pi * m / n
            w, g = fitting.fit_damped_cosine(ts, amps[:, m - 1], k, np.sqrt(c2), k * k * T0 * tau,
                                             offset=(mode == "thermal"))
            ratios.append(float((w * w + g * g) / (k * k) / c2))
        out[mode] = {"cs2_over_predicted": ratios, "predicted_cs2": c2}
        if mode == "thermal":
            out["mlups"] = n * n * 1000 / timed_steps(lat, 1000, 0) / 1e6
        del lat
    print(f"[bench] acoustic: c_s^2 ratios thermal {out['thermal']['cs2_over_predicted']}, "
          f"iso {out['iso']['cs2_over_predicted']}", file=sys.stderr, flush=True)
    return out


def run_large(n=512, steps=500, tau=0.6, seed=5):
    """Random smooth fields on a 512^3 lattice in FP16-deviation storage, against the same run in
    FP32 storage: MLUPS, achieved algorithmic GB/s, and the relative L2 error of rho, u, T."""
    import torch
    from paper_2501_00620_amd import lbm, workloads
    rho, u, T = workloads.fourier_fields(n, n, n, seed=seed)
    res, out = {}, {"workload": f"Fourier fields {n}^3, tau {tau}, {steps} steps"}
    for storage in ("f32", "f16dev"):
        lat = lbm.Lattice(n, n, n, tau, storage=storage)
        lat.set_fields(rho, u, T)
        secs = timed_steps(lat, steps, 5)
        res[storage] = [x.double() for x in lat.moments()]
        bpv = BYTES_PER_VALUE[storage]
        out[storage] = {"mlups": n ** 3 * steps / secs / 1e6, "ms_per_step": secs * 1e3 / steps,
                        "achieved_gbs": n ** 3 * VALUES_PER_LUP * bpv / (secs / steps) / 1e9,
                        "nonfinite_sites": lat.health()[0]}
        out[storage]["frac"] = out[storage]["achieved_gbs"] / HBM_PEAK_GBS
        del lat
        torch.cuda.empty_cache()
    out["f16dev"]["rel_l2_vs_f32"] = {q: rel_l2(a, b) for q, a, b in zip(("rho", "u", "T"), res["f16dev"], res["f32"])}
    print(f"[bench] 512^3: f32 {out['f32']['mlups']:.0f}, f16dev {out['f16dev']['mlups']:.0f} MLUPS",
          file=sys.stderr, flush=True)
    return out


def run_standard(n, tau, mach, steps, warmup):
    """The standard lattice Boltzmann comparator (mode "standard") on the same Taylor-Green
    input: one kernel per step moving 2 x 19 values per site (it carries no variance)."""
    import torch
    from paper_2501_00620_amd import lbm, workloads
    rho, u, T = workloads.taylor_green(n, mach=mach)
    lat = lbm.Lattice(n, n, n, tau, storage="f32", mode="standard")
    lat.set_fields(rho, u, T)
    secs = timed_steps(lat, steps, warmup)
    health = lat.health()
    del lat
    torch.cuda.empty_cache()
    achieved = n ** 3 * 2 * 19 * 4 / (secs / steps) / 1e9
    print(f"[bench] standard comparator: {n ** 3 * steps / secs / 1e6:.0f} MLUPS", file=sys.stderr, flush=True)
    return {"mlups": n ** 3 * steps / secs / 1e6, "ms_per_step": secs * 1e3 / steps,
            "achieved_gbs": achieved, "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_site": 2 * 19 * 4,
            "nonfinite_sites": health[0], "workload": f"Taylor-Green vortex {n}^3, Mach {mach}, tau {tau}, FP32"}


def run_mrt(n, tau, mach, steps, warmup, tau_ghost=0.5):
    """The multiple-relaxation-time step (non-hydrodynamic moments of Table I at their own rate)
    beside the single-rate step on the same Taylor-Green input, FP32: in the split fused sweep
    (the default kernel) and in the two-pass kernel."""
    import torch
    from paper_2501_00620_amd import lbm, workloads
    rho, u, T = workloads.taylor_green(n, mach=mach)
    out = {"tau_ghost": tau_ghost, "workload": f"Taylor-Green vortex {n}^3, Mach {mach}, tau {tau}, FP32"}
    for kernel, prefix in (("auto", "fused_"), ("two_pass", "")):
        for name, tg in (("single_rate_mlups", None), ("mrt_mlups", tau_ghost)):
            lat = lbm.Lattice(n, n, n, tau, storage="f32", kernel=kernel)
            if tg is not None:
                lat.set_ghost_relaxation(tg)
            lat.set_fields(rho, u, T)
            secs = timed_steps(lat, steps, warmup)
            out[prefix + name] = n ** 3 * steps / secs / 1e6
            del lat
            torch.cuda.empty_cache()
    print(f"[bench] MRT: split sweep single rate {out['fused_single_rate_mlups']:.0f}, MRT {out['fused_mrt_mlups']:.0f}; "
          f"two-pass single rate {out['single_rate_mlups']:.0f}, MRT {out['mrt_mlups']:.0f} MLUPS",
          file=sys.stderr, flush=True)
    return out


def body_force(n=256, tau=0.55, mach=0.5, steps=100, N=64, T0=0.2, tau_k=0.6, A=1e-6, k_steps=8000):
    """Body force: the fused sweep (the split sweep of FP32) with a uniform acceleration and with
    the same acceleration as a field, and the two-pass step with the uniform one, on the
    Taylor-Green input; and the Kolmogorov flow a_y = A sin(kx) on the GPU, whose steady amplitude
    is A / (T tau k^2)."""
    import numpy as np
    import torch
    from paper_2501_00620_amd import lbm, workloads
    rho, u, T = workloads.taylor_green(n, mach=mach)
    out = {"workload": f"Taylor-Green vortex {n}^3 FP32 with a uniform acceleration; Kolmogorov flow {N} x 1 x 1, "
                       f"T {T0}, tau {tau_k}, {k_steps} steps"}
    for kernel, field, key in (("auto", False, "fused_mlups"), ("auto", True, "fused_field_mlups"),
                               ("two_pass", False, "two_pass_mlups")):
        lat = lbm.Lattice(n, n, n, tau, storage="f32", kernel=kernel)
        lat.set_fields(rho, u, T)
        lat.set_body_force([0.0, 1e-5, 0.0], field=field)
        secs = timed_steps(lat, steps, 5)
        out[key] = n ** 3 * steps / secs / 1e6
        del lat
        torch.cuda.empty_cache()
    k = 2 * np.pi / N
    x = np.arange(N)
    g = lbm.Lattice(N, 1, 1, tau_k, storage="f64", mode="iso")
    g.set_fields(np.ones((1, 1, N)), np.zeros((3, 1, 1, N)), np.full((1, 1, N), T0))
    accel = np.zeros((3, 1, 1, N))
    accel[1, 0, 0] = A * np.sin(k * x)
    g.set_body_force(accel)
    g.step(k_steps)
    uy = g.moments()[1][1].cpu().numpy().reshape(N)
    out["kolmogorov_amplitude_over_predicted"] = float(2.0 / N * np.sum(uy * np.sin(k * x)) / (A / (T0 * tau_k * k * k)))
    print(f"[bench] body force: fused {out['fused_mlups']:.0f} (as a field {out['fused_field_mlups']:.0f}), "
          f"two-pass {out['two_pass_mlups']:.0f} MLUPS, "
          f"Kolmogorov amplitude ratio "
          f"{out['kolmogorov_amplitude_over_predicted']:.4f}", file=sys.stderr, flush=True)
    return out


def walls(n=256, tau=0.55, mach=0.5, steps=100, nz=32, T0=1.0 / 6.0, tau_c=0.8, ratio=2.0, U=0.02):
    """Walls: a 256^3 channel (walls at rest normal to z, a driving acceleration along y) on the
    Taylor-Green input, stepped by the split fused sweep (interior planes; the wall planes with the
    wall kernel) and by the two-pass step, beside the periodic split sweep with the same force;
    and the gravity Couette flow of the paper's
    Galilean test on the GPU, walls moving at (0, 2U) and at (-U, U) under a_z = -g with
    g = ratio T / nz (density ratio e^ratio), in the bump scheme (prescribed T) and the standard
    comparator, against the closed form u_y = (u_t - u_b)(1 - e^(g z'/T)) / (1 - e^(g H/T)) + u_b."""
    import numpy as np
    import torch
    from paper_2501_00620_amd import lbm, workloads
    rho, u, T = workloads.taylor_green(n, mach=mach)
    out = {"workload": f"channel {n}^3 FP32 (Taylor-Green input, walls normal to z, uniform acceleration); "
                       f"gravity Couette {nz} x 1 x 1, T {T0:.4g}, tau {tau_c}, density ratio e^{ratio:g}, "
                       f"U {U}, {40 * nz * nz} steps"}
    for kernel, with_walls, key in (("auto", True, "fused_mlups"), ("two_pass", True, "two_pass_mlups"),
                                    ("auto", False, "periodic_fused_mlups")):
        lat = lbm.Lattice(n, n, n, tau, storage="f32", kernel=kernel)
        lat.set_fields(rho, u, T)
        if with_walls:
            lat.set_walls()
        lat.set_body_force([0.0, 1e-5, 0.0])
        secs = timed_steps(lat, steps, 5)
        out[key] = n ** 3 * steps / secs / 1e6
        del lat
        torch.cuda.empty_cache()
    out["fused_over_periodic"] = out["fused_mlups"] / out["periodic_fused_mlups"]
    g = ratio * T0 / nz
    zp = np.arange(nz) + 0.5
    for mode in ("iso", "standard"):
        prof = []
        for ub, ut in ((0.0, 2 * U), (-U, U)):
            exact = (ut - ub) * (1 - np.exp(g / T0 * zp)) / (1 - np.exp(g / T0 * nz)) + ub
            r0 = np.exp(-g / T0 * zp)
            u0 = np.zeros((3, nz, 1, 1))
            u0[1, :, 0, 0] = exact
            c = lbm.Lattice(1, 1, nz, tau_c, storage="f64", mode=mode)
            c.set_fields((r0 / r0.mean()).reshape(nz, 1, 1), u0, np.full((nz, 1, 1), T0))
            c.set_walls([0, ub, 0], [0, ut, 0])
            c.set_body_force([0.0, 0.0, -g])
            c.step(40 * nz * nz)
            prof.append((c.moments()[1][1].cpu().numpy().reshape(nz), exact))
        key = "bump" if mode == "iso" else "standard"
        out[key] = {"max_err_over_2U": float(max(np.abs(p - e).max() for p, e in prof) / (2 * U)),
                    "frame_difference_over_U": float(np.abs(prof[0][0] - U - prof[1][0]).max() / U)}
    print(f"[bench] walls: channel {out['fused_mlups']:.0f} MLUPS fused ({out['fused_over_periodic']:.3f} of periodic "
          f"{out['periodic_fused_mlups']:.0f}), two-pass {out['two_pass_mlups']:.0f}; gravity Couette frame difference "
          f"bump {out['bump']['frame_difference_over_U']:.3f} U, standard {out['standard']['frame_difference_over_U']:.3f} U",
          file=sys.stderr, flush=True)
    return out


# Algorithmic bytes per site update of the projected one-launch step, FP32: the state read once
# and written once (12 values per site D2Q9 ISO, 18 THERMAL, 4 D1Q3 ISO, 8 THERMAL).
PROJ_BYTES = {(2, "iso"): 2 * 4 * 12, (2, "thermal"): 2 * 4 * 18, (1, "iso"): 2 * 4 * 4, (1, "thermal"): 2 * 4 * 8}


def projections(n2=4096, n1=1 << 24, tau=0.6, steps=200):
    """Projected lattices against the D3Q19 layout on the same planar (n2 x n2 x 1) and linear
    (n1 x 1 x 1) lattices, FP32, random smooth fields without transverse velocity: MLUPS of each,
    GB/s of the projected step (PROJ_BYTES), and the largest relative difference of the moments
    after the timed steps (the two layouts compute the same step)."""
    import numpy as np
    import torch
    from paper_2501_00620_amd import lbm, workloads
    out = {"workload": f"planar {n2} x {n2} x 1 and linear {n1} x 1 x 1, FP32, tau {tau}, {steps} steps"}
    for dims, shape in ((2, (n2, n2)), (1, (n1, 1))):
        rho, u, T = workloads.fourier_fields(shape[0], shape[1], 1, seed=7, u_max=0.1)
        u = np.array(u)
        u[2] = 0.0
        if dims == 1:
            u[1] = 0.0
        for mode in ("iso", "thermal"):
            rec = {}
            mom = []
            for proj in (3, dims):
                lat = lbm.Lattice(shape[0], shape[1], 1, tau, storage="f32", mode=mode)
                lat.set_projection(proj)
                lat.set_fields(rho, u, T)
                secs = timed_steps(lat, steps, 5)
                rec["d3q19_mlups" if proj == 3 else "projected_mlups"] = shape[0] * shape[1] * steps / secs / 1e6
                mom.append([q.double() for q in lat.moments()])
                del lat
                torch.cuda.empty_cache()
            rec["projected_GBps"] = rec["projected_mlups"] * PROJ_BYTES[(dims, mode)] / 1e3
            rec["speedup"] = rec["projected_mlups"] / rec["d3q19_mlups"]
            rec["max_rel_diff"] = max(rel_l2(a, b) for a, b in zip(mom[1], mom[0]))
            out[f"{'d2q9' if dims == 2 else 'd1q3'}_{mode}"] = rec
            print(f"[bench] {'D2Q9' if dims == 2 else 'D1Q3'} {mode}: {rec['projected_mlups']:.0f} MLUPS "
                  f"({rec['projected_GBps']:.0f} GB/s) vs D3Q19 {rec['d3q19_mlups']:.0f}", file=sys.stderr, flush=True)
    return out


def galilean_contrast(U=0.2, N=64, T0=1.0 / 3.0, tau=0.6, steps=2000, every=50):
    """The paper's Galilean-invariance contrast on the GPU: a shear wave u_y(x) on a background
    flow U along x decays with nu = T tau in the bump scheme and, by the standard scheme's third
    moment, with nu = tau (1/3 - U^2) in the standard one.  FP64 storage, N x 1 x 1 lattice."""
    import numpy as np
    from paper_2501_00620_amd import lbm
    k = 2 * np.pi / N
    x = np.arange(N)
    out = {"U": U, "T": T0, "tau": tau, "N": N, "predicted_standard": 1 - U * U / T0}
    for mode in ("thermal", "standard"):
        lat = lbm.Lattice(N, 1, 1, tau, storage="f64", mode=mode)
        u = np.zeros((3, 1, 1, N))
        u[0] = U
        u[1] = 1e-3 * np.sin(k * x)
        lat.set_fields(np.ones((1, 1, N)), u, np.full((1, 1, N), T0))
        ts, amp = [], []
        for t in range(0, steps + 1, every):
            if t:
                lat.step(every)
            uy = lat.moments()[1][1].cpu().numpy().reshape(N)
            ts.append(t)
            amp.append(np.hypot(uy @ np.sin(k * x), uy @ np.cos(k * x)))
        nu = -np.polyfit(np.array(ts[4:], float), np.log(amp[4:]), 1)[0] / k ** 2
        out["nu_over_Ttau_" + ("bump" if mode == "thermal" else "standard")] = nu / (T0 * tau)
    print(f"[bench] Galilean contrast at U={U}: bump {out['nu_over_Ttau_bump']:.4f}, "
          f"standard {out['nu_over_Ttau_standard']:.4f}", file=sys.stderr, flush=True)
    return out


def oracle_rate(seconds, n=48, mach=0.5, tau=0.55):
    """MLUPS of the FP64 CPU oracle as it stands on a Taylor-Green vortex n^3, stepping for about
    `seconds` (OpenMP threads from OMP_NUM_THREADS).  Returns (mlups, steps, seconds)."""
    import oracle
    from paper_2501_00620_amd import workloads
    rho, u, T = workloads.taylor_green(n, mach=mach)
    o = oracle.OracleLattice(n, n, n, tau)
    o.init(rho, u, T)
    o.step(1)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    return n ** 3 * steps / dt / 1e6, steps, dt


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds=10.0, n=48, mach=0.5, tau=0.55):
    """The oracle timed on this host: with OpenMP on all the threads OMP_NUM_THREADS allows
    (the reported value), and on one core in a child process (OMP_NUM_THREADS=1)."""
    import subprocess
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    mlups, steps, dt = oracle_rate(seconds, n, mach, tau)
    child = subprocess.run(
        [sys.executable, "-c", f"import json, bench; print(json.dumps(bench.oracle_rate({seconds}, {n}, {mach}, {tau})))"],
        cwd=ROOT, env={**os.environ, "OMP_NUM_THREADS": "1"}, capture_output=True, text=True)
    one = json.loads(child.stdout.strip().splitlines()[-1]) if child.returncode == 0 else None
    return {"value": round(mlups, 2), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"Taylor-Green vortex {n}^3, Mach {mach}, tau {tau}, FP64, {steps} steps "
                      f"({dt:.1f} s) on {threads} OpenMP threads",
            "single_core": None if one is None else {
                "value": round(one[0], 3), "unit": "MLUPS", "cores": 1,
                "sample": f"the same lattice, {one[1]} steps ({one[2]:.1f} s) on 1 thread"},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def copy_ceiling(nbytes=1 << 30, reps=10):
    """Bandwidth of a plain device copy (bytes read + written per second): the rate this GPU's
    HBM sustains for a simple stream, beside the 8 TB/s peak."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes * reps / secs / 1e9


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--kernel", default="auto")
    ap.add_argument("--variant-steps", type=int, default=2000)
    ap.add_argument("--quick", action="store_true", help="skip the precision variants and the CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-only", action="store_true", help="run only the served-batch workload")
    ap.add_argument("--projections-only", action="store_true", help="run only the projected-lattice workload")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the sweep has no multi-GPU path (a z-slab decomposition "
              "is designed, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    from paper_2501_00620_amd import lbm, workloads
    if args.serve_only:
        print(json.dumps({"served": run_served_comparison(n_requests=args.serve_requests)}))
        return
    if args.projections_only:
        print(json.dumps({"projections": projections()}))
        return
    n, tau, mach = args.n, 0.55, 0.5
    # the copy ceiling first: it also brings the device out of idle before the timed steps
    copy_gbs = copy_ceiling()
    rho, u, T = workloads.taylor_green(n, mach=mach)
    lat = lbm.Lattice(n, n, n, tau, storage=args.storage, kernel=args.kernel)
    lat.set_fields(rho, u, T)
    torch.cuda.synchronize()
    per_step = timed_windows(lat, args.steps, args.warmup)
    secs_step = float(np.median(per_step))
    print(f"[bench] timed {args.steps} steps in {len(per_step)} windows: median {secs_step * 1e3:.3f} ms/step "
          f"({', '.join(f'{t * 1e3:.3f}' for t in per_step)})", file=sys.stderr, flush=True)
    health = lat.health()
    sites = n ** 3
    ms_per_step = secs_step * 1e3
    mlups = sites / secs_step / 1e6
    bytes_per_step = sites * VALUES_PER_LUP * BYTES_PER_VALUE[args.storage]
    achieved = bytes_per_step / secs_step / 1e9
    kname = step_kernel(args.kernel, args.storage, n)
    workload = f"tgv{n}_{args.storage}"
    traffic = traffic_from_profiles(kname, workload, sites)
    del lat
    torch.cuda.empty_cache()

    line = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "timing": {"windows": len(per_step), "ms_per_step_each": [round(t * 1e3, 4) for t in per_step],
                   "statistic": "median over consecutive windows of the K timed steps"},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.storage == "f32" else args.storage,
        "data": "synthetic (seeded Taylor-Green vortex initial fields)",
        "config": {"workload": f"3-D compressible Taylor-Green vortex {n}^3 periodic D3Q19, Mach {mach}, "
                               f"tau {tau}, {args.storage} storage", "nx": n, "ny": n, "nz": n, "tau": tau,
                   "mach": mach, "storage": args.storage, "mode": "thermal", "kernel": kname,
                   "health_nonfinite_sites": health[0]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_step,
                     "copy_ceiling": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
    }
    if not args.quick:
        line["variants"] = run_variants(n, args.variant_steps, tau, mach)
        line["served"] = run_served_comparison(n_requests=args.serve_requests)
        line["configs"] = {"sod": run_sod(), "acoustic": run_acoustic(), "large": run_large()}
        line["comparator"] = {"standard": run_standard(n, tau, mach, args.steps, args.warmup),
                              "galilean": galilean_contrast(),
                              "mrt": run_mrt(n, tau, mach, args.steps, args.warmup),
                              "body_force": body_force(),
                              "walls": walls()}
        line["projections"] = projections()
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
