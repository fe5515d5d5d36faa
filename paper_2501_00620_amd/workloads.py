"""Seeded synthetic initial fields (rho, u, T) for the benchmark workloads and the tests.

This module only draws and shapes initial macroscopic fields; it holds none of the lattice
Boltzmann arithmetic, so both the GPU path and the CPU oracle take their inputs from it.

All fields are float64 numpy arrays in lattice units (dx = dt = c = 1), structure of arrays with
x fastest: rho (nz, ny, nx), u (3, nz, ny, nx), T (nz, ny, nx).

T_REF = c^2/3 is the temperature at which the equilibrium variance vanishes at rest (Appendix A
with u = 0), i.e. where each bump collapses to a point mass and the rest state is the ordinary
D3Q19 weight set.  GAMMA = 5/3 is the heat-capacity ratio of the energy-conserving mode (three
translational degrees of freedom in the 3x3 variance tensor).
"""
import numpy as np

T_REF = 1.0 / 3.0
GAMMA = 5.0 / 3.0


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def uniform(nx, ny, nz, rho=1.0, u=(0.0, 0.0, 0.0), T=T_REF):
    shape = (nz, ny, nx)
    return (np.full(shape, float(rho)),
            np.stack([np.full(shape, float(c)) for c in u]),
            np.full(shape, float(T)))


def sod(n=400, x0=200, rho=(1.0, 0.125), T_ratio=0.8, T_left=T_REF):
    """1-D shock tube on an n x 1 x 1 periodic lattice: left state for x < x0."""
    x = np.arange(n)
    left = x < x0
    r = np.where(left, rho[0], rho[1]).reshape(1, 1, n)
    T = np.where(left, T_left, T_ratio * T_left).reshape(1, 1, n)
    return r.astype(np.float64), np.zeros((3, 1, 1, n)), T.astype(np.float64)


def acoustic_pulse(n=256, amplitude=1e-3, sigma=8.0, T=T_REF):
    """2-D Gaussian density bump at the centre of an n x n x 1 periodic lattice, at rest."""
    x, y, _ = _grid(n, n, 1)
    c = n / 2.0
    r2 = (x - c) ** 2 + (y - c) ** 2
    rho = 1.0 + amplitude * np.exp(-r2 / (2.0 * sigma * sigma))
    return rho, np.zeros((3, 1, n, n)), np.full((1, n, n), float(T))


def taylor_green(n=256, mach=0.5, T0=T_REF, gamma=GAMMA, rho0=1.0):
    """3-D compressible Taylor-Green vortex, U0 = Ma sqrt(gamma T0), isothermal initial T."""
    x, y, z = _grid(n, n, n)
    k = 2.0 * np.pi / n
    U0 = mach * np.sqrt(gamma * T0)
    u = np.stack([U0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z),
                  -U0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z),
                  np.zeros_like(x)])
    p = rho0 * T0 + rho0 * U0 * U0 / 16.0 * (np.cos(2 * k * x) + np.cos(2 * k * y)) * (np.cos(2 * k * z) + 2.0)
    return p / T0, u, np.full_like(x, T0)


def _fourier(rng, shape, modes=4, kmax=4):
    nz, ny, nx = shape
    x, y, z = _grid(nx, ny, nz)
    g = np.zeros(shape)
    for _ in range(modes):
        while True:
            kv = rng.integers(-kmax, kmax + 1, size=3)
            if np.any(kv != 0):
                break
        a = rng.uniform(0.5, 1.0)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        g += a * np.cos(2 * np.pi * (kv[0] * x / nx + kv[1] * y / ny + kv[2] * z / nz) + ph)
    return g


def fourier_fields(nx, ny, nz, seed, rho_amp=0.05, u_max=0.3, T_rel=0.1, T0=T_REF):
    """Random smooth periodic fields: 4-mode Fourier sums (integer wave vectors in [-4,4]^3),
    rho = 1 +- rho_amp, max|u| = u_max, T in [1 - T_rel, 1 + T_rel] T0.  numpy PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nz, ny, nx)

    def scaled(amp):
        g = _fourier(rng, shape)
        m = np.max(np.abs(g))
        return amp * g / m if m > 0 else g

    rho = 1.0 + scaled(rho_amp)
    u = np.stack([_fourier(rng, shape) for _ in range(3)])
    umag = np.sqrt(np.sum(u * u, axis=0)).max()
    u = u * (u_max / umag) if umag > 0 else u
    T = T0 * (1.0 + scaled(T_rel))
    return rho, u, T


def riemann2d_request(rng, n=None, n_range=(64, 512), T0=T_REF):
    """One served request: an n x n x 1 four-quadrant Riemann problem.  Per quadrant rho is
    log-uniform in [0.1, 1], T log-uniform in [0.5, 1] T0, u_x, u_y uniform in [-0.2, 0.2]."""
    if n is None:
        n = int(rng.integers(n_range[0], n_range[1] + 1))
    q_rho = np.exp(rng.uniform(np.log(0.1), np.log(1.0), size=4))
    q_T = T0 * np.exp(rng.uniform(np.log(0.5), np.log(1.0), size=4))
    q_u = rng.uniform(-0.2, 0.2, size=(4, 2))
    x, y, _ = _grid(n, n, 1)
    quad = (x >= n // 2).astype(int) + 2 * (y >= n // 2).astype(int)
    rho = q_rho[quad]
    T = q_T[quad]
    u = np.stack([q_u[quad, 0], q_u[quad, 1], np.zeros_like(rho)])
    return rho, u, T


def served_batch(n_requests=512, rate=50.0, seed=2024):
    """The served batch: Poisson arrival times (rate per second), grid edges n ~ U{64..512} and
    per-request field seeds, all drawn with numpy PCG64(seed).  Request k's fields are
    served_request(sizes[k], field_seeds[k])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    sizes = rng.integers(64, 513, size=n_requests)
    field_seeds = rng.integers(0, 1 << 62, size=n_requests)
    return arrivals, sizes, field_seeds


def served_request(n, field_seed):
    """Fields of one request of the served batch: an n x n x 1 four-quadrant Riemann problem."""
    return riemann2d_request(np.random.Generator(np.random.PCG64(int(field_seed))), n=int(n))
