"""ctypes binding of the FP64 CPU oracle (``lbm_oracle.c``). Test infrastructure only.

Array conventions follow the C side: structure of arrays, x fastest.
  F   (19, nz, ny, nx)  post-stream auxiliary populations fbar_i
  b   (6, nz, ny, nx)   auxiliary variance bbar, components xx yy zz xy xz yz
  rho (nz, ny, nx), u (3, nz, ny, nx), T (nz, ny, nx)
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib_path():
    return _build.LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build(force=False)
        _lib = C.CDLL(_build.LIB)
        d, i, l = C.c_double, C.c_int, C.c_long
        P = C.POINTER(C.c_double)
        _lib.orc_feq.argtypes = [d, d, d, d, P]
        _lib.orc_beq.argtypes = [d, d, d, d, P]
        _lib.orc_table_m.argtypes = [P]
        _lib.orc_forcing.argtypes = [P, P, P]
        _lib.orc_velocity_set.argtypes = [C.POINTER(C.c_int), P]
        _lib.orc_gradient.argtypes = [i, i, i, P, i, P]
        _lib.orc_init.argtypes = [i, i, i, P, P, P, P, P]
        _lib.orc_step.argtypes = [i, i, i, d, i, P, P, P, l]
        _lib.orc_step.restype = i
        _lib.orc_step_mrt.argtypes = [i, i, i, d, d, i, P, P, P, l]
        _lib.orc_step_mrt.restype = i
        _lib.orc_step_ext.argtypes = [i, i, i, d, d, i, P, P, P, P, l]
        _lib.orc_step_ext.restype = i
        _lib.orc_moments_ext.argtypes = [i, i, i, d, i, P, P, P, P, P, P, P]
        _lib.orc_moments_ext.restype = i
        _lib.orc_moments.argtypes = [i, i, i, d, i, P, P, P, P, P, P]
        _lib.orc_moments.restype = i
        _lib.orc_forcing_moments.argtypes = [i, i, i, d, i, P, P, P, P, P]
        _lib.orc_forcing_moments.restype = i
        _lib.orc_invariants.argtypes = [i, i, i, P, P, P]
        _lib.orc_step_sites.argtypes = [i, i, i, d, i, P, P, P, l, C.POINTER(C.c_long), P, P, P]
        _lib.orc_step_sites.restype = i
        _lib.orc_feq_std.argtypes = [d, d, d, d, d, P]
        _lib.orc_init_std.argtypes = [i, i, i, P, P, P, P]
        _lib.orc_step_std.argtypes = [i, i, i, d, P, P, l]
        _lib.orc_step_std.restype = i
        _lib.orc_moments_std.argtypes = [i, i, i, P, P, P]
        _lib.orc_step_walls.argtypes = [i, i, i, d, d, i, P, P, P, P, P, l]
        _lib.orc_step_walls.restype = i
        _lib.orc_moments_walls.argtypes = [i, i, i, d, i, P, P, i, P, P, P, P, P]
        _lib.orc_moments_walls.restype = i
        _lib.orc_step_std_walls.argtypes = [i, i, i, d, P, P, P, P, l]
        _lib.orc_step_std_walls.restype = i
        _lib.orc_moments_std_ext.argtypes = [i, i, i, P, P, P, P]
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def velocity_set():
    """(e, w): the 19 velocities as int array (19, 3) and the weights (19,)."""
    e = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    _load().orc_velocity_set(e.ctypes.data_as(C.POINTER(C.c_int)), _p(w))
    return e, w


def feq(rho, ux, uy, uz):
    out = np.zeros(19)
    _load().orc_feq(float(rho), float(ux), float(uy), float(uz), _p(out))
    return out


def feq_std(rho, ux, uy, uz, T):
    """Equilibrium of the standard lattice Boltzmann comparator (Sec. I, Eq. 4), lattice units."""
    f = np.zeros(19)
    _load().orc_feq_std(float(rho), float(ux), float(uy), float(uz), float(T), _p(f))
    return f


def beq(ux, uy, uz, T):
    out = np.zeros(6)
    _load().orc_beq(float(ux), float(uy), float(uz), float(T), _p(out))
    return out


def table_m():
    m = np.zeros((19, 19))
    _load().orc_table_m(_p(m))
    return m


def forcing(Fv, S):
    """Phi_i from the force F (3,) and second-moment source S (6,: xx yy zz xy xz yz)."""
    Fv, S = _f64(Fv), _f64(S)
    out = np.zeros(19)
    _load().orc_forcing(_p(Fv), _p(S), _p(out))
    return out


def gradient(phi, axis):
    """Isotropic D3Q19 finite difference of a periodic field phi (nz, ny, nx) along axis 0=x."""
    phi = _f64(phi)
    nz, ny, nx = phi.shape
    out = np.zeros_like(phi)
    _load().orc_gradient(nx, ny, nz, _p(phi), int(axis), _p(out))
    return out


def projection_classes(dims):
    """Classes of the D3Q19 populations that share their in-plane velocity, for a flow that does
    not vary along z (dims=2: keys (e_x, e_y)) or along y and z (dims=1: keys e_x), in the order of
    the projected layout.  Returns (classes, et2): a list of index arrays and |e_t|^2 per
    population (the squared transverse speed)."""
    e, _ = velocity_set()
    if dims == 2:
        keys = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)]
        classes = [np.flatnonzero((e[:, 0] == kx) & (e[:, 1] == ky)) for kx, ky in keys]
        et2 = e[:, 2] ** 2
    else:
        classes = [np.flatnonzero(e[:, 0] == kx) for kx in (0, 1, -1)]
        et2 = e[:, 1] ** 2 + e[:, 2] ** 2
    return classes, et2


def project(F, b, dims, thermal):
    """A D3Q19 state of a flow without z (dims=2) or y, z (dims=1) dependence as class sums: F_c,
    then (thermal) G_c = sum |e_t|^2 f over the classes with transverse members; b as xx yy xy [zz]
    (dims=2) or xx [yy+zz] (dims=1).  F: (19, ...), b: (6, ...)."""
    classes, et2 = projection_classes(dims)
    Fp = [F[c].sum(axis=0) for c in classes]
    if thermal:
        Fp += [np.tensordot(et2[c], F[c], axes=1) for c in classes if et2[c].max() > 0]
    if dims == 2:
        bp = [b[0], b[1], b[3]] + ([b[2]] if thermal else [])
    else:
        bp = [b[0]] + ([b[1] + b[2]] if thermal else [])
    return np.stack(Fp), np.stack(bp)


# thermal: temperature from the total second moment; iso: prescribed temperature field;
# standard: the standard lattice Boltzmann comparator (Sec. I, Eq. 4; no variance, prescribed T)
MODES = {"thermal": 0, "iso": 1, "standard": 2}


class OracleLattice:
    """An nx*ny*nz lattice stepped by the oracle, state held in numpy arrays. Periodic in x and y;
    in z periodic, or bounded by two moving walls (set_walls)."""

    def __init__(self, nx, ny, nz, tau, mode="thermal", T_field=None, tau_ghost=None):
        """tau_ghost: relaxation time of the non-hydrodynamic moments (rows 11-19 of Table I);
        None keeps the single relaxation time tau."""
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n = self.nx * self.ny * self.nz
        self.tau = float(tau)
        self.tau_ghost = self.tau if tau_ghost is None else float(tau_ghost)
        self.accel = None  # body-force acceleration field (3, nz, ny, nx), or None
        self.walls = None  # (u_bottom, u_top) as 6 float64 values, or None (periodic in z)
        self.mode = MODES[mode]
        shape = (self.nz, self.ny, self.nx)
        self.F = np.zeros((19,) + shape)
        self.b = np.zeros((6,) + shape)
        if T_field is None:
            T_field = np.zeros(shape)
        self.T_field = _f64(np.broadcast_to(T_field, shape))
        self.steps = 0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def init(self, rho, u, T):
        rho = _f64(np.broadcast_to(rho, self.shape))
        u = _f64(np.broadcast_to(u, (3,) + self.shape))
        T = _f64(np.broadcast_to(T, self.shape))
        if self.mode in (1, 2):
            self.T_field = T.copy()
        if self.mode == 2:
            self.b = np.zeros((6,) + self.shape)
            _load().orc_init_std(self.nx, self.ny, self.nz, _p(rho), _p(u), _p(T), _p(self.F))
        else:
            _load().orc_init(self.nx, self.ny, self.nz, _p(rho), _p(u), _p(T), _p(self.F), _p(self.b))
        self.steps = 0

    def set_body_force(self, accel):
        """Body-force acceleration field (3, nz, ny, nx) or a 3-vector; None removes it."""
        if accel is None:
            self.accel = None
        else:
            self.accel = _f64(np.broadcast_to(np.asarray(accel, dtype=np.float64).reshape(
                (3,) + (1,) * 3 if np.size(accel) == 3 else (3,) + self.shape), (3,) + self.shape))

    def set_walls(self, u_bottom=None, u_top=None, on=True):
        """Walls normal to z half-way outside the first and last planes (half-way bounce-back),
        moving with the tangential velocities u_bottom and u_top (3-vectors, default at rest).
        on=False restores the periodic z direction."""
        if not on:
            self.walls = None
            return
        ub = np.zeros(3) if u_bottom is None else np.asarray(u_bottom, dtype=np.float64).reshape(3)
        ut = np.zeros(3) if u_top is None else np.asarray(u_top, dtype=np.float64).reshape(3)
        self.walls = _f64(np.concatenate([ub, ut]))

    def set_state(self, F, b):
        self.F = _f64(F).reshape((19,) + self.shape).copy()
        self.b = _f64(b).reshape((6,) + self.shape).copy()

    def state(self):
        return self.F.copy(), self.b.copy()

    def step(self, n=1):
        acc = None if self.accel is None else _p(self.accel)
        uw = None if self.walls is None else _p(self.walls)
        if self.mode == 2:
            rc = _load().orc_step_std_walls(self.nx, self.ny, self.nz, self.tau, _p(self.T_field), acc, uw,
                                            _p(self.F), int(n))
        else:
            rc = _load().orc_step_walls(self.nx, self.ny, self.nz, self.tau, self.tau_ghost, self.mode,
                                        _p(self.T_field), acc, uw, _p(self.F), _p(self.b), int(n))
        if rc == -3:
            raise ValueError("walls need nz >= 3 and tangential wall velocities")
        if rc != 0:
            raise MemoryError("oracle step failed")
        self.steps += int(n)

    def moments(self):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        T = np.zeros(self.shape)
        acc = None if self.accel is None else _p(self.accel)
        if self.mode == 2:
            _load().orc_moments_std_ext(self.nx, self.ny, self.nz, acc, _p(self.F), _p(rho), _p(u))
            return rho, u, self.T_field.copy()
        rc = _load().orc_moments_walls(self.nx, self.ny, self.nz, self.tau, self.mode, _p(self.T_field), acc,
                                       int(self.walls is not None), _p(self.F), _p(self.b), _p(rho), _p(u), _p(T))
        if rc != 0:
            raise MemoryError("oracle moments failed")
        return rho, u, T

    def forcing_moments(self):
        Fv = np.zeros((3,) + self.shape)
        S = np.zeros((6,) + self.shape)
        rc = _load().orc_forcing_moments(self.nx, self.ny, self.nz, self.tau, self.mode,
                                         _p(self.T_field), _p(self.F), _p(self.b), _p(Fv), _p(S))
        if rc != 0:
            raise MemoryError("oracle forcing moments failed")
        return Fv, S

    def invariants(self):
        out = np.zeros(5)
        _load().orc_invariants(self.nx, self.ny, self.nz, _p(self.F), _p(self.b), _p(out))
        return out

    def step_sites(self, sites, F=None, b=None, with_bstar=False):
        """One step evaluated only at flat site indices `sites` (of the given or held state).
        Returns (F, b) post-stream at the sites, plus bbar* (post-collision, before the gather)
        at the sites if with_bstar."""
        F = self.F if F is None else _f64(F).reshape((19,) + self.shape)
        b = self.b if b is None else _f64(b).reshape((6,) + self.shape)
        sites = np.ascontiguousarray(sites, dtype=np.int64)
        m = sites.size
        Fo = np.zeros((m, 19))
        bo = np.zeros((m, 6))
        bs = np.zeros((m, 6))
        rc = _load().orc_step_sites(self.nx, self.ny, self.nz, self.tau, self.mode,
                                    _p(self.T_field), _p(F), _p(b), m,
                                    sites.ctypes.data_as(C.POINTER(C.c_long)), _p(Fo), _p(bo), _p(bs))
        if rc != 0:
            raise ValueError("oracle step_sites failed (%d)" % rc)
        return (Fo, bo, bs) if with_bstar else (Fo, bo)
