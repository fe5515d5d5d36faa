"""Python binding of liblbm (ctypes): argument marshalling only.

Every step of the method runs in the HIP kernels behind the C ABI of ``include/lbm.h``; this
module passes torch tensors' device pointers and the current torch stream to it.  There is no
CPU fallback: if ``liblbm.so`` is missing or no HIP device is present, calls raise.

Array shapes (x fastest):  rho, T (nz, ny, nx);  u (3, nz, ny, nx);
state F (19, nz, ny, nx) and b (6, nz, ny, nx), float64.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK = 0
ERRORS = {-1: "ARG", -2: "OOM", -3: "HIP", -4: "DIVERGED", -5: "RANGE", -6: "BUSY", -7: "STATE"}
STORAGE = {"f64": 0, "f32": 1, "f16dev": 2, "bf16dev": 3}
MODE = {"thermal": 0, "iso": 1, "standard": 2}
KERNEL = {"auto": 0, "two_pass": 1, "fused": 2, "fused_pc": 3}


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblbm {ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class lbm_params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("tau", C.c_double),
                ("T_ref", C.c_double), ("rho_ref", C.c_double), ("storage", C.c_int), ("mode", C.c_int)]


_lib = None

# every symbol declared in include/lbm.h, with its ctypes signature
SIGNATURES = {
    "lbm_create": ([C.POINTER(lbm_params), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "lbm_set_fields": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int], C.c_int),
    "lbm_step": ([C.c_void_p, C.c_long], C.c_int),
    "lbm_get_moments": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int], C.c_int),
    "lbm_get_state": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "lbm_set_state": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "lbm_get_codec": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "lbm_get_raw": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "lbm_get_stored": ([C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.c_int], C.c_int),
    "lbm_invariants": ([C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "lbm_invariants_noalloc": ([C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "lbm_health": ([C.c_void_p, C.POINTER(C.c_long), C.POINTER(C.c_double)], C.c_int),
    "lbm_set_kernel": ([C.c_void_p, C.c_int], C.c_int),
    "lbm_set_ghost_relaxation": ([C.c_void_p, C.c_double], C.c_int),
    "lbm_set_body_force": ([C.c_void_p, C.c_void_p, C.c_int, C.c_int], C.c_int),
    "lbm_set_walls": ([C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "lbm_set_body_force_uniform": ([C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "lbm_set_projection": ([C.c_void_p, C.c_int], C.c_int),
    "lbm_get_projection": ([C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
    "lbm_sync": ([C.c_void_p], C.c_int),
    "lbm_destroy": ([C.c_void_p], None),
    "lbm_last_error": ([], C.c_char_p),
    "lbm_steps_done": ([C.c_void_p], C.c_long),
    "lbm_lattice_bytes": ([C.c_void_p], C.c_size_t),
    "lbm_server_create": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "lbm_server_submit": ([C.c_void_p, C.POINTER(lbm_params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                           C.c_long, C.POINTER(C.c_long)], C.c_int),
    "lbm_server_poll": ([C.c_void_p, C.c_long, C.POINTER(C.c_int), C.POINTER(C.c_double)], C.c_int),
    "lbm_server_wait": ([C.c_void_p, C.c_long, C.c_double], C.c_int),
    "lbm_server_fetch": ([C.c_void_p, C.c_long, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "lbm_server_release": ([C.c_void_p, C.c_long], C.c_int),
    "lbm_server_error": ([C.c_void_p, C.c_long], C.c_char_p),
    "lbm_server_stats": ([C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "lbm_server_destroy": ([C.c_void_p], None),
}


class lbm_server_params(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("bundle_steps", C.c_int), ("storage", C.c_int),
                ("max_lattices", C.c_int), ("health_every", C.c_int)]


REQ_STATUS = {0: "queued", 1: "running", 2: "done", 3: "failed"}


def load_library(path=LIB_PATH):
    """Load liblbm.so and declare its signatures; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
        lib = C.CDLL(path)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(rc):
    if rc != LBM_OK:
        raise LBMError(rc, _lib.lbm_last_error().decode())
    return rc


def _torch():
    import torch
    return torch


def _device_tensor(a, dtype, shape):
    """A contiguous CUDA tensor of `dtype` and `shape` holding `a` (numpy, CPU or CUDA tensor)."""
    torch = _torch()
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a))
    if not torch.is_tensor(a):
        a = torch.as_tensor(a)
    a = a.to(device="cuda", dtype=dtype)
    a = a.expand(shape) if tuple(a.shape) != tuple(shape) else a
    return a.contiguous()


class Lattice:
    """A periodic nx*ny*nz bump-function D3Q19 lattice resident on the current HIP device."""

    def __init__(self, nx, ny, nz, tau, storage="f32", mode="thermal", T_ref=1.0 / 3.0, rho_ref=1.0,
                 stream=None, kernel="auto"):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP device (torch.cuda.is_available() is False)")
        lib = load_library()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n = self.nx * self.ny * self.nz
        self.storage, self.mode, self.tau = storage, mode, float(tau)
        p = lbm_params(self.nx, self.ny, self.nz, float(tau), float(T_ref), float(rho_ref),
                       STORAGE[storage], MODE[mode])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib.lbm_create(C.byref(p), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.set_kernel(kernel)

    # -- lifetime ---------------------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def handle(self):
        return self._h

    def set_kernel(self, kernel):
        _check(_lib.lbm_set_kernel(self._h, KERNEL[kernel] if isinstance(kernel, str) else int(kernel)))

    def set_body_force(self, accel, field=False):
        """Body-force acceleration: an array (3, nz, ny, nx), a 3-vector (uniform; with
        field=True it is broadcast to a field instead), or None to remove it.  Both the fused and
        the two-pass step take it."""
        if accel is None:
            _check(_lib.lbm_set_body_force(self._h, None, 0, 0))
            return
        a = np.asarray(accel, dtype=np.float64)
        if a.size == 3 and not field:
            _check(_lib.lbm_set_body_force_uniform(self._h, (C.c_double * 3)(*a.reshape(3))))
            return
        shape = (3, self.nz, self.ny, self.nx)
        a = np.ascontiguousarray(np.broadcast_to(a.reshape(3, 1, 1, 1) if a.size == 3 else a, shape))
        _check(_lib.lbm_set_body_force(self._h, a.ctypes.data_as(C.c_void_p), 0, 0))

    def set_walls(self, u_bottom=None, u_top=None, on=True):
        """Walls normal to z half-way outside planes 0 and nz - 1 (half-way bounce-back), moving
        with the tangential velocities u_bottom and u_top (3-vectors, default at rest); on=False
        restores the periodic z direction.  A float or 16-bit lattice with walls steps its interior
        planes in the split fused sweep and its wall planes with the two-pass wall kernel; double
        precision steps two-pass."""
        if not on:
            _check(_lib.lbm_set_walls(self._h, 0, None, None))
            return
        vec = lambda v: (C.c_double * 3)(*(np.zeros(3) if v is None else np.asarray(v, np.float64).reshape(3)))
        _check(_lib.lbm_set_walls(self._h, 1, vec(u_bottom), vec(u_top)))

    def set_ghost_relaxation(self, tau_ghost):
        """Relaxation time of the non-hydrodynamic moments (Table I rows 11-19); tau_ghost = tau
        is the single-rate scheme.  In float and 16-bit storage it steps in the split fused sweep."""
        _check(_lib.lbm_set_ghost_relaxation(self._h, float(tau_ghost)))

    # -- fields and state -------------------------------------------------------------------------
    def _sync_torch(self):
        # tensors handed to the library were written on torch's current stream
        torch = _torch()
        if torch.cuda.current_stream().cuda_stream != self.stream.cuda_stream:
            torch.cuda.current_stream().synchronize()

    def set_fields(self, rho, u, T, dtype=None):
        torch = _torch()
        dt = dtype or torch.float64
        r = _device_tensor(rho, dt, self.shape)
        uu = _device_tensor(u, dt, (3,) + self.shape)
        t = _device_tensor(T, dt, self.shape)
        self._sync_torch()
        code = 0 if dt == torch.float64 else 1
        _check(_lib.lbm_set_fields(self._h, C.c_void_p(r.data_ptr()), C.c_void_p(uu.data_ptr()),
                                   C.c_void_p(t.data_ptr()), code, 1))

    def step(self, n=1):
        _check(_lib.lbm_step(self._h, int(n)))

    def sync(self):
        _check(_lib.lbm_sync(self._h))

    def moments(self, dtype=None):
        torch = _torch()
        dt = dtype or torch.float64
        rho = torch.empty(self.shape, dtype=dt, device="cuda")
        u = torch.empty((3,) + self.shape, dtype=dt, device="cuda")
        T = torch.empty(self.shape, dtype=dt, device="cuda")
        self._sync_torch()
        _check(_lib.lbm_get_moments(self._h, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr()),
                                    C.c_void_p(T.data_ptr()), 0 if dt == torch.float64 else 1, 1))
        return rho, u, T

    def projection(self):
        """(dims, nf, nb): 3 for D3Q19, else the projected lattice and its state planes."""
        d, f, b = C.c_int(), C.c_int(), C.c_int()
        _check(_lib.lbm_get_projection(self._h, C.byref(d), C.byref(f), C.byref(b)))
        return d.value, f.value, b.value

    def set_projection(self, dims):
        """Hold the lattice as a projected D2Q9 (dims=2, nz = 1) or D1Q3 (dims=1, ny = nz = 1)
        lattice of class sums, or as D3Q19 (dims=3).  Call before set_fields."""
        _check(_lib.lbm_set_projection(self._h, int(dims)))

    def get_state(self):
        """(F, b) in float64: 19 + 6 planes, or on a projected lattice the planes of projection()."""
        torch = _torch()
        _, nf, nb = self.projection()
        F = torch.empty((nf,) + self.shape, dtype=torch.float64, device="cuda")
        b = torch.empty((nb,) + self.shape, dtype=torch.float64, device="cuda")
        self._sync_torch()
        _check(_lib.lbm_get_state(self._h, C.c_void_p(F.data_ptr()), C.c_void_p(b.data_ptr()), 1))
        return F, b

    def get_stored(self):
        """(F, b, b_is_gathered): the stored representation decoded to float64 (no gather)."""
        torch = _torch()
        F = torch.empty((19,) + self.shape, dtype=torch.float64, device="cuda")
        b = torch.empty((6,) + self.shape, dtype=torch.float64, device="cuda")
        g = C.c_int()
        self._sync_torch()
        _check(_lib.lbm_get_stored(self._h, C.c_void_p(F.data_ptr()), C.c_void_p(b.data_ptr()), C.byref(g), 1))
        return F, b, bool(g.value)

    def set_state(self, F, b):
        torch = _torch()
        F = _device_tensor(F, torch.float64, (19,) + self.shape)
        b = _device_tensor(b, torch.float64, (6,) + self.shape)
        self._sync_torch()
        _check(_lib.lbm_set_state(self._h, C.c_void_p(F.data_ptr()), C.c_void_p(b.data_ptr()), 1))

    def codec(self):
        s = (C.c_double * 25)()
        r = (C.c_double * 25)()
        _check(_lib.lbm_get_codec(self._h, s, r))
        return np.array(s[:]), np.array(r[:])

    def raw_codes(self):
        torch = _torch()
        F = torch.empty((19,) + self.shape, dtype=torch.int16, device="cuda")
        b = torch.empty((6,) + self.shape, dtype=torch.int16, device="cuda")
        self._sync_torch()
        _check(_lib.lbm_get_raw(self._h, C.c_void_p(F.data_ptr()), C.c_void_p(b.data_ptr()), 1))
        return F.cpu().numpy().view(np.uint16), b.cpu().numpy().view(np.uint16)

    def invariants(self):
        out = (C.c_double * 5)()
        _check(_lib.lbm_invariants(self._h, out))
        return np.array(out[:])

    def invariants_noalloc(self, out=None):
        """lbm_invariants_noalloc: into `out`, a CUDA float64 tensor of 5 (enqueued on the
        lattice's stream, returned without waiting), or, if out is None, as a numpy array."""
        if out is None:
            res = (C.c_double * 5)()
            _check(_lib.lbm_invariants_noalloc(self._h, C.cast(res, C.c_void_p), 0))
            return np.array(res[:])
        torch = _torch()
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < 5 or not out.is_contiguous():
            raise ValueError("out must be a contiguous CUDA float64 tensor of at least 5 elements")
        _check(_lib.lbm_invariants_noalloc(self._h, C.c_void_p(out.data_ptr()), 1))
        return out

    def health(self):
        """(n_nonfinite, n_rho_nonpositive, max|u*|); raises LBMError DIVERGED if unhealthy."""
        cnt = (C.c_long * 2)()
        mx = C.c_double()
        rc = _lib.lbm_health(self._h, cnt, C.byref(mx))
        if rc not in (LBM_OK, -4):
            _check(rc)
        return int(cnt[0]), int(cnt[1]), float(mx.value)

    @property
    def steps_done(self):
        return int(_lib.lbm_steps_done(self._h))


def lattice_bytes(nx, ny, nz, storage="f32", mode="thermal"):
    """Device bytes a lattice of this shape and storage occupies."""
    lib = load_library()
    p = lbm_params(int(nx), int(ny), int(nz), 1.0, 1.0 / 3.0, 1.0, STORAGE[storage], MODE[mode])
    return int(lib.lbm_lattice_bytes(C.byref(p)))


def codec_reference(rho, T, rho_ref=None, T_ref=None):
    """(rho_ref, T_ref) of a lattice's deviation codec: the given values, else the mean density
    and mean temperature of the initial fields (else 1 and 1/3 when those are not usable; the
    fields themselves are then rejected where they are set)."""
    if rho_ref is None:
        m = float(np.mean(rho))
        rho_ref = m if np.isfinite(m) and m > 0 else 1.0
    if T_ref is None:
        m = float(np.mean(T))
        T_ref = m if np.isfinite(m) else 1.0 / 3.0
    return rho_ref, T_ref


class Server:
    """Continuous batching of many independent lattices (see include/lbm.h, lbm_server_*).

    Requests are submitted from host arrays and served by a worker thread inside the library;
    results come back as host (numpy) arrays."""

    def __init__(self, budget_bytes, bundle_steps=50, storage="f32", max_lattices=1024, health_every=0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP device (torch.cuda.is_available() is False)")
        lib = load_library()
        p = lbm_server_params(int(budget_bytes), int(bundle_steps), STORAGE[storage], int(max_lattices),
                              int(health_every))
        h = C.c_void_p()
        _check(lib.lbm_server_create(C.byref(p), None, C.byref(h)))
        self._h = h
        self.storage = storage
        self.shapes = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.lbm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, rho, u, T, tau, steps, mode="thermal", T_ref=None, rho_ref=None):
        """Queue one simulation (host arrays, copied).  The deviation codec's reference
        equilibrium defaults to the request's mean density (a conserved quantity) and mean
        temperature, which keeps stored deviations small where the density varies widely."""
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        nz, ny, nx = rho.shape
        u = np.ascontiguousarray(np.broadcast_to(u, (3, nz, ny, nx)), dtype=np.float64)
        T = np.ascontiguousarray(np.broadcast_to(T, (nz, ny, nx)), dtype=np.float64)
        rho_ref, T_ref = codec_reference(rho, T, rho_ref, T_ref)
        p = lbm_params(nx, ny, nz, float(tau), float(T_ref), float(rho_ref), STORAGE[self.storage], MODE[mode])
        rid = C.c_long()
        _check(_lib.lbm_server_submit(self._h, C.byref(p), rho.ctypes.data_as(C.c_void_p),
                                      u.ctypes.data_as(C.c_void_p), T.ctypes.data_as(C.c_void_p), 0,
                                      int(steps), C.byref(rid)))
        self.shapes[rid.value] = (nz, ny, nx)
        return rid.value

    def poll(self, rid):
        """(status, t_submit, t_admit, t_done); times in seconds on a monotonic clock."""
        st = C.c_int()
        t = (C.c_double * 3)()
        _check(_lib.lbm_server_poll(self._h, int(rid), C.byref(st), t))
        return REQ_STATUS[st.value], t[0], t[1], t[2]

    def wait(self, rid, timeout=120.0):
        _check(_lib.lbm_server_wait(self._h, int(rid), float(timeout)))
        return self.poll(rid)[0]

    def fetch(self, rid):
        shape = self.shapes[rid]
        rho = np.empty(shape)
        u = np.empty((3,) + shape)
        T = np.empty(shape)
        _check(_lib.lbm_server_fetch(self._h, int(rid), rho.ctypes.data_as(C.c_void_p),
                                     u.ctypes.data_as(C.c_void_p), T.ctypes.data_as(C.c_void_p), 0))
        return rho, u, T

    def release(self, rid):
        _check(_lib.lbm_server_release(self._h, int(rid)))
        self.shapes.pop(rid, None)

    def error(self, rid):
        return _lib.lbm_server_error(self._h, int(rid)).decode()

    def stats(self):
        out = (C.c_double * 8)()
        _check(_lib.lbm_server_stats(self._h, out))
        keys = ["resident_bytes", "running", "queued", "done", "failed", "bundles", "lattice_updates", "busy_s"]
        return dict(zip(keys, out[:]))
