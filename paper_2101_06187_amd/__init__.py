"""MI355X (gfx950) relativistic lattice Boltzmann library -- Python binding.

A thin ctypes layer over ``librlbm.so`` (C ABI in ``include/rlbm.h``): it
marshals arguments and uses PyTorch only for device memory and the current
HIP stream.  Every step of the method runs in the library's HIP kernels; there
is no CPU fallback -- if the library is missing, every call raises.

    import paper_2101_06187_amd as rl
    lat = rl.Lattice(512, 512, tau=0.55, storage="F32",
                     forcing=rl.Forcing(1e-5, 4, 6, seed=2))
    lat.set_state(e, ux, uy)          # float64 CUDA tensors [ny][nx]
    lat.step(1000)
    eps, bx, by, T = lat.fields()
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlbm.so")

STENCILS = {"SPH26": 0, "CIRC8": 1, "SPH26_ZFOLD": 2}
STORAGES = {"F64": 0, "F32": 1, "F16S": 2, "BF16S": 3}
KERNELS = {"tile": 0, "march": 1, "march2": 2, "staged": 3, "march_pairs": 4}
_KERNEL_NAMES = {v: k for k, v in KERNELS.items()}
RELAXATION = {"constant": 0, "eta_s": 1}

OK, EINVAL, ENOSPACE, EHIP, EUNSTABLE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5


class RlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rlbm error {code}: {msg}")
        self.code = code


class _Lattice(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("cfl", ctypes.c_double)]


class _Forcing(ctypes.Structure):
    _fields_ = [("amplitude", ctypes.c_double), ("k_lo", ctypes.c_double),
                ("k_hi", ctypes.c_double), ("seed", ctypes.c_uint64)]


@dataclass(frozen=True)
class Forcing:
    amplitude: float
    k_lo: float
    k_hi: float
    seed: int = 0

    def _c(self):
        return _Forcing(self.amplitude, self.k_lo, self.k_hi, self.seed)


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_D = ctypes.c_double

# (name, restype, argtypes) of every exported function of include/rlbm.h
SIGNATURES = [
    ("rlbm_status_string", ctypes.c_char_p, [_I]),
    ("rlbm_last_error", ctypes.c_char_p, []),
    ("rlbm_stencil_info", _I, [_I, _P, _P, _P]),
    ("rlbm_forcing_modes", _I, [_P, _P, _P, _P, _I32, _P]),
    ("rlbm_workspace_bytes", _I, [_P, _I, _I, _P, _P]),
    ("rlbm_init", _I, [_P, _P, _D, _I, _P, _I, _P, _SZ, _P]),
    ("rlbm_set_state", _I, [_P, _P, _P, _P]),
    ("rlbm_step", _I, [_P, _I64]),
    ("rlbm_check", _I, [_P]),
    ("rlbm_step_count", _I, [_P, _P]),
    ("rlbm_fields", _I, [_P, _P, _P, _P, _P]),
    ("rlbm_conserved", _I, [_P, _P]),
    ("rlbm_get_populations", _I, [_P, _P]),
    ("rlbm_set_populations", _I, [_P, _P]),
    ("rlbm_spectrum_scratch_bytes", _I, [_P, _P]),
    ("rlbm_spectrum", _I, [_P, _P, _SZ, _P, _I32, _P]),
    ("rlbm_spectrum_static", _I, [_P, _P, _I32, _P]),
    ("rlbm_filtered_velocity", _I, [_P, _P, _SZ, ctypes.c_double, ctypes.c_double, _P, _P, _P]),
    ("rlbm_spectrum_average", _I, [_P, _I32, _I32, _P, _P]),
    ("rlbm_shell_modes", _I, [_I32, _I32, _I32, _P]),
    ("rlbm_state_bytes", _I, [_P, _P]),
    ("rlbm_save", _I, [_P, _P, _SZ]),
    ("rlbm_load", _I, [_P, _P, _SZ]),
    ("rlbm_set_kernel", _I, [_P, _I32, _I32]),
    ("rlbm_get_kernel", _I, [_P, _P, _P]),
    ("rlbm_set_tile", _I, [_P, _I32]),
    ("rlbm_autotune", _I, [_P, _I32, _P]),
    ("rlbm_set_graph_chunk", _I, [_P, _I32]),
    ("rlbm_set_relaxation", _I, [_P, _I32]),
    ("rlbm_profile_step_kernel", _I, [_P, _I64, _P]),
    ("rlbm_stream_copy", _I, [_P, _P, _SZ, _I32, _P, _P]),
    ("rlbm_destroy", None, [_P]),
    ("rlbm_batch_workspace_bytes", _I, [_I32, _P, _I, _I, _P, _P]),
    ("rlbm_batch_init", _I, [_P, _I32, _P, _P, _I, _P, _I, _P, _SZ, _P]),
    ("rlbm_batch_set_state", _I, [_P, _I32, _P, _P, _P]),
    ("rlbm_batch_step", _I, [_P, _I64]),
    ("rlbm_batch_check", _I, [_P]),
    ("rlbm_batch_fields", _I, [_P, _I32, _P, _P, _P, _P]),
    ("rlbm_batch_get_populations", _I, [_P, _I32, _P]),
    ("rlbm_batch_set_graph_chunk", _I, [_P, _I32]),
    ("rlbm_batch_set_relaxation", _I, [_P, _I32]),
    ("rlbm_batch_set_kernel", _I, [_P, _I32, _I32]),
    ("rlbm_batch_get_kernel", _I, [_P, _P, _P]),
    ("rlbm_batch_step_count", _I, [_P, _P]),
    ("rlbm_batch_autotune", _I, [_P, _I32, _P]),
    ("rlbm_batch_destroy", None, [_P]),
]


def lib():
    """Load ``librlbm.so`` (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2101_06187_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        msg = lib().rlbm_last_error().decode(errors="replace")
        raise RlbmError(rc, msg or lib().rlbm_status_string(rc).decode())
    return rc


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _lattice(nx, ny, cfl):
    return _Lattice(int(nx), int(ny), float(cfl))


def stencil_info(stencil="SPH26"):
    """(v, w): the library's direction table (Q, 3) and weights (Q,)."""
    q = ctypes.c_int32()
    _check(lib().rlbm_stencil_info(STENCILS[stencil], ctypes.byref(q), None, None))
    v = np.zeros((q.value, 3))
    w = np.zeros(q.value)
    _check(lib().rlbm_stencil_info(STENCILS[stencil], ctypes.byref(q),
                                   v.ctypes.data_as(_P), w.ctypes.data_as(_P)))
    return v, w


def forcing_modes(nx, ny, forcing, cfl=1.0):
    """Driven (kx, ky) modes of a lattice in the library's numbering."""
    lat = _lattice(nx, ny, cfl)
    f = forcing._c()
    n = ctypes.c_int32()
    _check(lib().rlbm_forcing_modes(ctypes.byref(lat), ctypes.byref(f), None, None, 0,
                                    ctypes.byref(n)))
    kx = np.zeros(n.value, dtype=np.int32)
    ky = np.zeros(n.value, dtype=np.int32)
    _check(lib().rlbm_forcing_modes(ctypes.byref(lat), ctypes.byref(f), kx.ctypes.data_as(_P),
                                    ky.ctypes.data_as(_P), n.value, ctypes.byref(n)))
    return np.stack([kx, ky], axis=1)


def workspace_bytes(nx, ny, stencil="SPH26", storage="F64", forcing=None, cfl=1.0):
    lat = _lattice(nx, ny, cfl)
    out = ctypes.c_size_t()
    f = ctypes.byref(forcing._c()) if forcing is not None else None
    _check(lib().rlbm_workspace_bytes(ctypes.byref(lat), STENCILS[stencil], STORAGES[storage], f,
                                      ctypes.byref(out)))
    return out.value


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _f64(t, shape):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == shape):
        raise ValueError(f"expected a contiguous float64 CUDA tensor of shape {shape}")
    return t


def stream_copy(src, dst, reps=10):
    """Mean duration (ms) of one streaming copy of src (a CUDA tensor) into
    dst (same size, no overlap) by the library's copy kernel: the practical
    HBM streaming rate is 2 * bytes / time."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous CUDA tensors of the same size in bytes")
    ms = ctypes.c_double()
    _check(lib().rlbm_stream_copy(_ptr(src), _ptr(dst), nbytes, int(reps), _stream(src.device),
                                  ctypes.byref(ms)))
    return ms.value


def shell_modes(nx, ny, nbins):
    """Number of integer wave vectors in each shell of Lattice.spectrum; the
    shell sum divided by it is the average over the directions of k."""
    out = np.zeros(int(nbins), dtype=np.int64)
    _check(lib().rlbm_shell_modes(int(nx), int(ny), int(nbins), out.ctypes.data_as(_P)))
    return out


def spectrum_average(samples):
    """Time average and error estimate of sampled spectra (M x nbins array)."""
    a = np.ascontiguousarray(samples, dtype=np.float64)
    m, nb = a.shape
    mean, err = np.zeros(nb), np.zeros(nb)
    _check(lib().rlbm_spectrum_average(a.ctypes.data_as(_P), m, nb, mean.ctypes.data_as(_P),
                                       err.ctypes.data_as(_P)))
    return mean, err


class Lattice:
    """One periodic lattice advanced by the library (all work on the GPU)."""

    def __init__(self, nx, ny, tau, stencil="SPH26", storage="F64", cfl=1.0, forcing=None,
                 device="cuda:0"):
        import torch
        self.nx, self.ny, self.tau = int(nx), int(ny), float(tau)
        self.stencil, self.storage, self.cfl, self.forcing = stencil, storage, float(cfl), forcing
        self.device = torch.device(device)
        self.Q = len(stencil_info(stencil)[1])
        nbytes = workspace_bytes(nx, ny, stencil, storage, forcing, cfl)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._ctx = ctypes.c_void_p()
        lat = _lattice(nx, ny, cfl)
        f = ctypes.byref(forcing._c()) if forcing is not None else None
        _check(lib().rlbm_init(ctypes.byref(self._ctx), ctypes.byref(lat), self.tau,
                               STENCILS[stencil], f, STORAGES[storage],
                               ctypes.c_void_p(self._ws_ptr), nbytes, _stream(self.device)))

    # -- state ---------------------------------------------------------------
    def set_state(self, e, ux, uy):
        shape = (self.ny, self.nx)
        _check(lib().rlbm_set_state(self._ctx, _ptr(_f64(e, shape)), _ptr(_f64(ux, shape)),
                                    _ptr(_f64(uy, shape))))

    def set_populations(self, F):
        _check(lib().rlbm_set_populations(self._ctx, _ptr(_f64(F, (self.Q, self.ny, self.nx)))))

    def populations(self):
        import torch
        out = torch.empty((self.Q, self.ny, self.nx), dtype=torch.float64, device=self.device)
        _check(lib().rlbm_get_populations(self._ctx, _ptr(out)))
        return out

    def step(self, n=1):
        _check(lib().rlbm_step(self._ctx, int(n)))

    def check(self):
        return lib().rlbm_check(self._ctx)

    @property
    def steps(self):
        s = ctypes.c_int64()
        _check(lib().rlbm_step_count(self._ctx, ctypes.byref(s)))
        return s.value

    # -- diagnostics -----------------------------------------------------------
    def fields(self):
        import torch
        mk = lambda *s: torch.empty(s, dtype=torch.float64, device=self.device)  # noqa: E731
        e, ux, uy = mk(self.ny, self.nx), mk(self.ny, self.nx), mk(self.ny, self.nx)
        T = mk(6, self.ny, self.nx)
        _check(lib().rlbm_fields(self._ctx, _ptr(e), _ptr(ux), _ptr(uy), _ptr(T)))
        return e, ux, uy, T

    def conserved(self):
        out = np.zeros(3)
        _check(lib().rlbm_conserved(self._ctx, out.ctypes.data_as(_P)))
        return out

    def spectrum(self, nbins):
        import torch
        n = ctypes.c_size_t()
        _check(lib().rlbm_spectrum_scratch_bytes(self._ctx, ctypes.byref(n)))
        scratch = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        p = (scratch.data_ptr() + 255) // 256 * 256
        Ek = np.zeros(nbins)
        Z = ctypes.c_double()
        _check(lib().rlbm_spectrum(self._ctx, ctypes.c_void_p(p), n.value, Ek.ctypes.data_as(_P),
                                   nbins, ctypes.byref(Z)))
        return Ek, Z.value

    def spectrum_static(self, nbins):
        """spectrum() through the allocation-free entry point (the library's
        static device scratch; lattices up to 2^20 sites)."""
        Ek = np.zeros(nbins)
        Z = ctypes.c_double()
        _check(lib().rlbm_spectrum_static(self._ctx, Ek.ctypes.data_as(_P), nbins, ctypes.byref(Z)))
        return Ek, Z.value

    def filtered_velocity(self, k_lo, k_hi):
        """beta with the Fourier band k_lo <= |k| <= k_hi removed: (ux, uy, mean speed)."""
        import torch
        n = ctypes.c_size_t()
        _check(lib().rlbm_spectrum_scratch_bytes(self._ctx, ctypes.byref(n)))
        scratch = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        p = (scratch.data_ptr() + 255) // 256 * 256
        ux = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        uy = torch.empty_like(ux)
        speed = ctypes.c_double()
        _check(lib().rlbm_filtered_velocity(self._ctx, ctypes.c_void_p(p), n.value, float(k_lo),
                                            float(k_hi), _ptr(ux), _ptr(uy), ctypes.byref(speed)))
        return ux, uy, speed.value

    # -- checkpoints and launch shape ---------------------------------------------
    def save(self):
        n = ctypes.c_size_t()
        _check(lib().rlbm_state_bytes(self._ctx, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().rlbm_save(self._ctx, buf, n.value))
        return buf.raw

    def load(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().rlbm_load(self._ctx, buf, len(blob)))

    def set_tile(self, th):
        _check(lib().rlbm_set_tile(self._ctx, int(th)))

    def set_kernel(self, kind, param=0):
        """kind "tile" (param = tile height 1/2/4/8), "staged" (param 4),
        "march", "march_pairs" (16-bit storage) or "march2" (param = rows per
        strip segment; 0 = about one segment per resident wavefront for the
        one-step forms, 12 rows for "march2")."""
        _check(lib().rlbm_set_kernel(self._ctx, KERNELS[kind], int(param)))

    def kernel(self):
        k, p = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().rlbm_get_kernel(self._ctx, ctypes.byref(k), ctypes.byref(p)))
        return _KERNEL_NAMES[k.value], p.value

    def autotune(self, steps=20):
        """Time every kernel form for `steps` steps (advancing the state) and
        keep the fastest; returns the form as kernel() does."""
        th = ctypes.c_int32()
        _check(lib().rlbm_autotune(self._ctx, int(steps), ctypes.byref(th)))
        return self.kernel()

    def set_graph_chunk(self, chunk):
        _check(lib().rlbm_set_graph_chunk(self._ctx, int(chunk)))

    def set_relaxation(self, mode):
        """mode "constant" (tau everywhere) or "eta_s" (tau(eps) = tau eps^-1/4)."""
        _check(lib().rlbm_set_relaxation(self._ctx, RELAXATION[mode]))

    def profile_step_kernel(self, n):
        """n launches of the current kernel form (2 n steps for "march2");
        mean duration (ms) of one launch, from HIP events recorded around each
        launch on the library's stream."""
        ms = ctypes.c_double()
        _check(lib().rlbm_profile_step_kernel(self._ctx, int(n), ctypes.byref(ms)))
        return ms.value

    def close(self):
        if self._ctx:
            lib().rlbm_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Independent lattices advanced together by one persistent kernel per step."""

    def __init__(self, sizes, taus, stencil="SPH26", storage="F32", cfl=1.0, forcings=None,
                 device="cuda:0"):
        import torch
        self.sizes = [(int(nx), int(ny)) for nx, ny in sizes]
        self.n = len(self.sizes)
        self.device = torch.device(device)
        self.Q = len(stencil_info(stencil)[1])
        cfls = list(cfl) if isinstance(cfl, (list, tuple)) else [cfl] * self.n
        lats = (_Lattice * self.n)(*[_lattice(nx, ny, c) for (nx, ny), c in zip(self.sizes, cfls)])
        t = (ctypes.c_double * self.n)(*[float(x) for x in taus])
        fr = None
        if forcings is not None:
            fr = (_Forcing * self.n)(*[f._c() for f in forcings])
        nbytes = ctypes.c_size_t()
        _check(lib().rlbm_batch_workspace_bytes(self.n, lats, STENCILS[stencil], STORAGES[storage],
                                                fr, ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        p = (self.workspace.data_ptr() + 255) // 256 * 256
        self._b = ctypes.c_void_p()
        _check(lib().rlbm_batch_init(ctypes.byref(self._b), self.n, lats, t, STENCILS[stencil], fr,
                                     STORAGES[storage], ctypes.c_void_p(p), nbytes.value,
                                     _stream(self.device)))

    def set_state(self, r, e, ux, uy):
        nx, ny = self.sizes[r]
        _check(lib().rlbm_batch_set_state(self._b, r, _ptr(_f64(e, (ny, nx))),
                                          _ptr(_f64(ux, (ny, nx))), _ptr(_f64(uy, (ny, nx)))))

    def step(self, n=1):
        _check(lib().rlbm_batch_step(self._b, int(n)))

    def check(self):
        return lib().rlbm_batch_check(self._b)

    def fields(self, r):
        import torch
        nx, ny = self.sizes[r]
        mk = lambda *s: torch.empty(s, dtype=torch.float64, device=self.device)  # noqa: E731
        e, ux, uy, T = mk(ny, nx), mk(ny, nx), mk(ny, nx), mk(6, ny, nx)
        _check(lib().rlbm_batch_fields(self._b, r, _ptr(e), _ptr(ux), _ptr(uy), _ptr(T)))
        return e, ux, uy, T

    def populations(self, r):
        import torch
        nx, ny = self.sizes[r]
        out = torch.empty((self.Q, ny, nx), dtype=torch.float64, device=self.device)
        _check(lib().rlbm_batch_get_populations(self._b, r, _ptr(out)))
        return out

    def set_graph_chunk(self, chunk):
        _check(lib().rlbm_batch_set_graph_chunk(self._b, int(chunk)))

    def set_relaxation(self, mode):
        _check(lib().rlbm_batch_set_relaxation(self._b, RELAXATION[mode]))

    def set_kernel(self, kind, param=0):
        _check(lib().rlbm_batch_set_kernel(self._b, KERNELS[kind], int(param)))

    def kernel(self):
        k, p = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().rlbm_batch_get_kernel(self._b, ctypes.byref(k), ctypes.byref(p)))
        return _KERNEL_NAMES[k.value], p.value

    @property
    def steps(self):
        s = ctypes.c_int64()
        _check(lib().rlbm_batch_step_count(self._b, ctypes.byref(s)))
        return s.value

    def autotune(self, steps=20):
        """Time every kernel form for `steps` steps (advancing the state) and
        keep the fastest; returns the form as kernel() does."""
        th = ctypes.c_int32()
        _check(lib().rlbm_batch_autotune(self._b, int(steps), ctypes.byref(th)))
        return self.kernel()

    def close(self):
        if self._b:
            lib().rlbm_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
