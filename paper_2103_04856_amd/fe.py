"""Python binding of the C ABI in include/fe.h (argument marshalling only).

Every step of the energy, gradient and descent runs in the HIP kernels of
libfe.so; this module only checks tensors, passes device pointers and the
current torch stream, and wraps the entry points for autograd. There is no
CPU path: the library must be built (python -m paper_2103_04856_amd.build) and
fields must live on a ROCm device.

Fields are torch tensors of shape [batch, nz, ny, nx] (or [nz, ny, nx] for a
single instance), contiguous, float32 or float64, x fastest.
"""

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfe.so")

FE_F32, FE_F64 = 0, 1
FE_OK, FE_EINVAL, FE_EHIP, FE_ENOMEM, FE_ENONFINITE = 0, -1, -2, -3, -4
_CODES = {FE_EINVAL: "FE_EINVAL", FE_EHIP: "FE_EHIP", FE_ENOMEM: "FE_ENOMEM", FE_ENONFINITE: "FE_ENONFINITE"}


class FeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class FeGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("batch", ctypes.c_int), ("h", ctypes.c_double), ("dtype", ctypes.c_int)]


_lib = None
_P = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)

# name -> (restype, argtypes); the full set of entry points of include/fe.h
SIGNATURES = {
    "fe_create": (ctypes.c_int, [ctypes.POINTER(FeGrid), _DP, _DP, _P, ctypes.POINTER(_P)]),
    "fe_set_params": (ctypes.c_int, [_P, _DP, _DP]),
    "fe_set_stream": (ctypes.c_int, [_P, _P]),
    "fe_energy": (ctypes.c_int, [_P, _P, _DP]),
    "fe_energy_grad": (ctypes.c_int, [_P, _P, _P, _DP]),
    "fe_energy_grad_async": (ctypes.c_int, [_P, _P, _P, _P]),
    "fe_grad_scaled_async": (ctypes.c_int, [_P, _P, _P, _P]),
    "fe_step": (ctypes.c_int, [_P, _P, _DP, ctypes.c_double, ctypes.c_int, _DP]),
    "fe_step_adam": (ctypes.c_int, [_P, _P, _DP, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, _DP]),
    "fe_adam_reset": (ctypes.c_int, [_P]),
    "fe_hminus_step": (ctypes.c_int, [_P, _P, _DP, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, _DP]),
    "fe_hminus_reset": (ctypes.c_int, [_P]),
    "fe_diagnostics": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, ctypes.c_double, _DP]),
    "fe_set_orientation": (ctypes.c_int, [_P, _DP, _DP]),
    "fe_set_coeff_field": (ctypes.c_int, [_P, _P]),
    "fe_set_mass_field": (ctypes.c_int, [_P, _P]),
    "fe_l2_create": (ctypes.c_int, [ctypes.POINTER(FeGrid), ctypes.c_double, _DP, ctypes.c_double, _P,
                                    ctypes.POINTER(_P)]),
    "fe_l2_set_lbfgs": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double]),
    "fe_l2_load": (ctypes.c_int, [_P, _P]),
    "fe_l2_store": (ctypes.c_int, [_P, _P]),
    "fe_l2_energy_grad": (ctypes.c_int, [_P, _P, _P, _DP]),
    "fe_l2_step": (ctypes.c_int, [_P, ctypes.c_int, _DP]),
    "fe_l2_set_stream": (ctypes.c_int, [_P, _P]),
    "fe_l2_destroy": (None, [_P]),
    "fe_energy_grad_noalloc": (ctypes.c_int, [ctypes.POINTER(FeGrid), _DP, _DP, _P, _P, _P, _P]),
    "fe_num_variants": (ctypes.c_int, []),
    "fe_variant_info": (ctypes.c_int, [ctypes.c_int, _IP, _IP, _IP, _IP]),
    "fe_set_launch": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
    "fe_get_launch": (ctypes.c_int, [_P, _IP, _IP]),
    "fe_autotune": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, _DP, _IP]),
    "fe_tune_cache_save": (ctypes.c_int, [ctypes.c_char_p]),
    "fe_tune_cache_load": (ctypes.c_int, [ctypes.c_char_p]),
    "fe_tune_cache_clear": (None, []),
    "fe_destroy": (None, [_P]),
    "fe_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libfe.so (once). Raises if the library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_04856_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != FE_OK:
        raise FeError(rc, lib().fe_last_error().decode())


def _dbl(values):
    arr = (ctypes.c_double * len(values))(*[float(v) for v in values])
    return arr


def variants():
    """[(tile_x, tile_y, threads, dtype_mask)] of every launch variant."""
    L = lib()
    out = []
    for v in range(L.fe_num_variants()):
        a, b, c, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(L.fe_variant_info(v, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        out.append((a.value, b.value, c.value, d.value))
    return out


def _torch_dtype(fe_dtype):
    return torch.float32 if fe_dtype == FE_F32 else torch.float64


class FeContext:
    """One set of B independent problems on an nz x ny x nx periodic grid.

    eps: float or [B]; coeffs: (a20, a11, a02, a10, a01, a00) or [B][6]
    (the coefficient order of Sec. 3.2). dtype: torch.float32 or torch.float64.
    """

    def __init__(self, shape, h, eps, coeffs, dtype=torch.float32, device=None):
        if len(shape) == 3:
            shape = (1, *shape)
        B, nz, ny, nx = (int(s) for s in shape)
        self.shape = (B, nz, ny, nx)
        self.h = float(h)
        self.dtype = dtype
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("dtype must be torch.float32 or torch.float64")
        self.device = (torch.device("cuda", torch.cuda.current_device()) if device is None
                       else torch.device(device))
        eps_l, coeff_l = self._param_lists(eps, coeffs, B)
        grid = FeGrid(nx, ny, nz, B, self.h, FE_F32 if dtype == torch.float32 else FE_F64)
        handle = _P()
        with torch.cuda.device(self.device):
            _check(lib().fe_create(ctypes.byref(grid), _dbl(eps_l), _dbl(coeff_l),
                                   _P(torch.cuda.current_stream().cuda_stream), ctypes.byref(handle)))
        self._h = handle
        self.eps, self.coeffs = eps_l, [coeff_l[6 * b:6 * b + 6] for b in range(B)]

    @staticmethod
    def _param_lists(eps, coeffs, B):
        if isinstance(eps, (int, float)):
            eps = [float(eps)] * B
        eps = [float(e) for e in eps]
        flat = [float(c) for c in np.asarray(coeffs, dtype=np.float64).reshape(-1)]
        if len(flat) == 6:
            flat = flat * B
        if len(eps) != B or len(flat) != 6 * B:
            raise ValueError(f"need {B} eps values and {B} x 6 coefficients")
        return eps, flat

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().fe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -------------------------------------------------------------
    def _field(self, t, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be a device tensor (there is no CPU path)")
        if t.dtype != self.dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, context expects {self.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        shp = tuple(t.shape)
        if shp != self.shape and not (self.shape[0] == 1 and shp == self.shape[1:]):
            raise ValueError(f"{name} has shape {shp}, context expects {self.shape}")
        return _P(t.data_ptr())

    def _sync_stream(self):
        _check(lib().fe_set_stream(self._h, _P(torch.cuda.current_stream(self.device).cuda_stream)))

    # -- API -------------------------------------------------------------------
    def set_params(self, eps, coeffs):
        eps_l, coeff_l = self._param_lists(eps, coeffs, self.shape[0])
        self._sync_stream()
        _check(lib().fe_set_params(self._h, _dbl(eps_l), _dbl(coeff_l)))
        self.eps, self.coeffs = eps_l, [coeff_l[6 * b:6 * b + 6] for b in range(self.shape[0])]

    def set_coeff_field(self, a_field):
        """Space-dependent coefficients a(x) [B, 6, nz, ny, nx] (Sec. 5.2), or None for the
        per-instance ones. The library keeps a scaled copy."""
        if a_field is None:
            _check(lib().fe_set_coeff_field(self._h, _P(0)))
            return
        exp = (self.shape[0], 6) + self.shape[1:]
        if not isinstance(a_field, torch.Tensor) or a_field.device.type != "cuda" or a_field.dtype != self.dtype \
                or tuple(a_field.shape) != exp or not a_field.is_contiguous():
            raise ValueError(f"a_field must be a contiguous {self.dtype} device tensor of shape {exp}")
        self._sync_stream()
        _check(lib().fe_set_coeff_field(self._h, _P(a_field.data_ptr())))

    def set_mass_field(self, m_field):
        """Space-dependent mass m(x) [B, nz, ny, nx] for hminus_step (Sec. 5.2), or None."""
        if m_field is None:
            _check(lib().fe_set_mass_field(self._h, _P(0)))
            return
        self._sync_stream()
        _check(lib().fe_set_mass_field(self._h, self._field(m_field, "m_field")))

    def set_orientation(self, mu, theta):
        """Orientation term eps mu (theta . grad u)^2 of Sec. 5.2, per instance (mu = 0: off)."""
        B = self.shape[0]
        mu_l = [float(mu)] * B if isinstance(mu, (int, float)) else [float(v) for v in mu]
        th = np.asarray(theta, dtype=np.float64).reshape(-1, 3)
        if th.shape[0] == 1:
            th = np.repeat(th, B, axis=0)
        if len(mu_l) != B or th.shape[0] != B:
            raise ValueError(f"need {B} mu values and {B} theta vectors")
        self._sync_stream()
        _check(lib().fe_set_orientation(self._h, _dbl(mu_l), _dbl(th.reshape(-1).tolist())))

    def energy(self, u):
        """F_h(u_b) for every instance, as a float64 CPU tensor [B] (synchronises)."""
        out = (ctypes.c_double * self.shape[0])()
        self._sync_stream()
        _check(lib().fe_energy(self._h, self._field(u, "u"), out))
        return torch.tensor(list(out), dtype=torch.float64)

    def energy_grad(self, u, g=None):
        """(F_h [B] float64 on CPU, g = dF_h/du); synchronises."""
        g = torch.empty_like(u) if g is None else g
        out = (ctypes.c_double * self.shape[0])()
        self._sync_stream()
        _check(lib().fe_energy_grad(self._h, self._field(u, "u"), self._field(g, "g"), out))
        return torch.tensor(list(out), dtype=torch.float64), g

    def energy_grad_async(self, u, g=None, energy_out=None, with_grad=True):
        """Stream-ordered, no sync: (energies as a float64 device tensor [B], g or None)."""
        if with_grad and g is None:
            g = torch.empty_like(u)
        if energy_out is None:
            energy_out = torch.empty(self.shape[0], dtype=torch.float64, device=u.device)
        self._sync_stream()
        _check(lib().fe_energy_grad_async(self._h, self._field(u, "u"),
                                          self._field(g, "g") if with_grad else _P(0),
                                          _P(energy_out.data_ptr())))
        return energy_out, g

    def grad_scaled_async(self, u, scale, g=None):
        """Stream-ordered, no sync: g_b = scale_b dF_h/du_b, scale a float64 device tensor [B]."""
        if g is None:
            g = torch.empty_like(u)
        if not isinstance(scale, torch.Tensor) or scale.device.type != "cuda" or scale.dtype != torch.float64 \
                or scale.numel() != self.shape[0] or not scale.is_contiguous():
            raise ValueError(f"scale must be a contiguous float64 device tensor of {self.shape[0]} values")
        self._sync_stream()
        _check(lib().fe_grad_scaled_async(self._h, self._field(u, "u"), self._field(g, "g"), _P(scale.data_ptr())))
        return g

    def step(self, u, mass, tau, nsteps):
        """nsteps mass-projected descent steps in place on u; returns F_h before the last step."""
        B = self.shape[0]
        if isinstance(mass, (int, float)):
            mass = [float(mass)] * B
        if len(mass) != B:
            raise ValueError(f"need {B} mass values")
        out = (ctypes.c_double * B)()
        self._sync_stream()
        _check(lib().fe_step(self._h, self._field(u, "u"), _dbl(mass), float(tau), int(nsteps), out))
        return torch.tensor(list(out), dtype=torch.float64)

    def step_adam(self, u, mass, nsteps, lr=1e-3, betas=(0.9, 0.999), adam_eps=1e-8):
        """nsteps mass-projected Adam steps in place on u (moments kept in the context);
        returns F_h before the last step."""
        B = self.shape[0]
        if isinstance(mass, (int, float)):
            mass = [float(mass)] * B
        if len(mass) != B:
            raise ValueError(f"need {B} mass values")
        out = (ctypes.c_double * B)()
        self._sync_stream()
        _check(lib().fe_step_adam(self._h, self._field(u, "u"), _dbl(mass), float(lr), float(betas[0]),
                                  float(betas[1]), float(adam_eps), int(nsteps), out))
        return torch.tensor(list(out), dtype=torch.float64)

    def adam_reset(self):
        self._sync_stream()
        _check(lib().fe_adam_reset(self._h))

    def hminus_step(self, A, m0, nsteps, sigma_k=2.0, lr=1e-3, betas=(0.9, 0.999), adam_eps=1e-8, u_out=None):
        """nsteps iterations of Algorithm 1 on the vector field A [B, 3, nz, ny, nx] (in place);
        u_out, if given, receives k * (div A + m0). Returns G before the last update."""
        B = self.shape[0]
        if isinstance(m0, (int, float)):
            m0 = [float(m0)] * B
        if m0 is not None and len(m0) != B:
            raise ValueError(f"need {B} m0 values")
        exp = (B, 3) + self.shape[1:]
        if not isinstance(A, torch.Tensor) or A.device.type != "cuda" or A.dtype != self.dtype \
                or not A.is_contiguous() or tuple(A.shape) not in (exp, exp[1:] if B == 1 else exp):
            raise ValueError(f"A must be a contiguous {self.dtype} device tensor of shape {exp}")
        out = (ctypes.c_double * B)()
        self._sync_stream()
        _check(lib().fe_hminus_step(self._h, _P(A.data_ptr()), _dbl(m0) if m0 is not None else None,
                                    float(sigma_k), float(lr),
                                    float(betas[0]), float(betas[1]), float(adam_eps), int(nsteps),
                                    self._field(u_out, "u_out") if u_out is not None else _P(0), out))
        return torch.tensor(list(out), dtype=torch.float64)

    def hminus_reset(self):
        self._sync_stream()
        _check(lib().fe_hminus_reset(self._h))

    def diagnostics(self, u, curvatures=False, nbins=0, kmax=100.0):
        """Diffuse curvatures, the curvature histogram and the viability summary of u.
        Returns (stats [B, 5] float64: F_h, A_eps, discrepancy, min u, max u;
        curvatures [B, 4, nz, ny, nx] (H, K, kappa1, kappa2) or None;
        histogram [B, nbins, nbins] float64 on the device, or None)."""
        B = self.shape[0]
        up = self._field(u, "u")
        curv = None
        if curvatures:
            curv = torch.empty((B, 4) + self.shape[1:], dtype=self.dtype, device=u.device)
        hist = torch.empty((B, nbins, nbins), dtype=torch.float64, device=u.device) if nbins else None
        out = (ctypes.c_double * (5 * B))()
        self._sync_stream()
        _check(lib().fe_diagnostics(self._h, up, _P(curv.data_ptr()) if curv is not None else _P(0),
                                    _P(hist.data_ptr()) if hist is not None else _P(0), int(nbins),
                                    float(kmax), out))
        stats = torch.tensor(list(out), dtype=torch.float64).reshape(B, 5)
        return stats, curv, hist

    def diagnostics_async(self, u, curv=None, hist=None, kmax=100.0):
        """Stream-ordered diagnostics into preallocated outputs (curv [B, 4, nz, ny, nx] in
        the context dtype, hist [B, nbins, nbins] float64); no summary, no synchronisation."""
        up = self._field(u, "u")
        nb = 0
        if hist is not None:
            if hist.dtype != torch.float64 or hist.dim() != 3 or hist.shape[1] != hist.shape[2] \
                    or hist.shape[0] != self.shape[0] or not hist.is_contiguous():
                raise ValueError("hist must be a contiguous float64 tensor [B, nbins, nbins]")
            nb = hist.shape[1]
        if curv is not None and (curv.dtype != self.dtype or tuple(curv.shape) != (self.shape[0], 4) + self.shape[1:]
                                 or not curv.is_contiguous()):
            raise ValueError("curv must be a contiguous tensor [B, 4, nz, ny, nx] of the context dtype")
        self._sync_stream()
        _check(lib().fe_diagnostics(self._h, up, _P(curv.data_ptr()) if curv is not None else _P(0),
                                    _P(hist.data_ptr()) if hist is not None else _P(0), nb, float(kmax), None))

    def set_launch(self, variant, z_chunk=0):
        _check(lib().fe_set_launch(self._h, int(variant), int(z_chunk)))

    def get_launch(self):
        v, z = ctypes.c_int(), ctypes.c_int()
        _check(lib().fe_get_launch(self._h, ctypes.byref(v), ctypes.byref(z)))
        return v.value, z.value

    TUNE_KINDS = {"grad": 0, "step": 1, "adam": 2}

    def autotune(self, u, work=None, kind="grad", iters=10):
        """Pick the launch shape for the sweep of `kind` ("grad": fe_energy_grad, "step":
        fe_step, "adam": fe_step_adam) and keep it; returns (variant, z_chunk, us, cached).
        u is not modified; work (u's shape, overwritten) is allocated here if not given."""
        work = torch.empty_like(u) if work is None else work
        best = ctypes.c_double()
        cached = ctypes.c_int()
        self._sync_stream()
        _check(lib().fe_autotune(self._h, self._field(u, "u"), self._field(work, "work"), self.TUNE_KINDS[kind],
                                 int(iters), ctypes.byref(best), ctypes.byref(cached)))
        v, z = self.get_launch()
        return v, z, best.value, bool(cached.value)


def tune_cache_save(path):
    """Save the autotuner's choices of this process to a text file."""
    _check(lib().fe_tune_cache_save(os.fsencode(path)))


def tune_cache_load(path):
    """Merge a saved file of autotuner choices into this process's cache."""
    _check(lib().fe_tune_cache_load(os.fsencode(path)))


def tune_cache_clear():
    lib().fe_tune_cache_clear()


NOALLOC_MAX_BATCH = 16


def energy_grad_noalloc(u, h, eps, coeffs, g=None, energy_out=None, with_grad=True):
    """fe_energy_grad_noalloc: energy (and gradient) of u [B, nz, ny, nx] without a context
    and without any device allocation by the library (its workspace is a static device
    array; calls that overlap on one device race). g and energy_out, if given, receive the
    results (else torch allocates them here). Stream-ordered on the current torch stream,
    no synchronisation. Returns (energies float64 [B] on the device, g or None)."""
    if not isinstance(u, torch.Tensor) or u.device.type != "cuda" or not u.is_contiguous() \
            or u.dtype not in (torch.float32, torch.float64):
        raise ValueError("u must be a contiguous float32/float64 device tensor")
    shape = tuple(u.shape) if u.dim() == 4 else (1, *u.shape)
    B, nz, ny, nx = shape
    eps_l, coeff_l = FeContext._param_lists(eps, coeffs, B)
    if with_grad and g is None:
        g = torch.empty_like(u)
    if g is not None and (g.shape != u.shape or g.dtype != u.dtype or not g.is_contiguous()
                          or g.device != u.device):
        raise ValueError("g must match u")
    if energy_out is None:
        energy_out = torch.empty(B, dtype=torch.float64, device=u.device)
    grid = FeGrid(nx, ny, nz, B, float(h), FE_F32 if u.dtype == torch.float32 else FE_F64)
    with torch.cuda.device(u.device):
        _check(lib().fe_energy_grad_noalloc(ctypes.byref(grid), _dbl(eps_l), _dbl(coeff_l), _P(u.data_ptr()),
                                            _P(g.data_ptr()) if g is not None else _P(0),
                                            _P(energy_out.data_ptr()),
                                            _P(torch.cuda.current_stream(u.device).cuda_stream)))
    return energy_out, g


class FeL2Flow:
    """Algorithm 2 (Sec. 4.2) on one box field [nz, ny, nx]: the L2 flow of F_h(k * u)
    with replicate boundaries, driven by L-BFGS (lr 1, history 10, 20 iterations per
    step unless set otherwise). Everything runs in libfe."""

    def __init__(self, shape, h, eps, coeffs, sigma_k=1.0, dtype=torch.float32, device=None):
        nz, ny, nx = (int(v) for v in shape)
        self.shape = (nz, ny, nx)
        self.dtype = dtype
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("dtype must be torch.float32 or torch.float64")
        self.device = (torch.device("cuda", torch.cuda.current_device()) if device is None
                       else torch.device(device))
        coeffs = [float(c) for c in np.asarray(coeffs, dtype=np.float64).reshape(-1)]
        if len(coeffs) != 6:
            raise ValueError("need 6 coefficients")
        grid = FeGrid(nx, ny, nz, 1, float(h), FE_F32 if dtype == torch.float32 else FE_F64)
        handle = _P()
        with torch.cuda.device(self.device):
            _check(lib().fe_l2_create(ctypes.byref(grid), float(eps), _dbl(coeffs), float(sigma_k),
                                      _P(torch.cuda.current_stream().cuda_stream), ctypes.byref(handle)))
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            lib().fe_l2_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _check(lib().fe_l2_set_stream(self._h, _P(torch.cuda.current_stream(self.device).cuda_stream)))

    def _box(self, t, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != self.dtype \
                or not t.is_contiguous() or tuple(t.shape[-3:]) != self.shape or t.numel() != np.prod(self.shape):
            raise ValueError(f"{name} must be a contiguous {self.dtype} device tensor of shape {self.shape}")
        return _P(t.data_ptr())

    def set_lbfgs(self, lr=1.0, history=10, max_iter=20, tolerance_grad=1e-7, tolerance_change=1e-9):
        _check(lib().fe_l2_set_lbfgs(self._h, float(lr), int(history), int(max_iter), float(tolerance_grad),
                                     float(tolerance_change)))

    def load(self, u):
        self._sync_stream()
        _check(lib().fe_l2_load(self._h, self._box(u, "u")))

    def store(self, u=None):
        if u is None:
            u = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        self._sync_stream()
        _check(lib().fe_l2_store(self._h, self._box(u, "u")))
        return u

    def energy_grad(self, u):
        """Loads u (resets the optimiser) and returns (F_h(k * u), dF/du)."""
        g = torch.empty(self.shape, dtype=self.dtype, device=u.device)
        E = ctypes.c_double()
        self._sync_stream()
        _check(lib().fe_l2_energy_grad(self._h, self._box(u, "u"), _P(g.data_ptr()), ctypes.byref(E)))
        return E.value, g

    def step(self, nsteps=1):
        """nsteps optimiser steps; returns the loss at the start of each."""
        out = (ctypes.c_double * max(nsteps, 1))()
        self._sync_stream()
        _check(lib().fe_l2_step(self._h, int(nsteps), out))
        return [out[i] for i in range(nsteps)]


class FeEnergy(torch.autograd.Function):
    """E = F_h(u) per instance (float64 [B]); backward recomputes the Hessian and
    applies the hand-written adjoint kernel with the incoming dL/dE_b folded into
    instance b's coefficients: dL/du_b = dL/dE_b dF_h/du_b, in one sweep."""

    @staticmethod
    def forward(ctx, u, fe):
        E, _ = fe.energy_grad_async(u, with_grad=False)
        ctx.fe = fe
        ctx.save_for_backward(u)
        return E

    @staticmethod
    def backward(ctx, gE):
        (u,) = ctx.saved_tensors
        scale = gE.to(torch.float64).reshape(-1).contiguous()
        return ctx.fe.grad_scaled_async(u.contiguous(), scale), None


def feps(u, fe):
    """Differentiable F_h(u) through the HIP kernels (see FeEnergy)."""
    return FeEnergy.apply(u, fe)
