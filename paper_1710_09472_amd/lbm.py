"""ctypes binding of the HIP library ``liblbm_hip.so`` (C ABI in ``include/lbm.h``).

This module only marshals arguments: every step of the lattice Boltzmann update runs in
the library's kernels. PyTorch provides device memory and the HIP stream. If the
library has not been built, loading fails with an error; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "liblbm_hip.so"

LATTICES = {"D2V9": 0, "D3V19": 1, "D3V15": 2, "D1V7": 3}
STATS = {"fd": 0, "be": 1, "hermite": 2}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
FORCING = {"source": 0, "shift": 1}
ROUNDING = {"nearest": 0, "stochastic": 1}
SLIP_Y, SLIP_Z = 1, 2

LBM_OK, LBM_EINVAL, LBM_EUNSUPPORTED, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5

#: Every function the header declares (checked by the tests).
EXPORTS = [
    "lbm_compute_constants", "lbm_lattice_info", "lbm_workspace_bytes", "lbm_buffer_sizes", "lbm_create",
    "lbm_init",
    "lbm_step", "lbm_step_from", "lbm_moments", "lbm_current", "lbm_get_state", "lbm_set_state",
    "lbm_export_f64", "lbm_set_fields", "lbm_set_tau", "lbm_adjoint_seed", "lbm_adjoint_step",
    "lbm_density_from_mu", "lbm_mu_from_density", "lbm_init_thermal", "lbm_thetabar", "lbm_energy",
    "lbm_speed_change", "lbm_destroy", "lbm_last_error", "lbm_status_string", "lbm_current_noalloc",
    "lbm_set_step_index",
]


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int), ("stats", ctypes.c_int), ("storage", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("theta", ctypes.c_double), ("mu", ctypes.c_double), ("tau", ctypes.c_double),
        ("E", ctypes.c_double * 3), ("B", ctypes.c_double * 3), ("rho0", ctypes.c_double),
        ("dev_scale_log2", ctypes.c_int), ("forcing", ctypes.c_int), ("slip", ctypes.c_int),
        ("order", ctypes.c_int), ("rounding", ctypes.c_int),
    ]


class LbmConstants(ctypes.Structure):
    _fields_ = [
        ("I0", ctypes.c_double), ("I2", ctypes.c_double), ("I4", ctypes.c_double),
        ("c0", ctypes.c_double), ("c1", ctypes.c_double), ("c2", ctypes.c_double),
        ("c2bar", ctypes.c_double), ("c2p", ctypes.c_double),
        ("J2", ctypes.c_double), ("Delta2", ctypes.c_double), ("theta_bar", ctypes.c_double),
        ("cs", ctypes.c_double), ("w", ctypes.c_double * 4), ("what", ctypes.c_double * 4),
        ("A", ctypes.c_double), ("Bc", ctypes.c_double), ("C", ctypes.c_double * 4),
    ]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} [status {code}]")
        self.code = code


_lib = None


def load_library() -> ctypes.CDLL:
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1710_09472_amd.build`")
        lib = ctypes.CDLL(str(LIB_PATH))
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        sz = ctypes.POINTER(ctypes.c_size_t)
        P = ctypes.POINTER(LbmParams)
        lib.lbm_compute_constants.argtypes = [P, ctypes.POINTER(LbmConstants)]
        lib.lbm_lattice_info.argtypes = [i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
        lib.lbm_workspace_bytes.argtypes = [P, sz, sz]
        lib.lbm_buffer_sizes.argtypes = [P, sz, sz, sz, sz]
        lib.lbm_create.argtypes = [P, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
        lib.lbm_init.argtypes = [vp, vp, vp]
        lib.lbm_init_thermal.argtypes = [vp, vp, vp, vp]
        lib.lbm_thetabar.argtypes = [vp, vp]
        lib.lbm_energy.argtypes = [vp, ctypes.POINTER(d)]
        lib.lbm_speed_change.argtypes = [vp, vp, vp, i, ctypes.POINTER(d)]
        lib.lbm_step.argtypes = [vp, i]
        lib.lbm_step_from.argtypes = [vp, vp, vp]
        lib.lbm_set_step_index.argtypes = [vp, ctypes.c_ulonglong]
        lib.lbm_moments.argtypes = [vp, vp, vp]
        lib.lbm_current.argtypes = [vp, ctypes.POINTER(d)]
        lib.lbm_current_noalloc.argtypes = [vp, vp]
        lib.lbm_get_state.argtypes = [vp, vp]
        lib.lbm_set_state.argtypes = [vp, vp]
        lib.lbm_export_f64.argtypes = [vp, vp, vp]
        lib.lbm_set_fields.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(d)]
        lib.lbm_set_tau.argtypes = [vp, d]
        lib.lbm_adjoint_seed.argtypes = [vp, i, d, vp]
        lib.lbm_adjoint_step.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.lbm_density_from_mu.argtypes = [vp, vp, vp, ctypes.c_size_t, vp]
        lib.lbm_mu_from_density.argtypes = [vp, vp, vp, ctypes.c_size_t, vp]
        lib.lbm_destroy.argtypes = [vp]
        lib.lbm_destroy.restype = None
        lib.lbm_last_error.argtypes = [vp]
        lib.lbm_last_error.restype = ctypes.c_char_p
        lib.lbm_status_string.argtypes = [i]
        lib.lbm_status_string.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("lbm_destroy", "lbm_last_error", "lbm_status_string"):
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(rc, handle=None):
    if rc != LBM_OK:
        lib = load_library()
        msg = lib.lbm_last_error(handle).decode()
        raise LbmError(rc, msg or lib.lbm_status_string(rc).decode())


def make_params(lattice="D2V9", nx=1, ny=1, nz=1, tau=0.8, E=(0.0, 0.0, 0.0), B=(0.0, 0.0, 0.0),
                storage="f32", dev_scale_log2=0, rho0=1.0, stats="fd", theta=1.0 / 270.0, mu=1.0,
                forcing="source", slip=0, order=0, rounding="nearest") -> LbmParams:
    """forcing: "source" (xi-dependent source term) or "shift" (velocity shift);
    slip: free-slip wall planes, SLIP_Y | SLIP_Z; order: D1V7 equilibrium truncation,
    3 or 4 (0 = 4); rounding of 16-bit stored values: "nearest" or "stochastic"."""
    p = LbmParams()
    p.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
    p.stats = STATS[stats] if isinstance(stats, str) else int(stats)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.theta, p.mu, p.tau = float(theta), float(mu), float(tau)
    p.E = (ctypes.c_double * 3)(*[float(v) for v in E])
    p.B = (ctypes.c_double * 3)(*[float(v) for v in B])
    p.rho0 = float(rho0)
    p.dev_scale_log2 = int(dev_scale_log2)
    p.forcing = FORCING[forcing] if isinstance(forcing, str) else int(forcing)
    p.slip = int(slip)
    p.order = int(order)
    p.rounding = ROUNDING[rounding] if isinstance(rounding, str) else int(rounding)
    return p


def compute_constants(lattice="D2V9", stats="fd", theta=1.0 / 270.0, mu=1.0) -> dict:
    """Host-side constants of the library (no GPU needed)."""
    lib = load_library()
    out = LbmConstants()
    _check(lib.lbm_compute_constants(ctypes.byref(make_params(lattice, stats=stats, theta=theta, mu=mu)),
                                     ctypes.byref(out)))
    res = {}
    for name, typ in LbmConstants._fields_:
        v = getattr(out, name)
        res[name] = list(v) if hasattr(v, "__len__") else float(v)
    return res


def _density_convert(fn_name, x, lattice, stats, theta):
    import torch

    lib = load_library()
    x = torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    out = torch.empty_like(x)
    p = make_params(lattice, stats=stats, theta=theta)
    stream = torch.cuda.current_stream()
    _check(getattr(lib, fn_name)(ctypes.byref(p), _ptr(x), _ptr(out), ctypes.c_size_t(x.numel()),
                                 ctypes.c_void_p(stream.cuda_stream)))
    return out


def density_from_mu(mu, lattice="D2V9", stats="fd", theta=1.0 / 270.0):
    """rho = (pi theta)^(D/2) g_(D/2)(e^(mu/theta)) elementwise on the GPU (float64 tensor)."""
    return _density_convert("lbm_density_from_mu", mu, lattice, stats, theta)


def mu_from_density(rho, lattice="D2V9", stats="fd", theta=1.0 / 270.0):
    """The inverse of density_from_mu (NaN where no mu exists)."""
    return _density_convert("lbm_mu_from_density", rho, lattice, stats, theta)


def lattice_info(lattice="D2V9"):
    """(Q, D, e) with e an int array (Q, 3) in the library's velocity order."""
    lib = load_library()
    Q, D = ctypes.c_int(), ctypes.c_int()
    e = (ctypes.c_int * (27 * 3))()
    _check(lib.lbm_lattice_info(LATTICES[lattice], ctypes.byref(Q), ctypes.byref(D), e))
    return Q.value, D.value, np.array(e[: 3 * Q.value], dtype=np.int64).reshape(Q.value, 3)


def buffer_sizes(params: LbmParams) -> dict:
    lib = load_library()
    st, wk, ad, sd = (ctypes.c_size_t() for _ in range(4))
    _check(lib.lbm_buffer_sizes(ctypes.byref(params), ctypes.byref(st), ctypes.byref(wk), ctypes.byref(ad),
                                ctypes.byref(sd)))
    return {"state": st.value, "work": wk.value, "adjoint": ad.value, "stride": sd.value}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Simulation:
    """One lattice Boltzmann handle with its device buffers (torch tensors).

    Geometry arrays: ``mask`` (uint8, 1 = solid) and ``s`` (partial bounce-back
    fraction in [0, 1]) of N nodes, numpy or torch; they are copied to the device once.
    ``inplace=True`` binds one state buffer instead of two: the steps then update it in
    place (the AA access pattern), with the same results and half the state memory.
    """

    def __init__(self, lattice="D2V9", nx=1, ny=1, nz=1, tau=0.8, E=(0.0, 0.0, 0.0), B=(0.0, 0.0, 0.0),
                 storage="f32", dev_scale_log2=0, rho0=1.0, stats="fd", theta=1.0 / 270.0, mu=1.0,
                 mask=None, s=None, device="cuda", forcing="source", slip=0, work=None, inplace=False,
                 order=0, rounding="nearest"):
        import torch

        self.torch = torch
        self.lib = load_library()
        self.lattice = lattice
        self.params = make_params(lattice, nx, ny, nz, tau, E, B, storage, dev_scale_log2, rho0, stats, theta, mu,
                                  forcing, slip, order, rounding)
        self.sizes = buffer_sizes(self.params)
        self.Q, self.D, self.e = lattice_info(lattice)
        self.N = nx * ny * nz
        self.stride = self.sizes["stride"]
        self.device = torch.device(device)
        self.mask = None if mask is None else self._field(mask, torch.uint8)
        self.s = None if s is None else self._field(s, torch.float32)
        for name, arr in (("mask", self.mask), ("s", self.s)):
            if arr is not None and arr.numel() != self.N:
                raise ValueError(f"{name} must have {self.N} entries")
        self.inplace = bool(inplace)
        self.bufs = [torch.zeros(self.sizes["state"], dtype=torch.uint8, device=self.device)
                     for _ in range(1 if self.inplace else 2)]
        # workspace: the caller's (uint8 tensor of at least work bytes, any content) or zeros
        self.work = torch.zeros(self.sizes["work"], dtype=torch.uint8, device=self.device) if work is None else work
        if self.work.numel() < self.sizes["work"]:
            raise ValueError(f"work must hold {self.sizes['work']} bytes")
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        state_b = None if self.inplace else self.bufs[1]
        _check(self.lib.lbm_create(ctypes.byref(self.params), _ptr(self.mask), _ptr(self.s), _ptr(self.bufs[0]),
                                   _ptr(state_b), _ptr(self.work), ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h)))
        self.h = h
        self.constants = compute_constants(lattice, stats, theta, mu)

    def _field(self, a, dtype):
        torch = self.torch
        if isinstance(a, torch.Tensor):
            t = a.detach()
        else:
            t = torch.as_tensor(np.asarray(a))
        return t.to(device=self.device, dtype=dtype).reshape(-1).contiguous()

    # ------------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, dtype):
        t = self.torch.as_tensor(a) if not isinstance(a, self.torch.Tensor) else a
        return t.to(device=self.device, dtype=dtype).contiguous()

    # ------------------------------------------------------------------ forward
    def init(self, rho, u=None, thetabar=None):
        """f = f^eq(rho, u); rho (N,), u (D, N) or None, xi-units. The D1V7 thermal model
        also takes thetabar (N,) (None: the weight's I_2/I_0)."""
        self._rho_in = self._dev(rho, self.torch.float64).reshape(-1)
        self._u_in = None if u is None else self._dev(u, self.torch.float64).reshape(-1)
        if self._rho_in.numel() != self.N or (self._u_in is not None and self._u_in.numel() != self.D * self.N):
            raise ValueError("rho must have N entries and u D*N")
        if self.lattice == "D1V7":
            self._tb_in = None if thetabar is None else self._dev(thetabar, self.torch.float64).reshape(-1)
            if self._tb_in is not None and self._tb_in.numel() != self.N:
                raise ValueError("thetabar must have N entries")
            _check(self.lib.lbm_init_thermal(self.h, _ptr(self._rho_in), _ptr(self._u_in), _ptr(self._tb_in)),
                   self.h)
            return
        if thetabar is not None:
            raise ValueError("thetabar is a field of the D1V7 thermal model")
        _check(self.lib.lbm_init(self.h, _ptr(self._rho_in), _ptr(self._u_in)), self.h)

    def thetabar(self):
        """thetabar (N,) float32 device tensor of the current state (D1V7 thermal model)."""
        out = self.torch.empty(self.N, dtype=self.torch.float32, device=self.device)
        _check(self.lib.lbm_thetabar(self.h, _ptr(out)), self.h)
        return out

    def energy(self):
        """sum over nodes of sum_a f_a xi_a^2, FP64 (D1V7 thermal model)."""
        out = ctypes.c_double()
        _check(self.lib.lbm_energy(self.h, ctypes.byref(out)), self.h)
        return out.value

    def step(self, n=1):
        _check(self.lib.lbm_step(self.h, int(n)), self.h)

    def step_from(self, src, dst):
        _check(self.lib.lbm_step_from(self.h, _ptr(src), _ptr(dst)), self.h)

    def set_step_index(self, t):
        """Index of the next step (lbm_set_step_index): selects the random bits of
        stochastic rounding, so that recomputed steps repeat the forward run."""
        _check(self.lib.lbm_set_step_index(self.h, int(t)), self.h)

    def moments(self):
        """(rho (N,), u (D, N)) float32 device tensors of the current state."""
        rho = self.torch.empty(self.N, dtype=self.torch.float32, device=self.device)
        u = self.torch.empty(self.D * self.N, dtype=self.torch.float32, device=self.device)
        _check(self.lib.lbm_moments(self.h, _ptr(rho), _ptr(u)), self.h)
        return rho, u.reshape(self.D, self.N)

    def current(self):
        """(sum rho, sum rho u_x, sum rho u_y, sum rho u_z) over fluid nodes, FP64."""
        out = (ctypes.c_double * 4)()
        _check(self.lib.lbm_current(self.h, out), self.h)
        return np.array(out[:])

    def current_noalloc(self, out=None):
        """The totals of current() into a float64 (4,) device tensor, asynchronously, with
        the reduction in the library's static scratch (lbm_current_noalloc: no workspace,
        allocation or synchronisation inside the call)."""
        if out is None:
            out = self.torch.empty(4, dtype=self.torch.float64, device=self.device)
        _check(self.lib.lbm_current_noalloc(self.h, _ptr(out)), self.h)
        return out

    def speed_change(self, u, speed, have_previous=True):
        """Convergence measure of Sec. 9.4 (lbm_speed_change): the average over nodes with
        non-zero |u| of | |u| - speed | / |u|; speed (float32 (N,) device tensor) is then
        overwritten with |u|. u as returned by moments()."""
        out = ctypes.c_double()
        _check(self.lib.lbm_speed_change(self.h, _ptr(u), _ptr(speed), int(bool(have_previous)), ctypes.byref(out)),
               self.h)
        return out.value

    def run_until_steady(self, tol=1e-7, check_every=1000, max_steps=10 ** 6, span=100):
        """Step until the relative speed change per step (Sec. 9.4: the average over fluid
        nodes of | |u_new| - |u_old| | / |u_new|) falls below tol, checked every check_every
        steps. The change is taken across the last `span` steps of each check interval and
        divided by span (span = 1: two consecutive steps, the literal reading). While the
        flow settles the speeds change smoothly, so the quotient is the per-step change;
        but once that change nears FP32 rounding, every node's speed also jitters by about
        an ulp from step to step (a floor of a few 1e-7 on the 2D Ohm sample), which a
        difference across span steps divides by span. Returns (steps taken, last change);
        the rule was met if the change is below tol (else max_steps passed first)."""
        if check_every < 1 or not 1 <= span <= check_every:
            raise ValueError("need check_every >= 1 and 1 <= span <= check_every")
        speed = self.torch.empty(self.N, dtype=self.torch.float32, device=self.device)
        steps, change = 0, float("inf")
        while steps < max_steps:
            self.step(check_every - span)
            _, u = self.moments()
            self.speed_change(u, speed, have_previous=False)
            self.step(span)
            _, u = self.moments()
            change = self.speed_change(u, speed) / span
            steps += check_every
            if change < tol:
                break
        return steps, change

    def export_f64(self, state=None):
        """Pre-collision populations (Q, N) float64 in library order."""
        out = self.torch.empty(self.Q * self.N, dtype=self.torch.float64, device=self.device)
        _check(self.lib.lbm_export_f64(self.h, _ptr(state), _ptr(out)), self.h)
        return out.reshape(self.Q, self.N)

    def new_state(self, zero=True):
        """A state buffer of state_bytes (zero-filled, or left as allocated with zero=False:
        a step writes every location a later pull reads)."""
        if not zero:
            return self.torch.empty(self.sizes["state"], dtype=self.torch.uint8, device=self.device)
        return self.torch.zeros(self.sizes["state"], dtype=self.torch.uint8, device=self.device)

    def get_state(self, dst=None):
        dst = self.new_state() if dst is None else dst
        _check(self.lib.lbm_get_state(self.h, _ptr(dst)), self.h)
        return dst

    def set_state(self, src):
        _check(self.lib.lbm_set_state(self.h, _ptr(src)), self.h)

    def set_fields(self, E, B=(0.0, 0.0, 0.0)):
        e = (ctypes.c_double * 3)(*[float(v) for v in E])
        b = (ctypes.c_double * 3)(*[float(v) for v in B])
        _check(self.lib.lbm_set_fields(self.h, e, b), self.h)
        self.params.E, self.params.B = e, b

    def set_tau(self, tau):
        _check(self.lib.lbm_set_tau(self.h, float(tau)), self.h)
        self.params.tau = float(tau)

    # ------------------------------------------------------------------ adjoint
    def new_adjoint(self):
        return self.torch.zeros(self.sizes["adjoint"] // 4, dtype=self.torch.float32, device=self.device)

    def adjoint_seed(self, axis=0, norm=None, lam=None):
        lam = self.new_adjoint() if lam is None else lam
        _check(self.lib.lbm_adjoint_seed(self.h, int(axis), float(self.N if norm is None else norm), _ptr(lam)),
               self.h)
        return lam

    def adjoint_step(self, state, lam_in, lam_out, grad_s=None, grad_scalars=None):
        _check(self.lib.lbm_adjoint_step(self.h, _ptr(state), _ptr(lam_in), _ptr(lam_out), _ptr(grad_s),
                                         _ptr(grad_scalars)), self.h)

    def adjoint_view(self, lam):
        """(Q, N) view of an adjoint buffer (drops the stride padding)."""
        return lam.reshape(self.Q, self.stride)[:, : self.N]
