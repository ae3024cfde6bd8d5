"""MI355X lock-exchange lattice Boltzmann library: Python binding.

A thin ctypes layer over the C ABI in include/lbm.h (liblbm.so, built by
``paper_2112_08479_amd.build``). It only marshals arguments: device memory is
a torch uint8 tensor handed to the library as its workspace, the HIP stream is
torch's current stream, and every step of the method runs in the library's
HIP kernels. There is no fallback: if the library is missing the import of
``lib()`` raises.
"""
import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENODEV, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5, -6
CUMULANT27_Q7, BGK19_SMAG_Q6, CUMULANT27_FCM27 = 0, 1, 2
F64, F32, F16, BF16, BF16_F16S = 0, 1, 2, 3, 4
OUT_F64, OUT_F32 = 0, 1
STORAGE_NAMES = {F64: "f64", F32: "f32", F16: "f16", BF16: "bf16", BF16_F16S: "bf16_f16s"}

ERRORS = {LBM_EINVAL: "EINVAL", LBM_ENOMEM: "ENOMEM", LBM_EDEVICE: "EDEVICE",
          LBM_ENODEV: "ENODEV", LBM_EUNSTABLE: "EUNSTABLE", LBM_ESTATE: "ESTATE"}

# every symbol the header declares
EXPORTS = [
    "lbm_derive_params", "lbm_workspace_bytes", "lbm_state_bytes", "lbm_create", "lbm_destroy",
    "lbm_init_lock_exchange", "lbm_init_from_field", "lbm_step", "lbm_moments",
    "lbm_wall_shear", "lbm_diagnostics", "lbm_get_step", "lbm_checkpoint_save", "lbm_checkpoint_load",
    "lbm_get_populations", "lbm_set_populations", "lbm_adjoint_workspace_bytes",
    "lbm_adjoint_run", "lbm_stream_copy", "lbm_last_error", "lbm_checkpoint_diagnostics",
]


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class c_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("model", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("re_b", ctypes.c_double), ("sc", ctypes.c_double), ("g_prime", ctypes.c_double),
                ("ub_lu", ctypes.c_double), ("cs_smag", ctypes.c_double), ("sc_t", ctypes.c_double),
                ("omega_bulk", ctypes.c_double), ("omega3", ctypes.c_double),
                ("omega4", ctypes.c_double), ("omega5", ctypes.c_double), ("omega6", ctypes.c_double),
                ("parametrized", ctypes.c_int32), ("limiter", ctypes.c_double),
                ("smag_paper_form", ctypes.c_int32)]


class c_params(ctypes.Structure):
    _fields_ = [("u_b", ctypes.c_double), ("g_prime", ctypes.c_double), ("nu0", ctypes.c_double),
                ("tau0", ctypes.c_double), ("d0", ctypes.c_double), ("tau_phi0", ctypes.c_double),
                ("cs2_phi", ctypes.c_double), ("q_flow", ctypes.c_int32), ("q_scalar", ctypes.c_int32),
                ("w_plus", ctypes.c_double), ("w_minus", ctypes.c_double), ("w_111", ctypes.c_double),
                ("coef_a", ctypes.c_double), ("coef_b", ctypes.c_double)]


class c_diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t_nd", ctypes.c_double), ("mass", ctypes.c_double),
                ("mass0", ctypes.c_double), ("chi_mass", ctypes.c_double),
                ("chi_mass0", ctypes.c_double), ("fw", ctypes.c_double), ("fw_nd", ctypes.c_double),
                ("x_front", ctypes.c_double), ("x_f", ctypes.c_double), ("x_f_nd", ctypes.c_double),
                ("umax", ctypes.c_double), ("nonfinite", ctypes.c_int64)]


_lib = None


def lib():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run python -m paper_2112_08479_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, dbl, cfgp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(c_config)
        sig = {
            "lbm_derive_params": (ctypes.c_int, [cfgp, ctypes.POINTER(c_params)]),
            "lbm_workspace_bytes": (ctypes.c_size_t, [cfgp]),
            "lbm_state_bytes": (ctypes.c_size_t, [cfgp]),
            "lbm_create": (ctypes.c_int, [cfgp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
            "lbm_destroy": (ctypes.c_int, [vp]),
            "lbm_init_lock_exchange": (ctypes.c_int, [vp, dbl, dbl, ctypes.c_uint64]),
            "lbm_init_from_field": (ctypes.c_int, [vp, vp, dbl]),
            "lbm_step": (ctypes.c_int, [vp, i64]),
            "lbm_moments": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp, vp, vp]),
            "lbm_wall_shear": (ctypes.c_int, [vp, ctypes.c_int, vp, vp]),
            "lbm_diagnostics": (ctypes.c_int, [vp, ctypes.POINTER(c_diag)]),
            "lbm_get_step": (ctypes.c_int, [vp, ctypes.POINTER(i64)]),
            "lbm_checkpoint_save": (ctypes.c_int, [vp, vp]),
            "lbm_checkpoint_load": (ctypes.c_int, [vp, vp]),
            "lbm_get_populations": (ctypes.c_int, [vp, vp, vp]),
            "lbm_set_populations": (ctypes.c_int, [vp, vp, vp]),
            "lbm_stream_copy": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
            "lbm_adjoint_workspace_bytes": (ctypes.c_size_t, [cfgp, i64, i64]),
            "lbm_adjoint_run": (ctypes.c_int, [vp, i64, i64, dbl, dbl, vp, ctypes.c_size_t,
                                               ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                               ctypes.POINTER(dbl), vp]),
            "lbm_last_error": (ctypes.c_char_p, []),
            "lbm_checkpoint_diagnostics": (ctypes.c_int, [cfgp, vp, vp, ctypes.POINTER(c_diag)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != LBM_OK:
        raise LBMError(rc, lib().lbm_last_error().decode())
    return rc


@dataclass
class Config:
    nx: int
    ny: int
    nz: int
    model: int = CUMULANT27_Q7
    storage: int = F32
    re_b: float = 1000.0
    sc: float = 1.0
    g_prime: float = 1e-4
    ub_lu: float = 0.0
    cs_smag: float = 0.0
    sc_t: float = 1.0
    omega_bulk: float = 1.0
    omega3: float = 1.0
    omega4: float = 1.0
    omega5: float = 1.0
    omega6: float = 1.0
    parametrized: bool = False     # parametrised cumulant (third-order rates from omega1)
    limiter: float = 0.0           # third-order limiter lambda; 0 = none
    smag_paper_form: bool = False  # nu_T = C_s |S| as printed (else (C_s)^2 |S|)

    def c(self):
        s = c_config()
        s.struct_size = ctypes.sizeof(c_config)
        for f in c_config._fields_[1:]:
            v = getattr(self, f[0])
            setattr(s, f[0], int(v) if f[1] is ctypes.c_int32 else v)
        return s

    @property
    def n(self):
        return self.nx * self.ny * self.nz


def derive_params(cfg):
    p = c_params()
    check(lib().lbm_derive_params(ctypes.byref(cfg.c()), ctypes.byref(p)))
    return {f[0]: getattr(p, f[0]) for f in c_params._fields_}


def workspace_bytes(cfg):
    return int(lib().lbm_workspace_bytes(ctypes.byref(cfg.c())))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def stream_copy(dst, src, nbytes, stream):
    """Plain streaming copy of nbytes between device tensors (measurement utility)."""
    check(lib().lbm_stream_copy(_ptr(dst), _ptr(src), int(nbytes), ctypes.c_void_p(stream.cuda_stream)))


class Lattice:
    """A lattice on one GPU. Device memory comes from torch (caller-owned
    workspace); all computation runs in the library's kernels on `stream`."""

    def __init__(self, cfg, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.L = lib()
        nbytes = workspace_bytes(cfg)
        if nbytes == 0:
            # re-run the validation to get the message
            check(self.L.lbm_derive_params(ctypes.byref(cfg.c()), ctypes.byref(c_params())))
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            check(self.L.lbm_create(ctypes.byref(cfg.c()), _ptr(self.ws), nbytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.params = derive_params(cfg)

    def close(self):
        if getattr(self, "h", None):
            self.L.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_lock_exchange(self, lock_fraction=0.125, noise_amp=1e-3, seed=0):
        check(self.L.lbm_init_lock_exchange(self.h, lock_fraction, noise_amp, seed))

    def init_from_field(self, chi0, lock_fraction=0.125):
        """chi0: float64 device tensor (nz, ny, nx) or flat."""
        self._chi0 = chi0.contiguous()
        check(self.L.lbm_init_from_field(self.h, _ptr(self._chi0), lock_fraction))

    def step(self, n=1):
        check(self.L.lbm_step(self.h, int(n)))

    @property
    def step_count(self):
        s = ctypes.c_int64()
        check(self.L.lbm_get_step(self.h, ctypes.byref(s)))
        return s.value

    def moments(self, dtype=OUT_F64):
        torch = self.torch
        tdt = torch.float64 if dtype == OUT_F64 else torch.float32
        shp = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        out = {k: torch.empty(shp, dtype=tdt, device=self.device) for k in ("rho", "ux", "uy", "uz", "chi")}
        check(self.L.lbm_moments(self.h, dtype, *(_ptr(out[k]) for k in ("rho", "ux", "uy", "uz", "chi"))))
        return out

    def wall_shear(self, dtype=OUT_F64):
        """Bottom-wall shear stress tau_w (ny, nx) and its span average (nx),
        lattice units, as device tensors."""
        torch = self.torch
        tdt = torch.float64 if dtype == OUT_F64 else torch.float32
        tau = torch.empty((self.cfg.ny, self.cfg.nx), dtype=tdt, device=self.device)
        bar = torch.empty((self.cfg.nx,), dtype=tdt, device=self.device)
        check(self.L.lbm_wall_shear(self.h, dtype, _ptr(tau), _ptr(bar)))
        return tau, bar

    def diagnostics(self, raise_unstable=True):
        d = c_diag()
        rc = self.L.lbm_diagnostics(self.h, ctypes.byref(d))
        if rc != LBM_OK and (rc != LBM_EUNSTABLE or raise_unstable):
            check(rc)
        return {f[0]: getattr(d, f[0]) for f in c_diag._fields_}

    def get_populations(self):
        p = self.params
        n = self.cfg.n
        f = np.empty((p["q_flow"], n), dtype=np.float64)
        phi = np.empty((p["q_scalar"], n), dtype=np.float64)
        check(self.L.lbm_get_populations(self.h, f.ctypes.data_as(ctypes.c_void_p),
                                         phi.ctypes.data_as(ctypes.c_void_p)))
        shp = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        return f.reshape(-1, *shp), phi.reshape(-1, *shp)

    def set_populations(self, f, phi):
        f = np.ascontiguousarray(f, dtype=np.float64)
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        check(self.L.lbm_set_populations(self.h, f.ctypes.data_as(ctypes.c_void_p),
                                         phi.ctypes.data_as(ctypes.c_void_p)))

    def state_bytes(self):
        return int(self.L.lbm_state_bytes(ctypes.byref(self.cfg.c())))

    def checkpoint_save(self, slot=None):
        torch = self.torch
        if slot is None:
            slot = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        check(self.L.lbm_checkpoint_save(self.h, _ptr(slot)))
        return slot

    def checkpoint_load(self, slot):
        check(self.L.lbm_checkpoint_load(self.h, _ptr(slot)))

    def adjoint_workspace_bytes(self, n_steps, k_ckpt=100):
        nb = int(self.L.lbm_adjoint_workspace_bytes(ctypes.byref(self.cfg.c()), int(n_steps), int(k_ckpt)))
        if nb == 0:
            check(LBM_EINVAL)
        return nb

    def adjoint_run(self, n_steps, k_ckpt=100, w_front=1.0, w_fw=1.0, ws=None, gchi=None):
        """Runs the forward n_steps from the current (initial) state and the
        hand-written adjoint. Returns (J, dJ/dC_s, dJ/dSc_T, dJ/dchi0 tensor).
        ws (uint8, adjoint_workspace_bytes) and gchi (float64, nz*ny*nx) may
        be given as preallocated device tensors; else they are allocated."""
        torch = self.torch
        nb = self.adjoint_workspace_bytes(n_steps, k_ckpt)
        if ws is None:
            ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        if gchi is None:
            gchi = torch.empty((self.cfg.nz, self.cfg.ny, self.cfg.nx), dtype=torch.float64, device=self.device)
        if ws.numel() * ws.element_size() < nb or gchi.dtype != torch.float64 or gchi.numel() != self.cfg.n:
            raise ValueError("adjoint workspace or gradient buffer of the wrong size or type")
        J, dcs, dsct = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        check(self.L.lbm_adjoint_run(self.h, int(n_steps), int(k_ckpt), float(w_front), float(w_fw),
                                     _ptr(ws), ws.numel() * ws.element_size(), ctypes.byref(J),
                                     ctypes.byref(dcs), ctypes.byref(dsct), _ptr(gchi)))
        return J.value, dcs.value, dsct.value, gchi


def lock_exchange_objective(chi0, cs_smag, sc_t, cfg, n_steps, k_ckpt=100, w_front=1.0, w_fw=1.0,
                            lock_fraction=0.125):
    """J = w_front x_f(n) + w_fw (1/n) sum_{m=1..n} F_w(m) of an n-step run from
    the initial concentration chi0 (float64 tensor (nz, ny, nx) on the GPU),
    differentiable with respect to chi0, cs_smag and sc_t (0-d tensors)
    through the library's hand-written adjoint (checkpoint every k_ckpt
    steps). cfg gives the grid, model, storage and the other parameters."""
    return _Objective.apply(chi0, cs_smag, sc_t, cfg, int(n_steps), int(k_ckpt), float(w_front),
                            float(w_fw), float(lock_fraction))


def _objective_cls():
    import dataclasses

    import torch

    class Objective(torch.autograd.Function):
        @staticmethod
        def forward(ctx, chi0, cs, sct, cfg, n_steps, k_ckpt, w_front, w_fw, lock_fraction):
            c = dataclasses.replace(cfg, cs_smag=float(cs), sc_t=float(sct))
            lat = Lattice(c, device=chi0.device)
            lat.init_from_field(chi0.detach().to(torch.float64).contiguous(), lock_fraction)
            J, dcs, dsct, gchi = lat.adjoint_run(n_steps, k_ckpt, w_front, w_fw)
            lat.close()
            ctx.save_for_backward(gchi.to(chi0.dtype), torch.tensor(dcs, dtype=cs.dtype),
                                  torch.tensor(dsct, dtype=sct.dtype))
            return torch.tensor(J, dtype=torch.float64, device=chi0.device)

        @staticmethod
        def backward(ctx, gJ):
            gchi, dcs, dsct = ctx.saved_tensors
            g = gJ.to(gchi.device)
            return (g * gchi, (g.cpu() * dcs).to(dcs.dtype), (g.cpu() * dsct).to(dsct.dtype),
                    None, None, None, None, None, None)

    return Objective


class _Lazy:
    _cls = None

    @classmethod
    def apply(cls, *a):
        if cls._cls is None:
            cls._cls = _objective_cls()
        return cls._cls.apply(*a)


_Objective = _Lazy
