"""ctypes binding of ``libphoebe_gpu.so`` (argument marshalling only).

Every computation happens in the HIP library; this module converts torch
tensors (device memory, streams) and numpy arrays (host lattice-vector lists)
into the C ABI's plain pointers and sizes.  The functions raise ``PhoebeError``
on any non-OK status, and loading fails loudly if the library has not been
built.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libphoebe_gpu.so")

PHOEBE_FP64, PHOEBE_FP32, PHOEBE_BF16X3, PHOEBE_BF16X6, PHOEBE_BF16 = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": PHOEBE_FP64, "fp32": PHOEBE_FP32, "bf16x3": PHOEBE_BF16X3,
              "bf16x6": PHOEBE_BF16X6, "bf16": PHOEBE_BF16}
STATUS = {0: "PHOEBE_OK", -1: "PHOEBE_E_INVALID", -2: "PHOEBE_E_NOMEM", -3: "PHOEBE_E_DEVICE",
          -4: "PHOEBE_E_UNSUPPORTED", -5: "PHOEBE_E_NUMERIC"}

#: every symbol the header declares
EXPORTS = (
    "phoebe_gpu_abi_version", "phoebe_gpu_create", "phoebe_gpu_destroy",
    "phoebe_gpu_last_error", "phoebe_gpu_electron_bands", "phoebe_gpu_phonon_modes",
    "phoebe_gpu_interp_g", "phoebe_gpu_scatter_rates", "phoebe_gpu_set_timing",
    "phoebe_gpu_kernel_time", "phoebe_gpu_reset_timing",
    "phoebe_gpu_batched_plan", "phoebe_gpu_batched_run", "phoebe_gpu_batched_info",
    "phoebe_gpu_batched_destroy", "phoebe_gpu_rate_terms", "phoebe_gpu_mlp_param_count",
    "phoebe_gpu_mlp_forward", "phoebe_gpu_mlp_grad", "phoebe_gpu_mlp_adam",
    "phoebe_gpu_mlp_features", "phoebe_gpu_propose_q", "phoebe_gpu_delta_weights",
    "phoebe_gpu_set_mesh_sum", "phoebe_gpu_mlp_feature_count", "phoebe_gpu_kernel_bytes",
    "phoebe_gpu_phonon_linewidth", "phoebe_gpu_velocities", "phoebe_gpu_polar_factor",
    "phoebe_gpu_interp_v3", "phoebe_gpu_philox_uniform", "phoebe_gpu_philox_randint",
    "phoebe_gpu_mlp_init", "phoebe_gpu_training_set", "phoebe_gpu_gather_rows",
    "phoebe_gpu_set_check_finite", "phoebe_gpu_scatter_rates_noalloc",
    "phoebe_gpu_noalloc_scratch_bytes", "phoebe_gpu_set_table_cache",
    "phoebe_gpu_set_fault_injection", "phoebe_gpu_interp_g_mesh",
)

SMEARING = {"gaussian": 0, "adaptive": 1}


class PhoebeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class CPolar(ctypes.Structure):
    _fields_ = [("born", ctypes.c_void_p), ("eps_inf", ctypes.c_double * 9),
                ("alpha", ctypes.c_double), ("g_max", ctypes.c_int32)]


class CSystem(ctypes.Structure):
    _fields_ = [
        ("n_wannier", ctypes.c_int32), ("n_atoms", ctypes.c_int32),
        ("n_rh", ctypes.c_int32), ("rh", ctypes.c_void_p), ("h_r", ctypes.c_void_p),
        ("n_rd", ctypes.c_int32), ("rd", ctypes.c_void_p), ("phi_r", ctypes.c_void_p),
        ("mass", ctypes.c_void_p),
        ("n_re", ctypes.c_int32), ("re", ctypes.c_void_p),
        ("n_rp", ctypes.c_int32), ("rp", ctypes.c_void_p),
        ("g_rr", ctypes.c_void_p),
        ("polar", ctypes.POINTER(CPolar)),
    ]


class CSystem3(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32),
        ("n_rd", ctypes.c_int32), ("rd", ctypes.c_void_p), ("phi_r", ctypes.c_void_p),
        ("mass", ctypes.c_void_p),
        ("n_r1", ctypes.c_int32), ("r1", ctypes.c_void_p),
        ("n_r2", ctypes.c_int32), ("r2", ctypes.c_void_p),
        ("phi3", ctypes.c_void_p),
    ]


class CRateParams(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("kT", ctypes.c_double), ("sigma", ctypes.c_double),
                ("win_lo", ctypes.c_double), ("win_hi", ctypes.c_double),
                ("omega_min", ctypes.c_double), ("smearing", ctypes.c_int32),
                ("adaptive_scale", ctypes.c_double)]


def rate_params(p: dict) -> CRateParams:
    """C rate parameters from a dict (mu, kT, sigma, win_lo, win_hi, optional omega_min,
    smearing "gaussian"/"adaptive" and adaptive_scale)."""
    return CRateParams(p["mu"], p["kT"], p["sigma"], p["win_lo"], p["win_hi"],
                       p.get("omega_min", 1e-4), SMEARING[p.get("smearing", "gaussian")],
                       float(p.get("adaptive_scale", 1.0)))


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2111_14999_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.phoebe_gpu_abi_version.restype = i32
    lib.phoebe_gpu_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(vp)]
    lib.phoebe_gpu_destroy.argtypes = [vp]
    lib.phoebe_gpu_last_error.argtypes = [vp]
    lib.phoebe_gpu_last_error.restype = ctypes.c_char_p
    lib.phoebe_gpu_electron_bands.argtypes = [vp, ctypes.POINTER(CSystem), vp, i64, vp, vp, vp]
    lib.phoebe_gpu_phonon_modes.argtypes = [vp, ctypes.POINTER(CSystem), vp, i64, vp, vp, vp]
    lib.phoebe_gpu_interp_g.argtypes = [vp, ctypes.POINTER(CSystem), vp, i64, vp, i64,
                                        ctypes.c_double, ctypes.c_int, vp, vp, vp, vp, vp]
    lib.phoebe_gpu_interp_g_mesh.argtypes = [vp, ctypes.POINTER(CSystem), vp, i64,
                                             ctypes.POINTER(i32), ctypes.c_double, i32, vp, vp,
                                             vp, vp, vp]
    lib.phoebe_gpu_scatter_rates.argtypes = [vp, ctypes.POINTER(CSystem),
                                             ctypes.POINTER(i32), ctypes.POINTER(i32), vp, i64,
                                             vp, vp, vp, ctypes.POINTER(CRateParams), ctypes.c_int,
                                             vp, vp, vp, ctypes.POINTER(i64), vp]
    lib.phoebe_gpu_scatter_rates_noalloc.argtypes = lib.phoebe_gpu_scatter_rates.argtypes
    lib.phoebe_gpu_noalloc_scratch_bytes.restype = ctypes.c_size_t
    lib.phoebe_gpu_noalloc_scratch_bytes.argtypes = []
    lib.phoebe_gpu_phonon_linewidth.argtypes = [vp, ctypes.POINTER(CSystem), ctypes.POINTER(i32),
                                                ctypes.POINTER(i32), ctypes.POINTER(CRateParams),
                                                ctypes.c_int, vp, vp, ctypes.POINTER(i64), vp]
    lib.phoebe_gpu_velocities.argtypes = [vp, ctypes.POINTER(CSystem), vp, i64, vp, vp, vp]
    lib.phoebe_gpu_polar_factor.argtypes = [vp, ctypes.POINTER(CSystem), vp, i64, ctypes.c_double,
                                            vp, vp]
    lib.phoebe_gpu_interp_v3.argtypes = [vp, ctypes.POINTER(CSystem3), vp, i64, vp, i64,
                                         ctypes.c_double, vp, vp, vp, vp, vp]
    u64 = ctypes.c_uint64
    lib.phoebe_gpu_philox_uniform.argtypes = [vp, u64, u64, i64, vp, vp]
    lib.phoebe_gpu_philox_randint.argtypes = [vp, u64, u64, i64, i64, vp, vp]
    lib.phoebe_gpu_mlp_init.argtypes = [vp, ctypes.c_int, vp, i32, i32, i32, u64, vp]
    lib.phoebe_gpu_training_set.argtypes = [vp, vp, vp, i64, i64, i32, ctypes.c_double,
                                            ctypes.c_double, i64, u64, vp, vp, vp, vp, i64,
                                            ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                            vp]
    lib.phoebe_gpu_gather_rows.argtypes = [vp, vp, i64, i64, vp, i64, vp, vp]
    lib.phoebe_gpu_set_check_finite.argtypes = [vp, ctypes.c_int]
    lib.phoebe_gpu_set_table_cache.argtypes = [vp, ctypes.c_int]
    lib.phoebe_gpu_set_fault_injection.argtypes = [vp, i64]
    lib.phoebe_gpu_set_timing.argtypes = [vp, ctypes.c_int]
    lib.phoebe_gpu_set_mesh_sum.argtypes = [vp, i32]
    lib.phoebe_gpu_kernel_bytes.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double)]
    lib.phoebe_gpu_reset_timing.argtypes = [vp]
    lib.phoebe_gpu_kernel_time.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i64),
                                           ctypes.POINTER(ctypes.c_double)]
    lib.phoebe_gpu_batched_plan.argtypes = [vp, ctypes.POINTER(CSystem), i32, ctypes.POINTER(i32),
                                            ctypes.POINTER(CRateParams), ctypes.c_int,
                                            ctypes.c_char_p, ctypes.POINTER(vp),
                                            ctypes.POINTER(i64), vp]
    lib.phoebe_gpu_batched_run.argtypes = [vp, ctypes.POINTER(vp), vp]
    lib.phoebe_gpu_batched_info.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                            ctypes.POINTER(i64), ctypes.POINTER(i64),
                                            ctypes.POINTER(ctypes.c_double)]
    lib.phoebe_gpu_batched_destroy.argtypes = [vp]
    lib.phoebe_gpu_rate_terms.argtypes = [vp, ctypes.POINTER(CSystem), ctypes.POINTER(i32), vp, i64,
                                          ctypes.POINTER(CRateParams), vp, vp, vp, vp, vp, i64,
                                          ctypes.POINTER(i64), vp]
    lib.phoebe_gpu_delta_weights.argtypes = [vp, ctypes.POINTER(CSystem), ctypes.POINTER(i32), vp,
                                             i64, ctypes.POINTER(CRateParams), vp, vp, vp, i64,
                                             ctypes.POINTER(i64), vp, vp]
    lib.phoebe_gpu_mlp_param_count.argtypes = [i32, i32, i32]
    lib.phoebe_gpu_mlp_param_count.restype = i64
    lib.phoebe_gpu_mlp_forward.argtypes = [vp, ctypes.c_int, vp, i32, i32, i32, vp, i64, vp, vp]
    lib.phoebe_gpu_mlp_grad.argtypes = [vp, ctypes.c_int, vp, i32, i32, i32, vp, vp, i64, vp,
                                        ctypes.POINTER(ctypes.c_double), vp]
    lib.phoebe_gpu_mlp_adam.argtypes = [vp, vp, vp, vp, vp, i64, i32, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double, vp]
    lib.phoebe_gpu_mlp_features.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i32), i32, i32, vp,
                                            vp, vp, vp, i64, ctypes.c_double, ctypes.c_double, vp,
                                            vp]
    lib.phoebe_gpu_mlp_feature_count.restype = i32
    lib.phoebe_gpu_mlp_feature_count.argtypes = [i32, i32]
    lib.phoebe_gpu_propose_q.argtypes = [vp, ctypes.POINTER(i32), i32, i32, ctypes.POINTER(i32),
                                         ctypes.POINTER(ctypes.c_double), i64, vp, vp, i32, i32,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, i32, vp, vp, vp, vp, vp]
    for name in EXPORTS:
        if name not in ("phoebe_gpu_abi_version", "phoebe_gpu_last_error",
                        "phoebe_gpu_mlp_param_count", "phoebe_gpu_noalloc_scratch_bytes"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _state_capacity(mesh, sys, per_q, per_q2, st_row, st_band) -> int:
    """Rows every per-state output can hold; per-(q, mode) outputs must be [rows, N_q, nModes]."""
    nq = int(mesh[0]) * int(mesh[1]) * int(mesh[2])
    caps = []
    for t in (per_q, per_q2):
        if t is not None:
            if tuple(t.shape[1:]) != (nq, 3 * sys.n_atoms):
                raise ValueError(f"per-(q, mode) output must be [states, {nq}, {3 * sys.n_atoms}]")
            caps.append(int(t.shape[0]))
    for t in (st_row, st_band):
        if t is not None:
            caps.append(int(t.shape[0]))
    return min(caps)


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


@dataclass
class DeviceSystem:
    """A system whose tensors live on the GPU (torch) and lattice lists on the host."""

    n_wannier: int
    n_atoms: int
    rh: np.ndarray
    h_r: object
    rd: np.ndarray
    phi_r: object
    mass: object
    re: np.ndarray
    rp: np.ndarray
    g_rr: object
    polar: Optional[dict] = None  # born [nat,3,3], eps_inf [3,3], alpha, g_max (host)

    @staticmethod
    def from_host(system, device="cuda:0", with_coupling=True) -> "DeviceSystem":
        """Copy a host system (numpy arrays) to the device."""
        import torch

        def dev(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device)

        def ivec(a):
            return np.ascontiguousarray(a, dtype=np.int32)

        g = dev(system.g_rr) if (with_coupling and system.g_rr is not None) else None
        polar = None
        if getattr(system, "born", None) is not None:
            polar = dict(born=np.ascontiguousarray(system.born, dtype=np.float64),
                         eps_inf=np.ascontiguousarray(system.eps_inf, dtype=np.float64),
                         alpha=float(system.ewald_alpha), g_max=int(system.g_max))
        return DeviceSystem(system.n_wannier, system.n_atoms, ivec(system.rh), dev(system.h_r),
                            ivec(system.rd), dev(system.phi_r), dev(system.mass),
                            ivec(system.re), ivec(system.rp), g, polar)

    def c_struct(self) -> CSystem:
        c = CSystem()
        if self.polar is not None:
            p = CPolar()
            p.born = self.polar["born"].ctypes.data
            p.eps_inf = (ctypes.c_double * 9)(*[float(x) for x in self.polar["eps_inf"].ravel()])
            p.alpha, p.g_max = self.polar["alpha"], self.polar["g_max"]
            self._cpolar = p  # kept alive with the struct that points to it
            c.polar = ctypes.pointer(p)
        c.n_wannier, c.n_atoms = self.n_wannier, self.n_atoms
        c.n_rh, c.rh, c.h_r = self.rh.shape[0], self.rh.ctypes.data, _ptr(self.h_r)
        c.n_rd, c.rd, c.phi_r = self.rd.shape[0], self.rd.ctypes.data, _ptr(self.phi_r)
        c.mass = _ptr(self.mass)
        c.n_re, c.re = self.re.shape[0], self.re.ctypes.data
        c.n_rp, c.rp = self.rp.shape[0], self.rp.ctypes.data
        c.g_rr = _ptr(self.g_rr)
        return c


@dataclass
class DeviceSystem3:
    """Harmonic and third-order force constants on the GPU, lattice lists on the host."""

    n_atoms: int
    rd: np.ndarray
    phi_r: object
    mass: object
    r1: np.ndarray
    r2: np.ndarray
    phi3: object

    @staticmethod
    def from_host(system, r, phi3, device="cuda:0") -> "DeviceSystem3":
        """From a host system (harmonic part) and third-order constants on lattice list r
        (used for both displacements)."""
        import torch

        def dev(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device)

        rr = np.ascontiguousarray(r, dtype=np.int32)
        return DeviceSystem3(system.n_atoms, np.ascontiguousarray(system.rd, dtype=np.int32),
                             dev(system.phi_r), dev(system.mass), rr, rr.copy(), dev(phi3))

    def c_struct(self) -> CSystem3:
        c = CSystem3()
        c.n_atoms = self.n_atoms
        c.n_rd, c.rd, c.phi_r, c.mass = self.rd.shape[0], self.rd.ctypes.data, _ptr(self.phi_r), \
            _ptr(self.mass)
        c.n_r1, c.r1 = self.r1.shape[0], self.r1.ctypes.data
        c.n_r2, c.r2 = self.r2.shape[0], self.r2.ctypes.data
        c.phi3 = _ptr(self.phi3)
        return c


class Library:
    """One handle of the HIP library on one device."""

    def __init__(self, device: int = 0, workspace_budget: int = 0):
        self.lib = load()
        h = ctypes.c_void_p()
        st = self.lib.phoebe_gpu_create(device, workspace_budget, ctypes.byref(h))
        if st != 0:
            raise PhoebeError(st, self.lib.phoebe_gpu_last_error(None).decode())
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self.lib.phoebe_gpu_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise PhoebeError(st, self.lib.phoebe_gpu_last_error(self.handle).decode())

    @staticmethod
    def abi_version() -> int:
        return int(load().phoebe_gpu_abi_version())

    # -- band structure -----------------------------------------------------
    def electron_bands(self, sys: DeviceSystem, k_frac, eps_out, u_out=None, stream=None):
        c = sys.c_struct()
        self._check(self.lib.phoebe_gpu_electron_bands(
            self.handle, ctypes.byref(c), _ptr(k_frac), k_frac.shape[0], _ptr(eps_out),
            _ptr(u_out), _stream(stream)))

    def phonon_modes(self, sys: DeviceSystem, q_frac, omega_out, z_out=None, stream=None):
        c = sys.c_struct()
        self._check(self.lib.phoebe_gpu_phonon_modes(
            self.handle, ctypes.byref(c), _ptr(q_frac), q_frac.shape[0], _ptr(omega_out),
            _ptr(z_out), _stream(stream)))

    # -- coupling -----------------------------------------------------------
    def interp_g(self, sys: DeviceSystem, k_frac, q_frac, g_out, omega_min=1e-4,
                 precision="fp64", eps_k=None, eps_kq=None, omega_q=None, stream=None):
        c = sys.c_struct()
        self._check(self.lib.phoebe_gpu_interp_g(
            self.handle, ctypes.byref(c), _ptr(k_frac), k_frac.shape[0], _ptr(q_frac),
            q_frac.shape[0], float(omega_min), PRECISIONS[precision], _ptr(g_out),
            _ptr(eps_k), _ptr(eps_kq), _ptr(omega_q), _stream(stream)))

    def interp_g_mesh(self, sys: DeviceSystem, k_frac, q_mesh, g_out, omega_min=1e-4,
                      precision="fp64", eps_k=None, eps_kq=None, omega_q=None, stream=None):
        """interp_g with q the full mesh q_mesh in linear order."""
        c = sys.c_struct()
        m = (ctypes.c_int32 * 3)(*[int(x) for x in q_mesh])
        self._check(self.lib.phoebe_gpu_interp_g_mesh(
            self.handle, ctypes.byref(c), _ptr(k_frac), k_frac.shape[0], m, float(omega_min),
            PRECISIONS[precision], _ptr(g_out), _ptr(eps_k), _ptr(eps_kq), _ptr(omega_q),
            _stream(stream)))

    # -- rates --------------------------------------------------------------
    def scatter_rates(self, sys: DeviceSystem, mesh, params: dict, gamma_out, k_idx=None,
                      q_lists=None, precision="fp64", band_mask=None, kept_k_out=None,
                      stream=None, q_mesh=None) -> int:
        c = sys.c_struct()
        m = (ctypes.c_int32 * 3)(*[int(x) for x in mesh])
        mq = (ctypes.c_int32 * 3)(*[int(x) for x in (mesh if q_mesh is None else q_mesh)])
        p = rate_params(params)
        nk = 0 if k_idx is None else int(k_idx.shape[0])
        q_off = q_idx = q_w = None
        if q_lists is not None:
            q_off, q_idx, q_w = q_lists
        n_kept = ctypes.c_int64(0)
        self._check(self.lib.phoebe_gpu_scatter_rates(
            self.handle, ctypes.byref(c), m, mq, _ptr(k_idx), nk, _ptr(q_off), _ptr(q_idx),
            _ptr(q_w), ctypes.byref(p), PRECISIONS[precision], _ptr(gamma_out), _ptr(band_mask),
            _ptr(kept_k_out), ctypes.byref(n_kept), _stream(stream)))
        return int(n_kept.value)

    def scatter_rates_noalloc(self, sys: DeviceSystem, mesh, params: dict, gamma_out,
                              k_idx=None, q_lists=None, precision="fp64", band_mask=None,
                              kept_k_out=None, stream=None, q_mesh=None) -> int:
        """scatter_rates with the library's static device scratch (no device allocation)."""
        c = sys.c_struct()
        m = (ctypes.c_int32 * 3)(*[int(x) for x in mesh])
        mq = (ctypes.c_int32 * 3)(*[int(x) for x in (mesh if q_mesh is None else q_mesh)])
        p = rate_params(params)
        nk = 0 if k_idx is None else int(k_idx.shape[0])
        q_off = q_idx = q_w = None
        if q_lists is not None:
            q_off, q_idx, q_w = q_lists
        n_kept = ctypes.c_int64(0)
        self._check(self.lib.phoebe_gpu_scatter_rates_noalloc(
            self.handle, ctypes.byref(c), m, mq, _ptr(k_idx), nk, _ptr(q_off), _ptr(q_idx),
            _ptr(q_w), ctypes.byref(p), PRECISIONS[precision], _ptr(gamma_out), _ptr(band_mask),
            _ptr(kept_k_out), ctypes.byref(n_kept), _stream(stream)))
        return int(n_kept.value)

    @staticmethod
    def noalloc_scratch_bytes() -> int:
        return int(load().phoebe_gpu_noalloc_scratch_bytes())

    def phonon_linewidth(self, sys: DeviceSystem, mesh, params: dict, p_out, gamma_out=None,
                         precision="fp64", stream=None, q_mesh=None) -> int:
        """P^{el-ph}[q, nu] on the full mesh (p_out [N, nModes]); returns the kept k count."""
        c = sys.c_struct()
        m = (ctypes.c_int32 * 3)(*[int(x) for x in mesh])
        mq = (ctypes.c_int32 * 3)(*[int(x) for x in (mesh if q_mesh is None else q_mesh)])
        p = rate_params(params)
        n_kept = ctypes.c_int64(0)
        self._check(self.lib.phoebe_gpu_phonon_linewidth(
            self.handle, ctypes.byref(c), m, mq, ctypes.byref(p), PRECISIONS[precision],
            _ptr(p_out), _ptr(gamma_out), ctypes.byref(n_kept), _stream(stream)))
        return int(n_kept.value)

    def velocities(self, sys: DeviceSystem, k_frac, v_out, eps_out=None, stream=None):
        c = sys.c_struct()
        self._check(self.lib.phoebe_gpu_velocities(
            self.handle, ctypes.byref(c), _ptr(k_frac), int(k_frac.shape[0]), _ptr(eps_out),
            _ptr(v_out), _stream(stream)))

    def polar_factor(self, sys: DeviceSystem, q_frac, l_out, omega_min=1e-4, stream=None):
        c = sys.c_struct()
        self._check(self.lib.phoebe_gpu_polar_factor(
            self.handle, ctypes.byref(c), _ptr(q_frac), int(q_frac.shape[0]), float(omega_min),
            _ptr(l_out), _stream(stream)))

    def interp_v3(self, sys3: "DeviceSystem3", q_frac, qp_frac, v3_out, omega_min=1e-4,
                  omega_q=None, omega_qp=None, omega_qpp=None, stream=None):
        c = sys3.c_struct()
        self._check(self.lib.phoebe_gpu_interp_v3(
            self.handle, ctypes.byref(c), _ptr(q_frac), int(q_frac.shape[0]), _ptr(qp_frac),
            int(qp_frac.shape[0]), float(omega_min), _ptr(v3_out), _ptr(omega_q), _ptr(omega_qp),
            _ptr(omega_qpp), _stream(stream)))

    def philox_uniform(self, seed, offset, out, stream=None):
        self._check(self.lib.phoebe_gpu_philox_uniform(
            self.handle, int(seed), int(offset), int(out.numel()), _ptr(out), _stream(stream)))

    def philox_randint(self, seed, offset, hi, out, stream=None):
        self._check(self.lib.phoebe_gpu_philox_randint(
            self.handle, int(seed), int(offset), int(out.numel()), int(hi), _ptr(out),
            _stream(stream)))

    def mlp_init(self, params, n_in, width, depth, seed, precision="bf16", stream=None):
        self._check(self.lib.phoebe_gpu_mlp_init(
            self.handle, PRECISIONS[precision], _ptr(params), n_in, width, depth, int(seed),
            _stream(stream)))

    def training_set(self, terms, dweights, n_states, d_threshold, c_frac, max_samples, seed,
                     out_state, out_q, out_nu, out_y, stream=None):
        """Returns (entries written, c)."""
        n = ctypes.c_int64(0)
        c = ctypes.c_double(0.0)
        self._check(self.lib.phoebe_gpu_training_set(
            self.handle, _ptr(terms), _ptr(dweights), int(n_states), int(terms.shape[1]),
            int(terms.shape[2]), float(d_threshold), float(c_frac), int(max_samples), int(seed),
            _ptr(out_state), _ptr(out_q), _ptr(out_nu), _ptr(out_y), int(out_y.shape[0]),
            ctypes.byref(n), ctypes.byref(c), _stream(stream)))
        return int(n.value), float(c.value)

    def gather_rows(self, src, idx, dst, stream=None):
        """dst[i] = src[idx[i]] (rows of src's trailing dimensions)."""
        row_bytes = int(src[0].numel() * src.element_size()) if src.shape[0] else 0
        self._check(self.lib.phoebe_gpu_gather_rows(
            self.handle, _ptr(src), int(src.shape[0]), row_bytes, _ptr(idx), int(idx.shape[0]),
            _ptr(dst), _stream(stream)))

    def set_fault_injection(self, at: int):
        """Report the at-th checked HIP call from now on as failed (0: off); for testing."""
        self._check(self.lib.phoebe_gpu_set_fault_injection(self.handle, int(at)))

    def set_table_cache(self, on: bool):
        """Reuse band and phonon tables across rate calls on the same system and mesh."""
        self._check(self.lib.phoebe_gpu_set_table_cache(self.handle, 1 if on else 0))

    def set_check_finite(self, on: bool):
        self._check(self.lib.phoebe_gpu_set_check_finite(self.handle, 1 if on else 0))

    # -- learned proposal ---------------------------------------------------
    def rate_terms(self, sys: DeviceSystem, mesh, params: dict, k_idx, gamma_out, terms,
                   dweights=None, st_row=None, st_band=None, stream=None) -> int:
        c = sys.c_struct()
        m = (ctypes.c_int32 * 3)(*[int(x) for x in mesh])
        p = rate_params(params)
        ns = ctypes.c_int64(0)
        self._check(self.lib.phoebe_gpu_rate_terms(
            self.handle, ctypes.byref(c), m, _ptr(k_idx), int(k_idx.shape[0]), ctypes.byref(p),
            _ptr(gamma_out), _ptr(terms), _ptr(dweights), _ptr(st_row), _ptr(st_band),
            _state_capacity(mesh, sys, terms, dweights, st_row, st_band), ctypes.byref(ns),
            _stream(stream)))
        return int(ns.value)

    def delta_weights(self, sys: DeviceSystem, mesh, params: dict, k_idx, dweights, gamma_scratch,
                      st_row=None, st_band=None, stream=None) -> int:
        c = sys.c_struct()
        m = (ctypes.c_int32 * 3)(*[int(x) for x in mesh])
        p = rate_params(params)
        ns = ctypes.c_int64(0)
        self._check(self.lib.phoebe_gpu_delta_weights(
            self.handle, ctypes.byref(c), m, _ptr(k_idx), int(k_idx.shape[0]), ctypes.byref(p),
            _ptr(dweights), _ptr(st_row), _ptr(st_band),
            _state_capacity(mesh, sys, dweights, None, st_row, st_band), ctypes.byref(ns),
            _ptr(gamma_scratch), _stream(stream)))
        return int(ns.value)

    @staticmethod
    def mlp_param_count(n_in, width, depth) -> int:
        return int(load().phoebe_gpu_mlp_param_count(n_in, width, depth))

    def mlp_forward(self, params, X, out, n_in, width, depth, precision="bf16", stream=None):
        self._check(self.lib.phoebe_gpu_mlp_forward(
            self.handle, PRECISIONS[precision], _ptr(params), n_in, width, depth, _ptr(X),
            int(X.shape[0]), _ptr(out), _stream(stream)))

    def mlp_grad(self, params, X, target, grad, n_in, width, depth, precision="bf16",
                 stream=None) -> float:
        loss = ctypes.c_double(0.0)
        self._check(self.lib.phoebe_gpu_mlp_grad(
            self.handle, PRECISIONS[precision], _ptr(params), n_in, width, depth, _ptr(X),
            _ptr(target), int(X.shape[0]), _ptr(grad), ctypes.byref(loss), _stream(stream)))
        return float(loss.value)

    def mlp_adam(self, params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                 stream=None):
        self._check(self.lib.phoebe_gpu_mlp_adam(
            self.handle, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(params.numel()),
            int(step), lr, beta1, beta2, eps, _stream(stream)))

    @staticmethod
    def mlp_feature_count(n_modes, n_harm=0) -> int:
        return int(load().phoebe_gpu_mlp_feature_count(n_modes, n_harm))

    def mlp_features(self, mesh, n_modes, k_idx, eps, q_idx, nu, X, e0, escale,
                     precision="bf16", n_harm=0, stream=None):
        m = (ctypes.c_int32 * 3)(*[int(x) for x in mesh])
        self._check(self.lib.phoebe_gpu_mlp_features(
            self.handle, PRECISIONS[precision], m, n_modes, n_harm, _ptr(k_idx), _ptr(eps), _ptr(q_idx),
            _ptr(nu), int(k_idx.shape[0]), e0, escale, _ptr(X), _stream(stream)))

    def propose_q(self, mesh, n_modes, k_idx, eps_k, dweights, params, width, depth, e0, escale,
                  d_threshold, mix, S, uniforms, q_off, q_idx, q_w, n_harm=0, stream=None):
        m = (ctypes.c_int32 * 3)(*[int(x) for x in mesh])
        nk = len(k_idx)
        kk = (ctypes.c_int32 * nk)(*[int(x) for x in k_idx])
        ee = (ctypes.c_double * nk)(*[float(x) for x in eps_k])
        self._check(self.lib.phoebe_gpu_propose_q(
            self.handle, m, n_modes, n_harm, kk, ee, nk, _ptr(dweights), _ptr(params), width, depth, e0,
            escale, d_threshold, mix, S, _ptr(uniforms), _ptr(q_off), _ptr(q_idx), _ptr(q_w),
            _stream(stream)))

    # -- batched form -------------------------------------------------------
    def batched_plan(self, systems, meshes, params_list, precision="fp32", tune_cache=None,
                     stream=None) -> "BatchedPlan":
        n = len(systems)
        cs = (CSystem * n)(*[sy.c_struct() for sy in systems])
        m = (ctypes.c_int32 * (3 * n))(*[int(x) for mm in meshes for x in mm])
        ps = (CRateParams * n)(*[rate_params(p) for p in params_list])
        kept = (ctypes.c_int64 * n)()
        plan = ctypes.c_void_p()
        path = tune_cache.encode() if tune_cache else None
        self._check(self.lib.phoebe_gpu_batched_plan(self.handle, cs, n, m, ps,
                                                     PRECISIONS[precision], path,
                                                     ctypes.byref(plan), kept, _stream(stream)))
        return BatchedPlan(self, plan, [int(x) for x in kept], systems)

    # -- timing -------------------------------------------------------------
    MESH_SUM = {"auto": 0, "direct": 1, "factored": 2}

    def set_mesh_sum(self, mode: str):
        """How full-mesh FP64 rate sums run over Rp: "auto", "direct" or "factored"."""
        self._check(self.lib.phoebe_gpu_set_mesh_sum(self.handle, self.MESH_SUM[mode]))

    def set_timing(self, on: bool):
        self._check(self.lib.phoebe_gpu_set_timing(self.handle, 1 if on else 0))

    def reset_timing(self):
        self._check(self.lib.phoebe_gpu_reset_timing(self.handle))

    def kernel_time(self, name: str):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        self._check(self.lib.phoebe_gpu_kernel_time(self.handle, name.encode(), ctypes.byref(n),
                                                    ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    def kernel_bytes(self, name: str) -> float:
        """Algorithmic HBM bytes recorded for the named kernel's timed launches."""
        b = ctypes.c_double(0.0)
        self._check(self.lib.phoebe_gpu_kernel_bytes(self.handle, name.encode(), ctypes.byref(b)))
        return float(b.value)


class BatchedPlan:
    """A captured multi-system plan (see phoebe_gpu_batched_plan)."""

    def __init__(self, lib: Library, plan, n_kept, systems):
        self.lib = lib
        self.plan = plan
        self.n_kept = n_kept
        self._systems = systems  # keeps the device tensors alive

    def run(self, gamma_outs=None, stream=None):
        n = len(self.n_kept)
        arr = None
        if gamma_outs is not None:
            arr = (ctypes.c_void_p * n)(*[_ptr(g) for g in gamma_outs])
        self.lib._check(self.lib.lib.phoebe_gpu_batched_run(self.plan, arr, _stream(stream)))

    def info(self, i):
        tq, tn = ctypes.c_int32(), ctypes.c_int32()
        ns, nt = ctypes.c_int64(), ctypes.c_int64()
        tm = ctypes.c_double()
        self.lib._check(self.lib.lib.phoebe_gpu_batched_info(
            self.plan, i, ctypes.byref(tq), ctypes.byref(tn), ctypes.byref(ns), ctypes.byref(nt),
            ctypes.byref(tm)))
        return dict(tq=tq.value, tn=tn.value, states=ns.value, tasks=nt.value, tune_ms=tm.value)

    def close(self):
        if self.plan:
            self.lib.lib.phoebe_gpu_batched_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
