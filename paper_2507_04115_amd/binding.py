"""ctypes binding of libtdse (include/libtdse.h): same entry points, argument
marshalling only.  Device buffers are torch tensors on the current HIP
device (float64 / int32, contiguous); streams are torch streams.  Every call
raises TDSEError with the library's own message on failure.

The HIP library must be built (``python -m paper_2507_04115_amd.build``);
loading fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdse.so")

TDSE_OK = 0
TDSE_E_INVALID = -1
TDSE_E_NOMEM = -2
TDSE_E_DEVICE = -3
TDSE_E_NOCONV = -4
TDSE_E_UNSUPPORTED = -5
TDSE_E_NONFINITE = -6

TDSE_SYS_OK = 0
TDSE_SYS_NONFINITE = 1
TDSE_SYS_NORM_GROWTH = 2

TDSE_OPT_NONE = 0
TDSE_OPT_PLAIN = 1
TDSE_OPT_NO_GRAPH = 2
TDSE_OPT_AUTOTUNE = 4
TDSE_OPT_STORE_CHECKPOINTS = 8

_lib = None


class TDSEError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what}: {detail} (status {status})")
        self.status = status


class tdse_params(ctypes.Structure):
    _fields_ = [("dx", ctypes.c_double), ("dt", ctypes.c_double), ("a", ctypes.c_double),
                ("charge_z", ctypes.c_double), ("mask_fraction", ctypes.c_double),
                ("mask_power", ctypes.c_double), ("nt", ctypes.c_int32), ("flags", ctypes.c_uint32)]


_vp = ctypes.c_void_p
_d = ctypes.c_double
_i32 = ctypes.c_int32
_PROTOS = {
    "tdse_version": (ctypes.c_char_p, []),
    "tdse_status_string": (ctypes.c_char_p, [_i32]),
    "tdse_last_error": (ctypes.c_char_p, []),
    "tdse_ground_state": (_i32, [ctypes.POINTER(tdse_params), _i32, _d, _i32, _d, _vp,
                                 ctypes.POINTER(_d), _vp]),
    "tdse_ground_state_noalloc": (_i32, [ctypes.POINTER(tdse_params), _i32, _d, _i32, _d, _vp,
                                         ctypes.POINTER(_d), _vp]),
    "tdse_soft_core_for_ip": (_i32, [_d, _i32, _d, _d, _d, _d, _d, ctypes.POINTER(_d),
                                     ctypes.POINTER(_d)]),
    "tdse_plan_create": (_i32, [ctypes.POINTER(tdse_params), _i32, ctypes.POINTER(_i32),
                                ctypes.c_uint32, _i32, ctypes.POINTER(_vp)]),
    "tdse_plan_destroy": (_i32, [_vp]),
    "tdse_plan_psi_offsets": (_i32, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    "tdse_plan_layout": (_i32, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                ctypes.POINTER(_i32)]),
    "tdse_plan_launch_info": (_i32, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                     ctypes.POINTER(_d)]),
    "tdse_plan_ground_state": (_i32, [_vp, _i32, _vp, ctypes.POINTER(_d)]),
    "tdse_set_tune_cache": (_i32, [ctypes.c_char_p]),
    "tdse_plan_graph_state": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "tdse_plan_kernel_info": (_i32, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                     ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                     ctypes.POINTER(_i32)]),
    "tdse_propagate_batch": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tdse_propagate_batch_populations": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _d,
                                                _vp, _vp, _vp]),
    "tdse_adjoint_batch": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tdse_plan_checkpoint_generation": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint64)]),
    "tdse_adjoint_batch_stored": (_i32, [_vp, ctypes.c_uint64, _vp, _vp, _vp, _vp, _vp]),
    "tdse_harmonic_band": (_i32, [_i32, _d, _d, _d, _d, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "tdse_harmonic_yield": (_i32, [_i32, _i32, _d, _d, _d, _d, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tdse_plan_energy_spectrum": (_i32, [_vp, _vp, _i32, _vp, _d, _vp, _vp, ctypes.c_size_t, _vp]),
    "tdse_plan_energy_spectrum_work": (_i32, [_vp, _i32, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "tdse_plan_stored_state": (_i32, [_vp, ctypes.c_uint64, _i32, _vp, _vp]),
    "tdse_plan_populations": (_i32, [_vp, ctypes.c_uint64, _vp, _d, _vp, _vp, _vp]),
    "tdse_gabor": (_i32, [_i32, _i32, _d, _vp, _i32, _vp, _i32, _vp, _d, _vp, _vp]),
    "tdse_energy_integral": (_i32, [_i32, _i32, _vp, _vp, _d, _vp, _vp]),
    "tdse_resample_field": (_i32, [_i32, _i32, _d, _d, _i32, _vp, _vp, ctypes.c_size_t, _vp, _vp]),
    "tdse_band_dft": (_i32, [_i32, _i32, _d, _d, _d, _d, _vp, _vp, _vp]),
    "tdse_band_dft_adjoint": (_i32, [_i32, _i32, _d, _d, _d, _d, _vp, _vp, _vp]),
    "tdse_far_field": (_i32, [_i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp, _d, _vp, _vp]),
    "tdse_far_field_adjoint": (_i32, [_i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp, _d, _vp,
                                      _vp]),
}


def exported_names() -> Sequence[str]:
    return tuple(_PROTOS)


def load(path: str = LIB_PATH):
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtdse is not built: {path} is missing "
                          "(run python -m paper_2507_04115_amd.build)")
    # torch brings its own HIP runtime (same SONAME as ROCm's); loading it
    # first makes libtdse bind to that runtime, so the process has exactly
    # one HIP/HSA runtime and torch buffers and streams are valid here.
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st: int, what: str):
    if st != TDSE_OK:
        detail = load().tdse_last_error().decode()
        raise TDSEError(st, what, detail or load().tdse_status_string(st).decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError("device buffers must be torch tensors")
    if not t.is_cuda:
        raise ValueError("device buffers must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return t.data_ptr()


def _f64(*ts):
    """Raises unless every given tensor is float64 (complex128 for the
    complex arrays is checked by the callers that take them)."""
    import torch

    for t in ts:
        if t is not None and t.dtype != torch.float64:
            raise TypeError(f"expected a float64 tensor, got {t.dtype}")


def _c128(*ts):
    import torch

    for t in ts:
        if t is not None and t.dtype not in (torch.complex128, torch.float64):
            raise TypeError(f"expected a complex128 (or interleaved float64) tensor, got {t.dtype}")


def _cplx_len(t) -> int:
    """Complex elements held by a complex128 tensor or an interleaved float64 one."""
    import torch

    return t.numel() if t.dtype == torch.complex128 else t.numel() // 2


def _need(t, n: int, name: str, complex_: bool = False):
    """Raises ValueError unless tensor t (if given) holds at least n elements
    (complex elements for complex_ buffers) and lives on the current device:
    a short buffer would make the kernels read or write past its end."""
    if t is None:
        return
    import torch

    if isinstance(t, torch.Tensor) and t.is_cuda and t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} lives on {t.device}, the current device is "
                         f"cuda:{torch.cuda.current_device()}")
    have = _cplx_len(t) if complex_ else t.numel()
    if have < n:
        kind = "complex elements" if complex_ else "elements"
        raise ValueError(f"{name} holds {have} {kind}, needs {n}")


def _stream(stream) -> Optional[int]:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def make_params(dx: float, dt: float, a: float, nt: int, charge_z: float = 1.0,
                mask_fraction: float = 0.1, mask_power: float = 0.125) -> tdse_params:
    return tdse_params(dx, dt, a, charge_z, mask_fraction, mask_power, int(nt), 0)


def tdse_set_tune_cache(path: Optional[str]):
    """File of the autotuner's choices across processes (None: none)."""
    _check(load().tdse_set_tune_cache(path.encode() if path else None), "tdse_set_tune_cache")


def tdse_version() -> str:
    return load().tdse_version().decode()


def tdse_ground_state(p: tdse_params, n: int, dtau: float, max_iter: int, tol: float, psi_out,
                      stream=None) -> float:
    _c128(psi_out)
    _need(psi_out, n, "psi_out", True)
    e = _d()
    _check(load().tdse_ground_state(ctypes.byref(p), n, dtau, max_iter, tol, _ptr(psi_out),
                                    ctypes.byref(e), _stream(stream)), "tdse_ground_state")
    return e.value


def tdse_ground_state_noalloc(p: tdse_params, n: int, dtau: float, max_iter: int, tol: float,
                              psi_out, stream=None) -> float:
    """tdse_ground_state without device allocations (static workspace)."""
    _c128(psi_out)
    _need(psi_out, n, "psi_out", True)
    e = _d()
    _check(load().tdse_ground_state_noalloc(ctypes.byref(p), n, dtau, max_iter, tol, _ptr(psi_out),
                                            ctypes.byref(e), _stream(stream)),
           "tdse_ground_state_noalloc")
    return e.value


def tdse_soft_core_for_ip(ip: float, n: int, dx: float, dtau: float = 1.0, tol: float = 1e-13,
                          a_lo: float = 0.5, a_hi: float = 3.0):
    a = _d()
    e = _d()
    _check(load().tdse_soft_core_for_ip(ip, n, dx, dtau, tol, a_lo, a_hi, ctypes.byref(a),
                                        ctypes.byref(e)), "tdse_soft_core_for_ip")
    return a.value, e.value


@dataclass
class Layout:
    points_per_lane: int
    lanes: int
    scan_levels: int


@dataclass
class KernelInfo:
    workgroup_lanes: int
    grid: int
    workgroups_per_cu: int
    lds_bytes: int
    vgprs: int

    @property
    def waves_per_simd(self) -> float:
        return self.workgroups_per_cu * self.workgroup_lanes / 64 / 4


@dataclass
class LaunchInfo:
    systems_per_workgroup: int
    lds_tables: int        # 0 global, 1 om and dV/dx in LDS, 2 om in LDS
    tuned_rate: float


class Plan:
    """Owns a tdse_plan handle (tdse_plan_create / tdse_plan_destroy)."""

    def __init__(self, p: tdse_params, n_per_system: Sequence[int], options: int = 0,
                 adjoint_k: int = 0):
        self.params = p
        self.n_per = [int(v) for v in n_per_system]
        self.batch = len(self.n_per)
        arr = (_i32 * self.batch)(*self.n_per)
        h = _vp()
        _check(load().tdse_plan_create(ctypes.byref(p), self.batch, arr, options, adjoint_k,
                                       ctypes.byref(h)), "tdse_plan_create")
        self.handle = h
        self.options = options
        self.adjoint_k = adjoint_k
        self._offsets = None

    @property
    def nt(self) -> int:
        return int(self.params.nt)

    @property
    def series_len(self) -> int:
        """Elements of a [batch][nt+1] series buffer."""
        return self.batch * (self.nt + 1)

    @property
    def psi_len(self) -> int:
        """Complex elements of a ragged wavefunction buffer."""
        return self.psi_offsets()[-1]

    def close(self):
        if getattr(self, "handle", None):
            _check(load().tdse_plan_destroy(self.handle), "tdse_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def psi_offsets(self):
        if self._offsets is None:
            off = (ctypes.c_int64 * (self.batch + 1))()
            _check(load().tdse_plan_psi_offsets(self.handle, off), "tdse_plan_psi_offsets")
            self._offsets = list(off)
        return list(self._offsets)

    def layout(self, n: int) -> Layout:
        c, t, l = _i32(), _i32(), _i32()
        _check(load().tdse_plan_layout(self.handle, n, ctypes.byref(c), ctypes.byref(t),
                                       ctypes.byref(l)), "tdse_plan_layout")
        return Layout(c.value, t.value, l.value)

    def launch_info(self, n: int) -> LaunchInfo:
        s_, l_, r_ = _i32(), _i32(), _d()
        _check(load().tdse_plan_launch_info(self.handle, n, ctypes.byref(s_), ctypes.byref(l_),
                                            ctypes.byref(r_)), "tdse_plan_launch_info")
        return LaunchInfo(s_.value, int(l_.value), r_.value)

    def graph_state(self) -> int:
        """0 no forward call yet, 1 graph replay, 2 direct launches (capture failed)."""
        v = _i32()
        _check(load().tdse_plan_graph_state(self.handle, ctypes.byref(v)), "tdse_plan_graph_state")
        return v.value

    def kernel_info(self, n: int) -> KernelInfo:
        v = [_i32() for _ in range(5)]
        _check(load().tdse_plan_kernel_info(self.handle, n, *[ctypes.byref(x) for x in v]),
               "tdse_plan_kernel_info")
        return KernelInfo(*[x.value for x in v])

    @property
    def stores_checkpoints(self) -> bool:
        return bool(self.options & TDSE_OPT_STORE_CHECKPOINTS)

    def checkpoint_generation(self) -> int:
        g = ctypes.c_uint64()
        _check(load().tdse_plan_checkpoint_generation(self.handle, ctypes.byref(g)),
               "tdse_plan_checkpoint_generation")
        return g.value

    def ground_state(self, n: int, psi_out) -> float:
        _c128(psi_out)
        _need(psi_out, n, "psi_out", True)
        e = _d()
        _check(load().tdse_plan_ground_state(self.handle, n, _ptr(psi_out), ctypes.byref(e)),
               "tdse_plan_ground_state")
        return e.value


def _i32t(*ts):
    import torch

    for t in ts:
        if t is not None and t.dtype != torch.int32:
            raise TypeError(f"expected an int32 tensor, got {t.dtype}")


def tdse_propagate_batch(plan: Plan, E, psi0, accel, xexp=None, norm=None, psi_final=None,
                         sys_status=None, stream=None):
    _f64(E, accel, xexp, norm)
    _c128(psi0, psi_final)
    _i32t(sys_status)
    for t, nm in ((E, "E"), (accel, "accel"), (xexp, "xexp"), (norm, "norm")):
        _need(t, plan.series_len, nm)
    _need(psi0, plan.psi_len, "psi0", True)
    _need(psi_final, plan.psi_len, "psi_final", True)
    _need(sys_status, plan.batch, "sys_status")
    _check(load().tdse_propagate_batch(plan.handle, _ptr(E), _ptr(psi0), _ptr(accel), _ptr(xexp),
                                       _ptr(norm), _ptr(psi_final), _ptr(sys_status),
                                       _stream(stream)), "tdse_propagate_batch")


def tdse_propagate_batch_populations(plan: Plan, E, psi0, accel, radius: float, gs_pop=None,
                                     vol_pop=None, xexp=None, norm=None, psi_final=None,
                                     sys_status=None, psi_ref=None, stream=None):
    """tdse_propagate_batch plus the ground-state (gs_pop) and volumetric
    (vol_pop, |x| <= radius) populations at every sample."""
    _f64(E, accel, xexp, norm, gs_pop, vol_pop)
    _c128(psi0, psi_final, psi_ref)
    _i32t(sys_status)
    for t, nm in ((E, "E"), (accel, "accel"), (xexp, "xexp"), (norm, "norm"), (gs_pop, "gs_pop"),
                  (vol_pop, "vol_pop")):
        _need(t, plan.series_len, nm)
    for t, nm in ((psi0, "psi0"), (psi_final, "psi_final"), (psi_ref, "psi_ref")):
        _need(t, plan.psi_len, nm, True)
    _need(sys_status, plan.batch, "sys_status")
    _check(load().tdse_propagate_batch_populations(
        plan.handle, _ptr(E), _ptr(psi0), _ptr(accel), _ptr(xexp), _ptr(norm), _ptr(psi_final),
        _ptr(sys_status), _ptr(psi_ref), float(radius), _ptr(gs_pop), _ptr(vol_pop),
        _stream(stream)), "tdse_propagate_batch_populations")


def tdse_adjoint_batch(plan: Plan, E, psi0, accel_bar, grad_E, accel=None, sys_status=None,
                       stream=None):
    _f64(E, accel_bar, grad_E, accel)
    _c128(psi0)
    _i32t(sys_status)
    for t, nm in ((E, "E"), (accel_bar, "accel_bar"), (grad_E, "grad_E"), (accel, "accel")):
        _need(t, plan.series_len, nm)
    _need(psi0, plan.psi_len, "psi0", True)
    _need(sys_status, plan.batch, "sys_status")
    _check(load().tdse_adjoint_batch(plan.handle, _ptr(E), _ptr(psi0), _ptr(accel_bar),
                                     _ptr(grad_E), _ptr(accel), _ptr(sys_status), _stream(stream)),
           "tdse_adjoint_batch")


def tdse_adjoint_batch_stored(plan: Plan, generation: int, E, accel_bar, grad_E, sys_status=None,
                              stream=None):
    _f64(E, accel_bar, grad_E)
    _i32t(sys_status)
    for t, nm in ((E, "E"), (accel_bar, "accel_bar"), (grad_E, "grad_E")):
        _need(t, plan.series_len, nm)
    _need(sys_status, plan.batch, "sys_status")
    _check(load().tdse_adjoint_batch_stored(plan.handle, generation, _ptr(E), _ptr(accel_bar),
                                            _ptr(grad_E), _ptr(sys_status), _stream(stream)),
           "tdse_adjoint_batch_stored")


def tdse_harmonic_band(nt: int, dt: float, omega0: float, h_lo: float, h_hi: float):
    k_lo, nk = _i32(), _i32()
    _check(load().tdse_harmonic_band(nt, dt, omega0, h_lo, h_hi, ctypes.byref(k_lo),
                                     ctypes.byref(nk)), "tdse_harmonic_band")
    return k_lo.value, nk.value


def tdse_harmonic_yield(batch: int, nt: int, dt: float, omega0: float, h_lo: float, h_hi: float,
                        accel, row_weight, work, yield_out, accel_bar=None, stream=None):
    _f64(accel, row_weight, work, yield_out, accel_bar)
    _, nk = tdse_harmonic_band(nt, dt, omega0, h_lo, h_hi)
    _need(accel, batch * (nt + 1), "accel")
    _need(accel_bar, batch * (nt + 1), "accel_bar")
    _need(row_weight, batch, "row_weight")
    _need(yield_out, batch, "yield_out")
    _need(work, 2 * batch * max(nk, 1), "work")
    _check(load().tdse_harmonic_yield(batch, nt, dt, omega0, h_lo, h_hi, _ptr(accel),
                                      _ptr(row_weight), _ptr(work), _ptr(yield_out),
                                      _ptr(accel_bar), _stream(stream)), "tdse_harmonic_yield")


def tdse_band_dft(batch: int, nt: int, dt: float, omega0: float, h_lo: float, h_hi: float, accel,
                  amp, stream=None):
    _f64(accel)
    _c128(amp)
    _, nk = tdse_harmonic_band(nt, dt, omega0, h_lo, h_hi)
    _need(accel, batch * (nt + 1), "accel")
    _need(amp, batch * nk, "amp", True)
    _check(load().tdse_band_dft(batch, nt, dt, omega0, h_lo, h_hi, _ptr(accel), _ptr(amp),
                                _stream(stream)), "tdse_band_dft")


def tdse_band_dft_adjoint(batch: int, nt: int, dt: float, omega0: float, h_lo: float, h_hi: float,
                          amp_bar, accel_bar, stream=None):
    _c128(amp_bar)
    _f64(accel_bar)
    _, nk = tdse_harmonic_band(nt, dt, omega0, h_lo, h_hi)
    _need(amp_bar, batch * nk, "amp_bar", True)
    _need(accel_bar, batch * (nt + 1), "accel_bar")
    _check(load().tdse_band_dft_adjoint(batch, nt, dt, omega0, h_lo, h_hi, _ptr(amp_bar),
                                        _ptr(accel_bar), _stream(stream)), "tdse_band_dft_adjoint")


def tdse_far_field(rho_src, z_src, weights, kwave, amp, rho_obs, z_obs: float, field, stream=None,
                   adjoint: bool = False):
    """field = far field of amp (adjoint=False), or amp_bar from field_bar
    (adjoint=True: `amp` is field_bar, `field` receives amp_bar)."""
    _f64(rho_src, z_src, weights, kwave, rho_obs)
    _c128(amp, field)
    nsrc, nk, nobs = int(rho_src.numel()) * int(z_src.numel()), int(kwave.numel()), int(rho_obs.numel())
    _need(weights, nsrc, "weights")
    _need(amp, (nobs if adjoint else nsrc) * nk, "field_bar" if adjoint else "amp", True)
    _need(field, (nsrc if adjoint else nobs) * nk, "amp_bar" if adjoint else "field", True)
    fn = load().tdse_far_field_adjoint if adjoint else load().tdse_far_field
    _check(fn(int(rho_src.numel()), int(z_src.numel()), _ptr(rho_src), _ptr(z_src), _ptr(weights),
              int(kwave.numel()), _ptr(kwave), _ptr(amp), int(rho_obs.numel()), _ptr(rho_obs),
              float(z_obs), _ptr(field), _stream(stream)),
           "tdse_far_field_adjoint" if adjoint else "tdse_far_field")


def tdse_plan_energy_spectrum(plan: Plan, psi, energies, eps: float, spectrum, work, stream=None):
    """spectrum[b][e] = electron energy distribution of psi_b at energies[e]
    (work: a device scratch tensor, its byte size is passed along)."""
    _f64(energies, spectrum)
    _c128(psi)
    _need(psi, plan.psi_len, "psi", True)
    _need(spectrum, plan.batch * int(energies.numel()), "spectrum")
    _check(load().tdse_plan_energy_spectrum(plan.handle, _ptr(psi), int(energies.numel()),
                                            _ptr(energies), float(eps), _ptr(spectrum), _ptr(work),
                                            work.numel() * work.element_size(), _stream(stream)),
           "tdse_plan_energy_spectrum")


def tdse_plan_energy_spectrum_work(plan: Plan, n_energy: int, lanes: int = 65536) -> int:
    """Bytes of work tdse_plan_energy_spectrum needs with `lanes` solves in flight."""
    b = ctypes.c_size_t()
    _check(load().tdse_plan_energy_spectrum_work(plan.handle, int(n_energy), int(lanes),
                                                 ctypes.byref(b)), "tdse_plan_energy_spectrum_work")
    return b.value


def tdse_gabor(accel, dt: float, t_centres, omegas, sigma: float, out, stream=None):
    """out[b][c][w] = Gabor transform of accel rows (see include/libtdse.h)."""
    _f64(accel, t_centres, omegas, out)
    batch, n1 = accel.shape
    _need(out, batch * int(t_centres.numel()) * int(omegas.numel()), "out")
    _check(load().tdse_gabor(batch, n1 - 1, float(dt), _ptr(accel), int(t_centres.numel()),
                             _ptr(t_centres), int(omegas.numel()), _ptr(omegas), float(sigma),
                             _ptr(out), _stream(stream)), "tdse_gabor")


def tdse_energy_integral(energies, spectrum, e_lo: float, out, stream=None):
    """out[b] = trapezoid integral of spectrum[b] over the grid points E >= e_lo
    (e_lo = 0: the ionisation probability); see include/libtdse.h."""
    _f64(energies, spectrum, out)
    n_e = int(energies.numel())
    batch = int(out.numel())
    _need(spectrum, batch * n_e, "spectrum")
    _check(load().tdse_energy_integral(batch, n_e, _ptr(energies), _ptr(spectrum), float(e_lo),
                                       _ptr(out), _stream(stream)), "tdse_energy_integral")


def tdse_plan_stored_state(plan: Plan, generation: int, index: int, psi_out, stream=None):
    _c128(psi_out)
    _need(psi_out, plan.psi_len, "psi_out", True)
    _check(load().tdse_plan_stored_state(plan.handle, generation, index, _ptr(psi_out),
                                         _stream(stream)), "tdse_plan_stored_state")


def tdse_plan_populations(plan: Plan, generation: int, radius: float, gs=None, vol=None,
                          psi_ref=None, stream=None):
    """gs[b][s], vol[b][s]: ground-state and volumetric populations of every
    stored state (s = 0 .. nt // adjoint_k); see include/libtdse.h."""
    _f64(gs, vol)
    _c128(psi_ref)
    need = plan.batch * (plan.params.nt // max(plan.adjoint_k, 1) + 1)
    for t in (gs, vol):
        if t is not None and t.numel() < need:
            raise ValueError(f"population outputs need {need} elements")
    _check(load().tdse_plan_populations(plan.handle, generation, _ptr(psi_ref), float(radius),
                                        _ptr(gs), _ptr(vol), _stream(stream)),
           "tdse_plan_populations")


def tdse_resample_field(e_coarse, dt_coarse: float, dt: float, nt: int, e_fine=None, work=None,
                        stream=None):
    """e_fine [P, nt+1] = the coarse rows e_coarse [P, M] interpolated to dt by
    Fourier zero-padding (see include/libtdse.h).  e_fine and work are
    allocated when not given."""
    import torch

    _f64(e_coarse, e_fine, work)
    if e_coarse.dim() == 1:
        e_coarse = e_coarse[None, :]
    batch, m = e_coarse.shape
    if e_fine is None:
        e_fine = torch.empty(batch, nt + 1, dtype=torch.float64, device=e_coarse.device)
    if work is None:
        work = torch.empty(2 * batch * (m // 2 + 1), dtype=torch.float64, device=e_coarse.device)
    _need(e_coarse, batch * m, "e_coarse")
    _need(e_fine, batch * (nt + 1), "e_fine")
    _need(work, 2 * batch * (m // 2 + 1), "work")
    _check(load().tdse_resample_field(batch, m, float(dt_coarse), float(dt), int(nt), _ptr(e_coarse),
                                      _ptr(work), work.numel() * work.element_size(), _ptr(e_fine),
                                      _stream(stream)), "tdse_resample_field")
    return e_fine
