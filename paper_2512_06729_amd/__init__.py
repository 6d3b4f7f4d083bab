"""Thin Python binding of libxod (the HIP implicit column solver).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  Device buffers are torch tensors (their data_ptr() is passed to
the C ABI); host inputs are numpy arrays copied by the library at create
time.  The names follow include/xod.h.

If libxod.so is missing, importing this package raises: there is no CPU
fallback.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxod.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "xod.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python paper_2512_06729_amd/build.py` "
        "(there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

c_int32 = ctypes.c_int32
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
P_int = ctypes.POINTER(ctypes.c_int32)
P_dbl = ctypes.POINTER(ctypes.c_double)

XOD_OK, XOD_EINVAL, XOD_ENOMEM, XOD_ESINGULAR, XOD_ENOTCONVERGED, \
    XOD_ENONFINITE, XOD_EHIP, XOD_ENOTIMPL, XOD_EBUSY = range(9)
STATUS_NAMES = ["OK", "EINVAL", "ENOMEM", "ESINGULAR", "ENOTCONVERGED",
                "ENONFINITE", "EHIP", "ENOTIMPL", "EBUSY"]
XOD_FP64, XOD_MIXED = 0, 1
XOD_SOLVER_THOMAS, XOD_SOLVER_CR = 0, 1


class XodError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"XOD_{name}: {message}")


class NetworkDesc(ctypes.Structure):
    _fields_ = [("S", c_int32), ("R", c_int32), ("E", c_int32),
                ("elem_comp", P_int), ("mass_amu", P_dbl), ("nasa7", P_dbl),
                ("t_mid", c_double), ("rtype", P_int), ("reac", P_int),
                ("prod", P_int), ("reversible", P_int), ("tb_kooij", P_int),
                ("params", P_dbl)]


class Profile(ctypes.Structure):
    _fields_ = [("N", c_int32), ("P_bar", P_dbl), ("T_K", P_dbl), ("Kzz", P_dbl),
                ("Dmol", P_dbl), ("alphaT", P_dbl), ("mbar_amu", c_double),
                ("g_cgs", c_double), ("sigma_tau", c_double)]


class Boundary(ctypes.Structure):
    _fields_ = [("escape_diff_limited", ctypes.POINTER(c_int32)),
                ("v_top", ctypes.POINTER(c_double)),
                ("v_dep", ctypes.POINTER(c_double)),
                ("phi_surf", ctypes.POINTER(c_double))]


class StepStats(ctypes.Structure):
    _fields_ = [("max_rel_change", c_double), ("min_ratio", c_double),
                ("resid_inf", c_double), ("refine_iters", c_int32),
                ("fp64_fallback", c_int32), ("nonfinite", c_int32), ("pad_", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class SSOpts(ctypes.Structure):
    _fields_ = [("tol_rel", c_double), ("y_floor", c_double), ("y_sig", c_double),
                ("t_end", c_double), ("dt0", c_double), ("max_steps", c_int32),
                ("max_consec_rejects", c_int32), ("use_mix_rule", c_int32),
                ("method", c_int32), ("y_neg", c_double)]


class ReuseStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("factorizations", ctypes.c_int64),
                ("newton_iters", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ParcelStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("rejects", ctypes.c_int64), ("clipped", c_double),
                ("visits", c_int32), ("pad_", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class TuneResult(ctypes.Structure):
    _fields_ = [("key", ctypes.c_char * 96), ("candidates", c_int32),
                ("fused_max_ld", c_int32), ("outer", c_int32), ("update32", c_int32),
                ("gemm_large", c_int32), ("gemm_k", c_int32), ("panel_sync", c_int32),
                ("gemm_waves", c_int32), ("best_ms", c_double), ("default_ms", c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["key"] = self.key.decode()
        return d


class SSResult(ctypes.Structure):
    _fields_ = [("t", c_double), ("dt", c_double), ("clipped", c_double),
                ("steps", ctypes.c_int64), ("rejects", ctypes.c_int64),
                ("converged", c_int32), ("factorizations", c_int32),
                ("newton_iters", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _sig(name, *args):
    f = getattr(_lib, name)
    f.restype = c_int32
    f.argtypes = list(args)
    return f


_f = {
    "xod_network_create": _sig("xod_network_create", ctypes.POINTER(NetworkDesc), ctypes.POINTER(c_void_p)),
    "xod_network_destroy": _sig("xod_network_destroy", c_void_p),
    "xod_network_sizes": _sig("xod_network_sizes", c_void_p, P_int, P_int, P_int),
    "xod_column_create": _sig("xod_column_create", c_void_p, ctypes.POINTER(Profile), P_dbl,
                              c_int32, c_void_p, ctypes.POINTER(c_void_p)),
    "xod_column_destroy": _sig("xod_column_destroy", c_void_p),
    "xod_column_get_state": _sig("xod_column_get_state", c_void_p, P_dbl, P_dbl, P_dbl),
    "xod_column_set_state": _sig("xod_column_set_state", c_void_p, P_dbl, c_double, c_double),
    "xod_column_state_ptr": _sig("xod_column_state_ptr", c_void_p, ctypes.POINTER(c_void_p)),
    "xod_column_grid": _sig("xod_column_grid", c_void_p, P_dbl, P_dbl, P_dbl, P_dbl),
    "xod_column_set_solver": _sig("xod_column_set_solver", c_void_p, c_int32),
    "xod_rates": _sig("xod_rates", c_void_p, c_void_p, c_void_p),
    "xod_rhs": _sig("xod_rhs", c_void_p, c_void_p, c_void_p, c_void_p, c_void_p),
    "xod_jacobian": _sig("xod_jacobian", c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                         c_void_p, c_void_p, c_void_p, c_int32),
    "xod_btd_factor": _sig("xod_btd_factor", c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                           c_void_p, c_int32),
    "xod_btd_solve": _sig("xod_btd_solve", c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                          c_void_p, c_void_p, c_int32),
    "xod_btd_solve_info": _sig("xod_btd_solve_info", c_void_p, P_int, P_int, P_dbl),
    "xod_step": _sig("xod_step", c_void_p, c_double, ctypes.POINTER(StepStats)),
    "xod_step_frozen": _sig("xod_step_frozen", c_void_p, c_double, ctypes.POINTER(StepStats)),
    "xod_step_ros2": _sig("xod_step_ros2", c_void_p, c_double, ctypes.POINTER(StepStats)),
    "xod_step_bdf2": _sig("xod_step_bdf2", c_void_p, c_double, ctypes.POINTER(StepStats)),
    "xod_step_newton": _sig("xod_step_newton", c_void_p, c_double, c_int32,
                            ctypes.POINTER(StepStats)),
    "xod_column_set_boundary": _sig("xod_column_set_boundary", c_void_p,
                                    ctypes.POINTER(Boundary)),
    "xod_integrate_to_steady_state": _sig("xod_integrate_to_steady_state", c_void_p,
                                          ctypes.POINTER(SSOpts), ctypes.POINTER(SSResult)),
    "xod_last_error": _sig("xod_last_error", ctypes.c_char_p, ctypes.c_size_t),
    "xod_parcel_pass": _sig("xod_parcel_pass", c_void_p, c_double, P_dbl,
                            ctypes.POINTER(ParcelStats)),
    "xod_integrate_fixed_dt": _sig("xod_integrate_fixed_dt", c_void_p, c_double, c_int32,
                                   c_int32, ctypes.POINTER(ReuseStats)),
    "xod_set_option": _sig("xod_set_option", ctypes.c_char_p, ctypes.c_int64),
    "xod_column_set_photolysis_spectrum": _sig("xod_column_set_photolysis_spectrum", c_void_p,
                                               ctypes.c_int32, ctypes.c_int32, c_void_p,
                                               c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                               c_double),
    "xod_photolysis_spectral": _sig("xod_photolysis_spectral", ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, c_void_p,
                                    c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_double, c_double, c_void_p, ctypes.c_size_t, c_void_p,
                                    c_void_p),
    "xod_photolysis_spectral_noalloc": _sig("xod_photolysis_spectral_noalloc", ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, c_void_p, c_void_p, c_void_p,
                                            c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                            c_double, c_void_p, c_void_p),
    "xod_get_option": _sig("xod_get_option", ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)),
    "xod_batch_create": _sig("xod_batch_create", ctypes.POINTER(c_void_p), c_int32,
                             ctypes.POINTER(c_void_p)),
    "xod_batch_destroy": _sig("xod_batch_destroy", c_void_p),
    "xod_batch_step": _sig("xod_batch_step", c_void_p, P_dbl, ctypes.POINTER(StepStats)),
    "xod_autotune": _sig("xod_autotune", c_void_p, c_double, c_int32, ctypes.POINTER(TuneResult)),
    "xod_batch_autotune": _sig("xod_batch_autotune", c_void_p, P_dbl, c_int32,
                               ctypes.POINTER(TuneResult), c_int32, ctypes.POINTER(c_int32)),
    "xod_autotune_clear": _sig("xod_autotune_clear"),
    "xod_profile_read": _sig("xod_profile_read", ctypes.c_char_p, P_dbl,
                             ctypes.POINTER(ctypes.c_int64)),
    "xod_profile_reset": _sig("xod_profile_reset"),
    "xod_serve_create": _sig("xod_serve_create", ctypes.c_size_t, c_int32, c_int32, c_void_p,
                             ctypes.POINTER(c_void_p)),
    "xod_serve_destroy": _sig("xod_serve_destroy", c_void_p),
    "xod_serve_set_solver": _sig("xod_serve_set_solver", c_void_p, c_int32),
    "xod_serve_footprint": _sig("xod_serve_footprint", c_void_p, c_int32, c_int32,
                                ctypes.POINTER(ctypes.c_size_t)),
    "xod_serve_submit": _sig("xod_serve_submit", c_void_p, c_void_p, ctypes.POINTER(Profile),
                             P_dbl, ctypes.POINTER(SSOpts), ctypes.POINTER(ctypes.c_uint64)),
    "xod_serve_step": _sig("xod_serve_step", c_void_p, P_int, P_int),
    "xod_serve_poll": _sig("xod_serve_poll", c_void_p, ctypes.c_uint64, P_int, P_dbl,
                           ctypes.POINTER(SSResult), P_dbl),
    "xod_serve_release": _sig("xod_serve_release", c_void_p, ctypes.c_uint64),
    "xod_serve_usage": _sig("xod_serve_usage", c_void_p, ctypes.POINTER(ctypes.c_size_t), P_int,
                            P_int, ctypes.POINTER(ctypes.c_int64)),
}


def profile_read(kernel):
    """(total milliseconds, launch count) of one profiled kernel kind."""
    ms, n = c_double(), ctypes.c_int64()
    _check(_f["xod_profile_read"](kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def profile_reset():
    _check(_f["xod_profile_reset"]())


def header_symbols(path=HEADER):
    """Function names declared in include/xod.h."""
    text = open(path).read()
    return sorted(set(re.findall(r"\b(xod_[a-z0-9_]+)\s*\(", text)))


def last_error():
    buf = ctypes.create_string_buffer(1024)
    _f["xod_last_error"](buf, 1024)
    return buf.value.decode(errors="replace")


def _check(status):
    if status != XOD_OK:
        raise XodError(status, last_error())


def set_option(name, value):
    _check(_f["xod_set_option"](name.encode(), int(value)))


_lib.xod_photolysis_workspace.restype = ctypes.c_size_t
_lib.xod_photolysis_workspace.argtypes = [ctypes.c_int32] * 4


def photolysis_workspace(N, A, L, P):
    """Bytes of device scratch xod_photolysis_spectral needs."""
    return int(_lib.xod_photolysis_workspace(int(N), int(A), int(L), int(P)))


def photolysis_spectral(n, dz, absorbers, sig_ext, J0, dlam, sig_ph, kph, work, t_f=1.0,
                        mu=1.0, stream=None):
    """Spectral photolysis rate coefficients into kph [N, P] (device tensors;
    n [N, S], dz [N], absorbers [A] int32, sig_ext [A, L], J0 [L], dlam [L],
    sig_ph [P, L], work a device byte buffer of photolysis_workspace() bytes)."""
    N, S = n.shape
    A = absorbers.shape[0]
    L = J0.shape[0]
    P = sig_ph.shape[0]
    _check(_f["xod_photolysis_spectral"](
        N, S, A, L, P, _dev(n), _dev(dz), _dev(absorbers) if A else None,
        _dev(sig_ext) if A else None, _dev(J0), _dev(dlam), _dev(sig_ph) if P else None,
        float(t_f), float(mu), _dev(work), work.numel() * work.element_size(),
        _dev(kph) if P else None, stream))


def photolysis_spectral_noalloc(n, dz, absorbers, sig_ext, J0, dlam, sig_ph, kph, t_f=1.0,
                                mu=1.0, stream=None):
    """photolysis_spectral without a workspace: the library's fixed device
    array serves instead (xod_photolysis_spectral_noalloc; no allocation)."""
    N, S = n.shape
    A = absorbers.shape[0]
    L = J0.shape[0]
    P = sig_ph.shape[0]
    _check(_f["xod_photolysis_spectral_noalloc"](
        N, S, A, L, P, _dev(n), _dev(dz), _dev(absorbers) if A else None,
        _dev(sig_ext) if A else None, _dev(J0), _dev(dlam), _dev(sig_ph) if P else None,
        float(t_f), float(mu), _dev(kph) if P else None, stream))


def get_option(name):
    v = ctypes.c_int64()
    _check(_f["xod_get_option"](name.encode(), ctypes.byref(v)))
    return v.value


def _ptr(arr, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def _dev(t):
    """Device pointer of a torch tensor (the library never frees it)."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return c_void_p(t.data_ptr())


class Network:
    """Device-resident reaction network (xod_network)."""

    def __init__(self, net):
        self._keep = dict(
            elem_comp=np.ascontiguousarray(net.elem_comp, np.int32),
            mass=np.ascontiguousarray(net.mass_amu, np.float64),
            nasa7=np.ascontiguousarray(net.nasa7, np.float64),
            rtype=np.ascontiguousarray(net.rtype, np.int32),
            reac=np.ascontiguousarray(net.reac, np.int32),
            prod=np.ascontiguousarray(net.prod, np.int32),
            rev=np.ascontiguousarray(net.reversible, np.int32),
            kooij=np.ascontiguousarray(net.tb_kooij, np.int32),
            params=np.ascontiguousarray(net.params, np.float64))
        k = self._keep
        S = k["mass"].shape[0]
        R = k["rtype"].shape[0]
        E = k["elem_comp"].shape[0]
        d = NetworkDesc(S, R, E, _ptr(k["elem_comp"], c_int32), _ptr(k["mass"], c_double),
                        _ptr(k["nasa7"], c_double), float(net.t_mid),
                        _ptr(k["rtype"], c_int32), _ptr(k["reac"], c_int32),
                        _ptr(k["prod"], c_int32), _ptr(k["rev"], c_int32),
                        _ptr(k["kooij"], c_int32), _ptr(k["params"], c_double))
        h = c_void_p()
        _check(_f["xod_network_create"](ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        S_, R_, ld = c_int32(), c_int32(), c_int32()
        _check(_f["xod_network_sizes"](h, ctypes.byref(S_), ctypes.byref(R_), ctypes.byref(ld)))
        self.S, self.R, self.ld = S_.value, R_.value, ld.value

    def close(self):
        if getattr(self, "handle", None):
            _f["xod_network_destroy"](self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Column:
    """One atmospheric column (xod_column): device state + workspace."""

    def __init__(self, network, col, precision=XOD_FP64, stream=None, n0=None,
                 solver=XOD_SOLVER_THOMAS):
        self.network = network
        N = int(np.asarray(col.P_bar).shape[0])
        S = network.S
        self.N, self.S, self.R, self.ld = N, S, network.R, network.ld
        self._keep = dict(P=np.ascontiguousarray(col.P_bar, np.float64),
                          T=np.ascontiguousarray(col.T_K, np.float64),
                          K=np.ascontiguousarray(col.Kzz, np.float64))
        k = self._keep
        if col.Dmol is not None:
            k["D"] = np.ascontiguousarray(col.Dmol, np.float64)
        if col.alphaT is not None:
            k["alpha"] = np.ascontiguousarray(col.alphaT, np.float64)
        prof = Profile(N, _ptr(k["P"], c_double), _ptr(k["T"], c_double), _ptr(k["K"], c_double),
                       _ptr(k["D"], c_double) if "D" in k else None,
                       _ptr(k["alpha"], c_double) if "alpha" in k else None,
                       float(col.mbar_amu), float(col.g_cgs), float(col.sigma_tau))
        n0 = np.ascontiguousarray(col.n0 if n0 is None else n0, np.float64)
        if n0.shape != (N, S):
            raise ValueError(f"n0 must have shape {(N, S)}")
        h = c_void_p()
        _check(_f["xod_column_create"](network.handle, ctypes.byref(prof), _ptr(n0, c_double),
                                       int(precision), c_void_p(stream or 0), ctypes.byref(h)))
        self.handle = h
        if solver != XOD_SOLVER_THOMAS:
            self.set_solver(solver)
        bnd = {name: getattr(col, name, None)
               for name in ("escape_diff_limited", "v_top", "v_dep", "phi_surf")}
        if any(v is not None for v in bnd.values()):
            self.set_boundary(**bnd)

    def set_boundary(self, escape_diff_limited=None, v_top=None, v_dep=None, phi_surf=None):
        """Open the column's ends (xod_column_set_boundary); all None closes them."""
        S = self.S
        keep = {}

        def arr(name, v, dtype, ctype):
            if v is None:
                return None
            a = np.ascontiguousarray(v, dtype)
            if a.shape != (S,):
                raise ValueError(f"{name} must have shape ({S},)")
            keep[name] = a
            return _ptr(a, ctype)

        b = Boundary(arr("escape_diff_limited", escape_diff_limited, np.int32, c_int32),
                     arr("v_top", v_top, np.float64, c_double),
                     arr("v_dep", v_dep, np.float64, c_double),
                     arr("phi_surf", phi_surf, np.float64, c_double))
        _check(_f["xod_column_set_boundary"](self.handle, ctypes.byref(b)))

    def set_solver(self, solver):
        """XOD_SOLVER_THOMAS or XOD_SOLVER_CR (xod_column_set_solver)."""
        _check(_f["xod_column_set_solver"](self.handle, int(solver)))

    def state(self):
        n = np.empty((self.N, self.S))
        t, dt = c_double(), c_double()
        _check(_f["xod_column_get_state"](self.handle, _ptr(n, c_double), ctypes.byref(t),
                                          ctypes.byref(dt)))
        return n

    def set_state(self, n, t=0.0, dt=0.0):
        n = np.ascontiguousarray(n, np.float64)
        _check(_f["xod_column_set_state"](self.handle, _ptr(n, c_double), t, dt))

    def grid(self):
        ng, tau, dz = np.empty(self.N), np.empty(self.N), np.empty(self.N)
        mix = c_double()
        _check(_f["xod_column_grid"](self.handle, _ptr(ng, c_double), _ptr(tau, c_double),
                                     _ptr(dz, c_double), ctypes.byref(mix)))
        return dict(ngas=ng, tau=tau, dz=dz, mix_time=mix.value)

    def set_photolysis_spectrum(self, absorbers=None, sig_ext=None, J0=None, dlam=None,
                                sig_ph=None, t_f=1.0, mu=1.0):
        """Spectral photolysis in this column's steps (device tensors, kept
        referenced here while in force); no J0: back to the gray law."""
        if J0 is None:
            _check(_f["xod_column_set_photolysis_spectrum"](self.handle, 0, 0, None, None, None,
                                                             None, None, 1.0, 1.0))
            self._spectrum = None
            return
        A = 0 if absorbers is None else absorbers.shape[0]
        L = J0.shape[0]
        _check(_f["xod_column_set_photolysis_spectrum"](
            self.handle, A, L, _dev(absorbers) if A else None, _dev(sig_ext) if A else None,
            _dev(J0), _dev(dlam), _dev(sig_ph) if sig_ph is not None and sig_ph.numel() else None,
            float(t_f), float(mu)))
        self._spectrum = (absorbers, sig_ext, J0, dlam, sig_ph)

    def close(self):
        if getattr(self, "handle", None):
            _f["xod_column_destroy"](self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- hot-path calls (torch device tensors) --------------------------------

def xod_rates(col, kf, kr):
    _check(_f["xod_rates"](col.handle, _dev(kf), _dev(kr)))


def xod_rhs(col, kf, kr, n, f):
    _check(_f["xod_rhs"](col.handle, _dev(kf), _dev(kr), _dev(n), _dev(f)))


def xod_jacobian(col, kf, kr, n, dt, B, a, c):
    _check(_f["xod_jacobian"](col.handle, _dev(kf), _dev(kr), _dev(n), float(dt), _dev(B),
                              _dev(a), _dev(c), col.ld))


def xod_btd_factor(col, B, a, c, piv, precision=XOD_FP64):
    _check(_f["xod_btd_factor"](col.handle, _dev(B), _dev(a), _dev(c), col.ld,
                                _dev(piv) if piv is not None else None, int(precision)))


def xod_btd_solve(col, B, a, c, piv, rhs, max_refine=10):
    _check(_f["xod_btd_solve"](col.handle, _dev(B), _dev(a), _dev(c), col.ld,
                               _dev(piv) if piv is not None else None, _dev(rhs),
                               int(max_refine)))


def xod_btd_solve_info(col):
    """(refinements, FP64 fallback, last correction size) of the last solve."""
    it, fb, size = c_int32(), c_int32(), c_double()
    _check(_f["xod_btd_solve_info"](col.handle, ctypes.byref(it), ctypes.byref(fb),
                                    ctypes.byref(size)))
    return it.value, fb.value, size.value


def xod_step(col, dt):
    st = StepStats()
    _check(_f["xod_step"](col.handle, float(dt), ctypes.byref(st)))
    return st.as_dict()


def xod_step_frozen(col, dt):
    """A step reusing the factorisation of the last xod_step (same dt)."""
    st = StepStats()
    _check(_f["xod_step_frozen"](col.handle, float(dt), ctypes.byref(st)))
    return st.as_dict()


def xod_step_ros2(col, dt):
    """One two-stage Rosenbrock (ROS2) step: one factorisation, two solves."""
    st = StepStats()
    _check(_f["xod_step_ros2"](col.handle, float(dt), ctypes.byref(st)))
    return st.as_dict()


def xod_step_newton(col, dt, iters):
    """Backward Euler by modified Newton: iters - 1 corrections on one factorisation."""
    st = StepStats()
    _check(_f["xod_step_newton"](col.handle, float(dt), int(iters), ctypes.byref(st)))
    return st.as_dict()


def xod_step_bdf2(col, dt):
    """One variable-step BDF2 step; its history is the previous step's start."""
    st = StepStats()
    _check(_f["xod_step_bdf2"](col.handle, float(dt), ctypes.byref(st)))
    return st.as_dict()


def xod_integrate_to_steady_state(col, tol_rel=0.0, y_floor=0.0, y_sig=0.0, t_end=0.0,
                                  dt0=0.0, max_steps=0, max_consec_rejects=0,
                                  use_mix_rule=1, check=True, method=0, y_neg=0.0):
    """method 0: backward-Euler steps, 1: ROS2 steps, 2: backward-Euler steps
    on step matrices kept across steps (1 and 2: FP64 columns)."""
    o = SSOpts(tol_rel, y_floor, y_sig, t_end, dt0, max_steps, max_consec_rejects,
               use_mix_rule, method, y_neg)
    r = SSResult()
    st = _f["xod_integrate_to_steady_state"](col.handle, ctypes.byref(o), ctypes.byref(r))
    if check and st not in (XOD_OK,):
        raise XodError(st, last_error())
    out = r.as_dict()
    out["status"] = st
    return out


def xod_parcel_pass(col, dt0=1e-8):
    """One bottom-to-top-to-bottom pass of the Lagrangian parcel over the
    column's profile (its state, updated in place); returns the statistics
    and the step size the last visit ended on."""
    st = ParcelStats()
    dt_last = c_double()
    _check(_f["xod_parcel_pass"](col.handle, float(dt0), ctypes.byref(dt_last),
                                 ctypes.byref(st)))
    out = st.as_dict()
    out["dt_last"] = dt_last.value
    return out


def xod_autotune(col, dt, trials=3):
    """Tile settings for columns like col (xod_autotune)."""
    r = TuneResult()
    _check(_f["xod_autotune"](col.handle, float(dt), int(trials), ctypes.byref(r)))
    return r.as_dict()


def xod_autotune_clear():
    _check(_f["xod_autotune_clear"]())


def xod_integrate_fixed_dt(col, dt, nsteps, reuse=1):
    """nsteps backward-Euler steps of size dt, keeping the step matrix across
    steps (modified Newton) when reuse = 1; returns the step statistics."""
    st = ReuseStats()
    _check(_f["xod_integrate_fixed_dt"](col.handle, float(dt), int(nsteps), int(reuse),
                                        ctypes.byref(st)))
    return st.as_dict()


class Batch:
    """Columns stepped together (xod_batch)."""

    def __init__(self, columns):
        self.columns = list(columns)
        arr = (c_void_p * len(self.columns))(*[c.handle for c in self.columns])
        h = c_void_p()
        _check(_f["xod_batch_create"](arr, len(self.columns), ctypes.byref(h)))
        self.handle = h

    def step(self, dts):
        dts = np.ascontiguousarray(dts, np.float64)
        stats = (StepStats * len(self.columns))()
        _check(_f["xod_batch_step"](self.handle, _ptr(dts, c_double), stats))
        return [s.as_dict() for s in stats]

    def autotune(self, dts, trials=2):
        """Tile settings per group of this batch (xod_batch_autotune)."""
        dts = np.ascontiguousarray(dts, np.float64)
        res = (TuneResult * 16)()
        n = c_int32()
        _check(_f["xod_batch_autotune"](self.handle, _ptr(dts, c_double), int(trials), res, 16,
                                        ctypes.byref(n)))
        return [res[i].as_dict() for i in range(n.value)]

    def close(self):
        if getattr(self, "handle", None):
            _f["xod_batch_destroy"](self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _profile_struct(col, N):
    keep = dict(P=np.ascontiguousarray(col.P_bar, np.float64),
                T=np.ascontiguousarray(col.T_K, np.float64),
                K=np.ascontiguousarray(col.Kzz, np.float64))
    if col.Dmol is not None:
        keep["D"] = np.ascontiguousarray(col.Dmol, np.float64)
    if col.alphaT is not None:
        keep["alpha"] = np.ascontiguousarray(col.alphaT, np.float64)
    prof = Profile(N, _ptr(keep["P"], c_double), _ptr(keep["T"], c_double),
                   _ptr(keep["K"], c_double),
                   _ptr(keep["D"], c_double) if "D" in keep else None,
                   _ptr(keep["alpha"], c_double) if "alpha" in keep else None,
                   float(col.mbar_amu), float(col.g_cgs), float(col.sigma_tau))
    return prof, keep


class Server:
    """Continuous-batching steady-state solver (xod_server)."""

    QUEUED, RUNNING, DONE, FAILED = 0, 1, 2, 3

    def __init__(self, hbm_budget_bytes, max_slots, precision=XOD_FP64, stream=None,
                 solver=XOD_SOLVER_CR):
        h = c_void_p()
        _check(_f["xod_serve_create"](int(hbm_budget_bytes), int(max_slots), int(precision),
                                      c_void_p(stream or 0), ctypes.byref(h)))
        self.handle = h
        self.precision = precision
        if solver != XOD_SOLVER_CR:
            _check(_f["xod_serve_set_solver"](h, int(solver)))
        self._shapes = {}

    @staticmethod
    def footprint(network, N, precision=XOD_FP64):
        b = ctypes.c_size_t()
        _check(_f["xod_serve_footprint"](network.handle, int(N), int(precision), ctypes.byref(b)))
        return b.value

    def submit(self, network, col, tol_rel=0.0, y_floor=0.0, y_sig=0.0, t_end=0.0, dt0=0.0,
               max_steps=0, max_consec_rejects=0, use_mix_rule=1, y_neg=0.0):
        if any(getattr(col, k, None) is not None
               for k in ("escape_diff_limited", "v_top", "v_dep", "phi_surf")):
            raise ValueError("served requests are closed columns (no boundary exchange)")
        N = int(np.asarray(col.P_bar).shape[0])
        prof, keep = _profile_struct(col, N)
        n0 = np.ascontiguousarray(col.n0, np.float64)
        o = SSOpts(tol_rel, y_floor, y_sig, t_end, dt0, max_steps, max_consec_rejects,
                   use_mix_rule, 0, y_neg)
        rid = ctypes.c_uint64()
        _check(_f["xod_serve_submit"](self.handle, network.handle, ctypes.byref(prof),
                                      _ptr(n0, c_double), ctypes.byref(o), ctypes.byref(rid)))
        self._shapes[rid.value] = (N, network.S)
        return rid.value

    def step(self):
        a, q = c_int32(), c_int32()
        _check(_f["xod_serve_step"](self.handle, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def poll(self, rid):
        st = c_int32()
        res = SSResult()
        lat = c_double()
        N, S = self._shapes[rid]
        n = np.zeros((N, S))
        status = _f["xod_serve_poll"](self.handle, rid, ctypes.byref(st), _ptr(n, c_double),
                                      ctypes.byref(res), ctypes.byref(lat))
        out = res.as_dict()
        out.update(state=st.value, latency_s=lat.value, status=status)
        if st.value >= 2:
            out["n"] = n
        return out

    def release(self, rid):
        _check(_f["xod_serve_release"](self.handle, rid))
        self._shapes.pop(rid, None)

    def usage(self):
        used, a, q, it = ctypes.c_size_t(), c_int32(), c_int32(), ctypes.c_int64()
        _check(_f["xod_serve_usage"](self.handle, ctypes.byref(used), ctypes.byref(a),
                                     ctypes.byref(q), ctypes.byref(it)))
        return dict(used_bytes=used.value, active=a.value, queued=q.value, iterations=it.value)

    def close(self):
        if getattr(self, "handle", None):
            _f["xod_serve_destroy"](self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
