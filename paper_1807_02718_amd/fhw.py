"""Thin ctypes binding of libfhw (include/fhw.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libfhw.so.  PyTorch supplies device memory and the HIP stream.  Importing this
module without a built library raises immediately -- there is no fallback.

`Context` wraps the C entry points (its methods drop the fhw_ prefix) with
tensor allocation; the loaded library's functions keep the C names.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfhw.so")

FHW_OK = 0
FHW_E_INVALID = -1
FHW_E_NOMEM = -2
FHW_E_HIP = -3
FHW_E_SINGULAR = -4
FHW_E_NOCONV = -5
FHW_E_STATE = -6
FHW_E_BUSY = -7
FHW_FP64 = 0
FHW_FP32_REFINE = 1
FHW_FORM_DIRECT = 0
FHW_FORM_COMBINED = 1
FHW_INC_PLANE = 0
FHW_INC_POINT = 1

_dp = C.POINTER(C.c_double)


class fhw_curve(C.Structure):
    _fields_ = [("degree", C.c_int32), ("cx", _dp), ("sx", _dp), ("cy", _dp), ("sy", _dp)]


class fhw_problem(C.Structure):
    _fields_ = [("W", C.c_double), ("F", C.c_int32), ("c", C.c_double), ("N_fixed", C.c_int32),
                ("ppw", C.c_double), ("n_min", C.c_int32), ("n_mult", C.c_int32), ("n_cap", C.c_int32),
                ("precision", C.c_int32), ("refine_tol", C.c_double), ("refine_max", C.c_int32),
                ("direction", C.c_double * 2), ("j_first", C.c_int32),
                ("lf_M", C.c_int32), ("lf_N", C.c_int32), ("lf_jc", C.c_int32), ("lf_q", C.c_double),
                ("formulation", C.c_int32)]


class fhw_signal(C.Structure):
    _fields_ = [("t0", C.c_double), ("dt", C.c_double), ("n", C.c_int64), ("f", C.c_void_p)]


class fhw_windows(C.Structure):
    _fields_ = [("H", C.c_double), ("tau0", C.c_double), ("track_tol", C.c_double)]


class fhw_incidence(C.Structure):
    _fields_ = [("kind", C.c_int32), ("v", C.c_double * 2)]


class fhw_boundary(C.Structure):
    _fields_ = [("b", C.c_void_p), ("N", C.c_int32), ("n_t", C.c_int64), ("t0", C.c_double), ("dt", C.c_double)]


class fhw_system(C.Structure):
    _fields_ = [("curve", C.c_int32), ("omega", C.c_double), ("N", C.c_int32)]


class fhw_request(C.Structure):
    _fields_ = [("curve", C.c_int32), ("n_freq", C.c_int32), ("omegas", _dp), ("N", C.c_int32),
                ("n_inc", C.c_int32), ("inc", C.POINTER(fhw_incidence)), ("psi", C.c_void_p), ("resid", _dp),
                ("sweeps", C.POINTER(C.c_int32))]


def window_range(t_lo, t_hi, H):
    """fhw_window_range: (k_first, n_win) of the windows meeting [t_lo, t_hi]."""
    k, n = C.c_int64(0), C.c_int32(0)
    rc = _lib.fhw_window_range(float(t_lo), float(t_hi), float(H), C.byref(k), C.byref(n))
    if rc:
        raise FhwError(rc, "window_range: bad arguments")
    return int(k.value), int(n.value)


class FhwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libfhw error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libfhw.so not built at {LIB_PATH}; run python -m paper_1807_02718_amd.build")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    p_i32, p_i64 = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    sig = {
        "fhw_create": [C.POINTER(vp), vp, sz],
        "fhw_destroy": [vp],
        "fhw_version": [],
        "fhw_plan": [vp, C.POINTER(fhw_curve), C.POINTER(fhw_problem), p_i32, p_i64],
        "fhw_plan_curves": [vp, C.POINTER(fhw_curve), i32, C.POINTER(fhw_problem), p_i32, p_i64],
        "fhw_plan_systems": [vp, C.POINTER(fhw_curve), i32, C.POINTER(fhw_system), i32, C.POINTER(fhw_problem), p_i64],
        "fhw_factor": [vp],
        "fhw_solve_range": [vp, i32, i32, C.POINTER(fhw_incidence), i32, vp, _dp, p_i32],
        "fhw_solve_range_noalloc": [vp, i32, i32, C.POINTER(fhw_incidence), i32, vp, _dp, p_i32],
        "fhw_solve_densities": [vp, vp, _dp, p_i32, i32],
        "fhw_solve_incidences": [vp, C.POINTER(fhw_incidence), i32, vp, _dp, p_i32, i32],
        "fhw_solve_cached": [vp, C.POINTER(fhw_incidence), i32, vp, _dp, p_i32],
        "fhw_eval_field": [vp, vp, _dp, i32, C.c_double, vp],
        "fhw_eval_field_curve": [vp, i32, vp, _dp, i32, C.c_double, vp],
        "fhw_eval_field_lowfreq": [vp, vp, _dp, i32, C.c_double, vp],
        "fhw_synthesize_lowfreq": [vp, C.POINTER(fhw_signal), C.POINTER(fhw_windows), vp, vp, i32, _dp, i32, vp],
        "fhw_synthesize": [vp, C.POINTER(fhw_signal), C.POINTER(fhw_windows), vp, i32, _dp, i32, vp],
        "fhw_synthesize_uniform": [vp, C.POINTER(fhw_signal), C.POINTER(fhw_windows), vp, i32, C.c_double,
                                   C.c_double, i32, i32, vp],
        "fhw_synth_active_pairs": [vp, p_i64, p_i64],
        "fhw_run": [vp, C.POINTER(fhw_signal), C.POINTER(fhw_windows), _dp, i32, _dp, i32, vp, vp, vp, _dp, p_i32],
        "fhw_window_range": [C.c_double, C.c_double, C.c_double, p_i64, p_i32],
        "fhw_solve_general": [vp, C.POINTER(fhw_boundary), C.c_double, i64, i32, vp, _dp, p_i32],
        "fhw_eval_field_windows": [vp, vp, i32, _dp, i32, vp],
        "fhw_eval_field_windows_lowfreq": [vp, vp, i32, _dp, i32, vp],
        "fhw_synthesize_windows": [vp, C.POINTER(fhw_windows), i64, i32, vp, i32, _dp, i32, vp],
        "fhw_synthesize_windows_lowfreq": [vp, C.POINTER(fhw_windows), i64, i32, vp, vp, i32, _dp, i32, vp],
        "fhw_geometry": [vp, i32, vp],
        "fhw_kress_weights": [vp, i32, vp, vp],
        "fhw_assemble": [vp, i32, i32, vp, p_i64, vp, p_i64],
        "fhw_lu_factor": [vp, i32, p_i32, p_i64, vp, p_i64, vp, p_i64, vp, i32],
        "fhw_lu_solve": [vp, i32, p_i32, p_i64, vp, p_i64, vp, p_i64, vp, p_i64, vp, i32],
        "fhw_window_spectra": [vp, C.POINTER(fhw_signal), C.POINTER(fhw_windows), i64, i32, vp],
        "fhw_fourier_coefficients": [vp, vp, i32, vp, i32, C.c_double, vp],
        "fhw_hankel01": [vp, vp, i64, vp],
        "fhw_server_create": [C.POINTER(vp), C.POINTER(fhw_curve), i32, C.POINTER(fhw_problem), i32, sz, sz],
        "fhw_server_submit": [vp, C.POINTER(fhw_request), p_i64],
        "fhw_server_poll": [vp, i64, i32, p_i32],
        "fhw_server_stats": [vp, p_i64, _dp],
        "fhw_server_destroy": [vp],
        "fhw_profile": [vp, i32],
        "fhw_profile_read": [vp, _dp, p_i64],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.fhw_last_error.argtypes = [vp]
    lib.fhw_last_error.restype = C.c_char_p
    return lib


_lib = _load()
EXPORTED = ("fhw_create", "fhw_destroy", "fhw_last_error", "fhw_version", "fhw_plan", "fhw_plan_curves",
            "fhw_plan_systems", "fhw_factor", "fhw_solve_range", "fhw_solve_range_noalloc",
            "fhw_solve_densities", "fhw_solve_incidences", "fhw_solve_cached", "fhw_eval_field", "fhw_eval_field_curve", "fhw_eval_field_lowfreq", "fhw_synthesize", "fhw_synthesize_lowfreq", "fhw_synthesize_uniform", "fhw_synth_active_pairs", "fhw_run", "fhw_window_range", "fhw_solve_general",
            "fhw_eval_field_windows", "fhw_eval_field_windows_lowfreq", "fhw_synthesize_windows",
            "fhw_synthesize_windows_lowfreq", "fhw_geometry", "fhw_kress_weights", "fhw_assemble",
            "fhw_lu_factor", "fhw_lu_solve", "fhw_window_spectra", "fhw_fourier_coefficients", "fhw_hankel01",
            "fhw_profile", "fhw_profile_read", "fhw_server_create", "fhw_server_submit", "fhw_server_poll",
            "fhw_server_stats", "fhw_server_destroy")
STAGES = ("geometry", "kress", "assemble", "lu_panel", "lu_diaginv", "lu_swap", "lu_trsm", "lu_update", "solve",
          "residual", "field", "spectra", "coeffs", "synth")


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("device tensor expected")
        if not t.is_contiguous():
            raise ValueError("contiguous tensor expected")
        return C.c_void_p(t.data_ptr())
    raise TypeError(type(t))


def _host(a, dtype):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    return a, a.ctypes.data_as(C.POINTER(np.ctypeslib.as_ctypes_type(dtype)))


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """A libfhw context bound to one HIP stream."""

    def __init__(self, stream=None, hbm_budget_bytes=0, device=None):
        if device is not None:
            torch.cuda.set_device(device)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = _lib.fhw_create(C.byref(h), _stream_handle(self.stream), hbm_budget_bytes)
        if rc != FHW_OK:
            raise FhwError(rc, "fhw_create failed")
        self._h = h
        self.F = None

    def close(self):
        if getattr(self, "_h", None):
            _lib.fhw_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != FHW_OK:
            raise FhwError(rc, _lib.fhw_last_error(self._h).decode())

    # -- plan -----------------------------------------------------------------
    def plan(self, curve, W, F, N=None, c=1.0, ppw=10.0, n_min=64, n_mult=32, n_cap=4096, precision="fp64",
             refine_tol=1e-12, refine_max=10, direction=(1.0, 0.0), j_first=0, lowfreq=None, formulation="direct"):
        """Plan one curve, or several (a list: fhw_plan_curves, system s = k F + j).
        j_first > 0 plans the band (j_first + j) W / F, j = 1..F (solves only).
        lowfreq = dict(jc, M, n, q) adds the graded low-frequency systems
        (M n - 1 of them after the F grid systems; one curve).  formulation
        "combined": the exterior Dirichlet problem for arbitrary data (general
        boundary data, fhw_solve_general; one curve, fixed N).
        Returns (N per system, psi offsets)."""
        many = isinstance(curve, (list, tuple))
        curves = list(curve) if many else [curve]
        self._cv = [[np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (cv.cx, cv.sx, cv.cy, cv.sy)]
                    for cv in curves]
        arr = (fhw_curve * len(curves))()
        for k, vs in enumerate(self._cv):
            arr[k] = fhw_curve(len(vs[0]) - 1, *[v.ctypes.data_as(_dp) for v in vs])
        pr = fhw_problem()
        pr.W, pr.F, pr.c = float(W), int(F), float(c)
        pr.N_fixed = int(N) if N is not None else 0
        pr.ppw, pr.n_min, pr.n_mult, pr.n_cap = float(ppw), int(n_min), int(n_mult), int(n_cap)
        pr.precision = {"fp64": FHW_FP64, "fp32_refine": FHW_FP32_REFINE}[precision]
        pr.refine_tol, pr.refine_max = float(refine_tol), int(refine_max)
        pr.direction[0], pr.direction[1] = float(direction[0]), float(direction[1])
        pr.j_first = int(j_first)
        pr.formulation = {"direct": FHW_FORM_DIRECT, "combined": FHW_FORM_COMBINED}[formulation]
        extra = 0
        if lowfreq is not None:
            pr.lf_M, pr.lf_N, pr.lf_jc = int(lowfreq["M"]), int(lowfreq["n"]), int(lowfreq["jc"])
            pr.lf_q = float(lowfreq["q"])
            extra = pr.lf_M * pr.lf_N - 1
        S = len(curves) * int(F) + extra
        Ns = np.zeros(S, dtype=np.int32)
        off = np.zeros(S + 1, dtype=np.int64)
        pN, po = Ns.ctypes.data_as(C.POINTER(C.c_int32)), off.ctypes.data_as(C.POINTER(C.c_int64))
        if many:
            self._check(_lib.fhw_plan_curves(self._h, arr, len(curves), C.byref(pr), pN, po))
        else:
            self._check(_lib.fhw_plan(self._h, arr, C.byref(pr), pN, po))
        self.F, self.W, self.Ns, self.psi_off = int(F), float(W), Ns, off
        self.S, self.n_curves = S, len(curves)
        self.precision = precision
        self.lowfreq = dict(lowfreq) if lowfreq is not None else None
        return Ns, off

    def plan_systems(self, curves, systems, c=1.0, precision="fp64", refine_tol=1e-12, refine_max=10,
                     direction=(1.0, 0.0)):
        """fhw_plan_systems: systems = sequence of (curve index, omega, N).
        Returns the psi offsets (n_systems + 1)."""
        self._cv = [[np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (cv.cx, cv.sx, cv.cy, cv.sy)]
                    for cv in curves]
        arr = (fhw_curve * len(curves))()
        for k, vs in enumerate(self._cv):
            arr[k] = fhw_curve(len(vs[0]) - 1, *[v.ctypes.data_as(_dp) for v in vs])
        S = len(systems)
        sy = (fhw_system * max(S, 1))()
        for s, (k, om, N) in enumerate(systems):
            sy[s] = fhw_system(int(k), float(om), int(N))
        pr = fhw_problem()
        pr.W, pr.F, pr.c = 1.0, 1, float(c)
        pr.precision = {"fp64": FHW_FP64, "fp32_refine": FHW_FP32_REFINE}[precision]
        pr.refine_tol, pr.refine_max = float(refine_tol), int(refine_max)
        pr.direction[0], pr.direction[1] = float(direction[0]), float(direction[1])
        off = np.zeros(S + 1, dtype=np.int64)
        self._check(_lib.fhw_plan_systems(self._h, arr, len(curves), sy, S, C.byref(pr),
                                          off.ctypes.data_as(C.POINTER(C.c_int64))))
        self.F, self.W, self.Ns, self.psi_off = 0, 0.0, np.array([n for _, _, n in systems], dtype=np.int32), off
        self.S, self.n_curves = S, len(curves)
        self.precision = precision
        return off

    def factor(self):
        """fhw_factor: assemble and factor every planned system; factors stay resident."""
        self._check(_lib.fhw_factor(self._h))

    def solve_range(self, s0, count, incidences, psi=None, noalloc=False):
        """fhw_solve_range on systems s0 .. s0+count-1 (noalloc: the
        allocation-free variant fhw_solve_range_noalloc, same results).
        Returns (psi [n_inc, E] complex128, resid [n_inc, count], sweeps
        [n_inc, count])."""
        kinds = {"plane": FHW_INC_PLANE, "point": FHW_INC_POINT}
        n = len(incidences)
        arr = (fhw_incidence * max(n, 1))()
        for q, (kind, v) in enumerate(incidences):
            arr[q].kind = kinds[kind] if isinstance(kind, str) else int(kind)
            arr[q].v[0], arr[q].v[1] = float(v[0]), float(v[1])
        ok = 0 <= s0 and count >= 1 and s0 + count <= self.S
        E = int(self.psi_off[s0 + count] - self.psi_off[s0]) if ok else 1   # else the library refuses the range
        if psi is None:
            psi = torch.empty((max(n, 1), E), dtype=torch.complex128, device=self.device)
        resid = np.zeros((max(n, 1), count))
        sweeps = np.zeros((max(n, 1), count), dtype=np.int32)
        call = _lib.fhw_solve_range_noalloc if noalloc else _lib.fhw_solve_range
        self._check(call(self._h, int(s0), int(count), arr, n, _ptr(psi), resid.ctypes.data_as(_dp),
                         sweeps.ctypes.data_as(C.POINTER(C.c_int32))))
        return psi, resid, sweeps

    # -- hot path ---------------------------------------------------------------
    def solve_densities(self, psi=None, compute_resid=False):
        if psi is None:
            psi = torch.empty(int(self.psi_off[-1]), dtype=torch.complex128, device=self.device)
        resid = np.zeros(self.S)
        sweeps = np.zeros(self.S, dtype=np.int32)
        self._check(_lib.fhw_solve_densities(self._h, _ptr(psi), resid.ctypes.data_as(_dp),
                                             sweeps.ctypes.data_as(C.POINTER(C.c_int32)), int(bool(compute_resid))))
        return psi, resid, sweeps

    def _incidences(self, incidences, psi):
        kinds = {"plane": FHW_INC_PLANE, "point": FHW_INC_POINT}
        n = len(incidences)
        arr = (fhw_incidence * max(n, 1))()
        for q, (kind, v) in enumerate(incidences):
            arr[q].kind = kinds[kind] if isinstance(kind, str) else int(kind)
            arr[q].v[0], arr[q].v[1] = float(v[0]), float(v[1])
        if psi is None:
            psi = torch.empty((max(n, 1), int(self.psi_off[-1])), dtype=torch.complex128, device=self.device)
        resid = np.zeros((max(n, 1), self.S))
        sweeps = np.zeros((max(n, 1), self.S), dtype=np.int32)
        return arr, n, psi, resid, sweeps

    def solve_incidences(self, incidences, psi=None, compute_resid=False):
        """incidences: sequence of ("plane", (p1, p2)) or ("point", (x, y)).
        Returns (psi [n_inc, psi_off[F]] complex128, resid [n_inc, F], sweeps [n_inc, F])."""
        arr, n, psi, resid, sweeps = self._incidences(incidences, psi)
        self._check(_lib.fhw_solve_incidences(self._h, arr, n, _ptr(psi), resid.ctypes.data_as(_dp),
                                              sweeps.ctypes.data_as(C.POINTER(C.c_int32)), int(bool(compute_resid))))
        return psi, resid, sweeps

    def solve_cached(self, incidences, psi=None):
        """As solve_incidences, with the factors left resident by the last solve."""
        arr, n, psi, resid, sweeps = self._incidences(incidences, psi)
        self._check(_lib.fhw_solve_cached(self._h, arr, n, _ptr(psi), resid.ctypes.data_as(_dp),
                                          sweeps.ctypes.data_as(C.POINTER(C.c_int32))))
        return psi, resid, sweeps

    def eval_field(self, psi, obs, zero_value=1.0, V=None, curve=0):
        obs_h, obs_p = _host(obs, np.float64)
        Nr = obs_h.shape[0]
        if V is None:
            V = torch.empty((Nr, 2 * self.F), dtype=torch.complex128, device=self.device)
        if curve == 0:
            self._check(_lib.fhw_eval_field(self._h, _ptr(psi), obs_p, Nr, float(zero_value), _ptr(V)))
        else:
            self._check(_lib.fhw_eval_field_curve(self._h, int(curve), _ptr(psi), obs_p, Nr, float(zero_value),
                                                  _ptr(V)))
        return V

    def eval_field_lowfreq(self, psi, obs, zero_value=1.0, V_sing=None):
        """fhw_eval_field_lowfreq: the field at the graded nodes (ascending,
        0 .. omega_c), complex128 [N_r][M n + 1]."""
        obs_h, obs_p = _host(obs, np.float64)
        Nr = obs_h.shape[0]
        if V_sing is None:
            lf = self.lowfreq or {"M": 0, "n": 0}
            V_sing = torch.empty((Nr, lf["M"] * lf["n"] + 1), dtype=torch.complex128, device=self.device)
        self._check(_lib.fhw_eval_field_lowfreq(self._h, _ptr(psi), obs_p, Nr, float(zero_value), _ptr(V_sing)))
        return V_sing

    def synthesize_lowfreq(self, f, t0, dt, H, tau0, V, V_sing, times, u=None):
        """fhw_synthesize_lowfreq: time samples with the 2D low-frequency
        decomposition from V [N_r][2F] and V_sing [N_r][M n + 1]."""
        f = f if isinstance(f, torch.Tensor) else torch.as_tensor(np.asarray(f, dtype=np.float64), device=self.device)
        sg = fhw_signal(float(t0), float(dt), int(f.numel()), _ptr(f).value)
        wn = fhw_windows(float(H), float(tau0), 0.0)
        th, tp = _host(times, np.float64)
        Nr = V.shape[0]
        if u is None:
            u = torch.empty((Nr, len(th)), dtype=torch.float64, device=self.device)
        self._check(_lib.fhw_synthesize_lowfreq(self._h, C.byref(sg), C.byref(wn), _ptr(V), _ptr(V_sing), Nr, tp,
                                                len(th), _ptr(u)))
        return u

    def synthesize(self, f, t0, dt, H, tau0, V, times, u=None, track_tol=0.0):
        f = f if isinstance(f, torch.Tensor) else torch.as_tensor(np.asarray(f, dtype=np.float64), device=self.device)
        sg = fhw_signal(float(t0), float(dt), int(f.numel()), _ptr(f).value)
        wn = fhw_windows(float(H), float(tau0), float(track_tol))
        th, tp = _host(times, np.float64)
        Nr = V.shape[0]
        if u is None:
            u = torch.empty((Nr, len(th)), dtype=torch.float64, device=self.device)
        self._check(_lib.fhw_synthesize(self._h, C.byref(sg), C.byref(wn), _ptr(V), Nr, tp, len(th), _ptr(u)))
        return u

    def synthesize_uniform(self, f, t0, dt, H, tau0, V, t_first, t_step, n_t, L=0, u=None, track_tol=0.0):
        """fhw_synthesize_uniform: u[r][n] at t_first + n t_step by the fast
        scaled convolution of size L (0 = max(4F, 8))."""
        f = f if isinstance(f, torch.Tensor) else torch.as_tensor(np.asarray(f, dtype=np.float64), device=self.device)
        sg = fhw_signal(float(t0), float(dt), int(f.numel()), _ptr(f).value)
        wn = fhw_windows(float(H), float(tau0), float(track_tol))
        Nr = V.shape[0]
        if u is None:
            u = torch.empty((Nr, int(n_t)), dtype=torch.float64, device=self.device)
        self._check(_lib.fhw_synthesize_uniform(self._h, C.byref(sg), C.byref(wn), _ptr(V), Nr, float(t_first),
                                                float(t_step), int(n_t), int(L), _ptr(u)))
        return u

    # -- stage entry points -------------------------------------------------------
    def run(self, f, t0, dt, H, tau0, obs, times, psi=None, V=None, u=None):
        """fhw_run: densities, field (V(r, 0) = 1) and time samples in one call.
        Returns (u, psi, V, resid, sweeps)."""
        f = f if isinstance(f, torch.Tensor) else torch.as_tensor(np.asarray(f, dtype=np.float64), device=self.device)
        sg = fhw_signal(float(t0), float(dt), int(f.numel()), _ptr(f).value)
        wn = fhw_windows(float(H), float(tau0), 0.0)
        obs_h, obs_p = _host(obs, np.float64)
        th, tp = _host(times, np.float64)
        Nr = obs_h.shape[0]
        if psi is None:
            psi = torch.empty(int(self.psi_off[-1]), dtype=torch.complex128, device=self.device)
        if V is None:
            V = torch.empty((Nr, 2 * self.F), dtype=torch.complex128, device=self.device)
        if u is None:
            u = torch.empty((Nr, len(th)), dtype=torch.float64, device=self.device)
        resid = np.zeros(self.S)
        sweeps = np.zeros(self.S, dtype=np.int32)
        self._check(_lib.fhw_run(self._h, C.byref(sg), C.byref(wn), obs_p, Nr, tp, len(th), _ptr(psi), _ptr(V),
                                 _ptr(u), resid.ctypes.data_as(_dp), sweeps.ctypes.data_as(C.POINTER(C.c_int32))))
        return u, psi, V, resid, sweeps

    # -- general incident fields ---------------------------------------------------
    def solve_general(self, b, t0, dt, H, k_first=None, n_win=None, psi=None):
        """fhw_solve_general on a plan of the combined formulation: b device
        float64 [n_t][N] (Dirichlet data -u_inc at the nodes); windows k_first
        .. k_first + n_win - 1 (default: all that meet the samples' range).
        Returns (psi [n_win, psi_off[S]] complex128, resid [n_win, S], sweeps
        [n_win, S], k_first)."""
        n_t, N = int(b.shape[0]), int(b.shape[1])
        if k_first is None or n_win is None:
            k_first, n_win = window_range(t0, t0 + dt * (n_t - 1), H)
        bd = fhw_boundary(_ptr(b).value, N, n_t, float(t0), float(dt))
        if psi is None:
            psi = torch.empty((max(int(n_win), 1), int(self.psi_off[-1])), dtype=torch.complex128, device=self.device)
        resid = np.zeros((max(int(n_win), 1), self.S))
        sweeps = np.zeros((max(int(n_win), 1), self.S), dtype=np.int32)
        self._check(_lib.fhw_solve_general(self._h, C.byref(bd), float(H), int(k_first), int(n_win), _ptr(psi),
                                           resid.ctypes.data_as(_dp), sweeps.ctypes.data_as(C.POINTER(C.c_int32))))
        return psi, resid, sweeps, int(k_first)

    def eval_field_windows(self, psi, obs, V=None):
        """fhw_eval_field_windows: V [n_win, N_r, 2F] complex128, V(r, 0) = 0."""
        obs_h, obs_p = _host(obs, np.float64)
        Nr, nw = obs_h.shape[0], int(psi.shape[0])
        if V is None:
            V = torch.empty((nw, Nr, 2 * self.F), dtype=torch.complex128, device=self.device)
        self._check(_lib.fhw_eval_field_windows(self._h, _ptr(psi), nw, obs_p, Nr, _ptr(V)))
        return V

    def eval_field_windows_lowfreq(self, psi, obs, V_sing=None):
        """fhw_eval_field_windows_lowfreq: V_sing [n_win, N_r, M n + 1] complex128."""
        obs_h, obs_p = _host(obs, np.float64)
        Nr, nw = obs_h.shape[0], int(psi.shape[0])
        if V_sing is None:
            lf = self.lowfreq or {"M": 0, "n": 0}
            V_sing = torch.empty((nw, Nr, lf["M"] * lf["n"] + 1), dtype=torch.complex128, device=self.device)
        self._check(_lib.fhw_eval_field_windows_lowfreq(self._h, _ptr(psi), nw, obs_p, Nr, _ptr(V_sing)))
        return V_sing

    def synthesize_windows(self, H, tau0, k_first, V, times, u=None):
        """fhw_synthesize_windows: u [N_r, N_t] from each window's own field."""
        wn = fhw_windows(float(H), float(tau0), 0.0)
        th, tp = _host(times, np.float64)
        nw, Nr = int(V.shape[0]), int(V.shape[1])
        if u is None:
            u = torch.empty((Nr, len(th)), dtype=torch.float64, device=self.device)
        self._check(_lib.fhw_synthesize_windows(self._h, C.byref(wn), int(k_first), nw, _ptr(V), Nr, tp, len(th),
                                                _ptr(u)))
        return u

    def synthesize_windows_lowfreq(self, H, tau0, k_first, V, V_sing, times, u=None):
        """fhw_synthesize_windows_lowfreq: u [N_r, N_t] with the low-frequency
        decomposition from each window's own fields."""
        wn = fhw_windows(float(H), float(tau0), 0.0)
        th, tp = _host(times, np.float64)
        nw, Nr = int(V.shape[0]), int(V.shape[1])
        if u is None:
            u = torch.empty((Nr, len(th)), dtype=torch.float64, device=self.device)
        self._check(_lib.fhw_synthesize_windows_lowfreq(self._h, C.byref(wn), int(k_first), nw, _ptr(V),
                                                        _ptr(V_sing), Nr, tp, len(th), _ptr(u)))
        return u

    def synth_active_pairs(self):
        """(window, point) pairs of the last synthesis and how many tracking kept."""
        p, a = C.c_int64(0), C.c_int64(0)
        self._check(_lib.fhw_synth_active_pairs(self._h, C.byref(p), C.byref(a)))
        return int(p.value), int(a.value)

    def geometry(self, N):
        g = torch.empty((9, N), dtype=torch.float64, device=self.device)
        self._check(_lib.fhw_geometry(self._h, int(N), _ptr(g)))
        return g

    def kress_weights(self, N):
        R = torch.empty(N, dtype=torch.float64, device=self.device)
        L = torch.empty(N, dtype=torch.float64, device=self.device)
        self._check(_lib.fhw_kress_weights(self._h, int(N), _ptr(R), _ptr(L)))
        return R, L

    def assemble(self, j0, count):
        Ns = self.Ns[j0:j0 + count].astype(np.int64)
        a_off = np.concatenate([[0], np.cumsum(Ns * Ns)[:-1]]).astype(np.int64)
        g_off = np.concatenate([[0], np.cumsum(Ns)[:-1]]).astype(np.int64)
        A = torch.empty(int((Ns * Ns).sum()), dtype=torch.complex128, device=self.device)
        g = torch.empty(int(Ns.sum()), dtype=torch.complex128, device=self.device)
        self._check(_lib.fhw_assemble(self._h, int(j0), int(count), _ptr(A), a_off.ctypes.data_as(C.POINTER(C.c_int64)),
                                      _ptr(g), g_off.ctypes.data_as(C.POINTER(C.c_int64))))
        # column-major storage: the (N, N) row-major view of each block is A^T
        mats = [A[a_off[q]:a_off[q] + Ns[q] * Ns[q]].view(int(Ns[q]), int(Ns[q])).t() for q in range(count)]
        vecs = [g[g_off[q]:g_off[q] + Ns[q]] for q in range(count)]
        return mats, vecs

    def lu_factor(self, A_flat, Ns, precision="fp64"):
        """In-place batched LU of column-major matrices packed in A_flat
        (complex128 or complex64)."""
        Ns = np.asarray(Ns, dtype=np.int32)
        a_off = np.concatenate([[0], np.cumsum(Ns.astype(np.int64) ** 2)[:-1]]).astype(np.int64)
        p_off = np.concatenate([[0], np.cumsum(Ns.astype(np.int64))[:-1]]).astype(np.int64)
        l_off = np.concatenate([[0], np.cumsum(4096 * ((Ns.astype(np.int64) + 63) // 64))[:-1]]).astype(np.int64)
        piv = torch.empty(int(Ns.sum()), dtype=torch.int32, device=self.device)
        ltot = int((4096 * ((Ns.astype(np.int64) + 63) // 64)).sum())
        linv = torch.empty(ltot, dtype=A_flat.dtype, device=self.device)
        prec = {"fp64": FHW_FP64, "fp32_refine": FHW_FP32_REFINE}[precision]
        self._check(_lib.fhw_lu_factor(self._h, len(Ns), Ns.ctypes.data_as(C.POINTER(C.c_int32)),
                                       a_off.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(A_flat),
                                       p_off.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(piv),
                                       l_off.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(linv), prec))
        return dict(Ns=Ns, a_off=a_off, p_off=p_off, l_off=l_off, piv=piv, linv=linv, LU=A_flat, prec=prec)

    def lu_solve(self, fac, b_flat):
        Ns = fac["Ns"]
        b_off = np.concatenate([[0], np.cumsum(Ns.astype(np.int64))[:-1]]).astype(np.int64)
        self._check(_lib.fhw_lu_solve(self._h, len(Ns), Ns.ctypes.data_as(C.POINTER(C.c_int32)),
                                      fac["a_off"].ctypes.data_as(C.POINTER(C.c_int64)), _ptr(fac["LU"]),
                                      fac["p_off"].ctypes.data_as(C.POINTER(C.c_int64)), _ptr(fac["piv"]),
                                      fac["l_off"].ctypes.data_as(C.POINTER(C.c_int64)), _ptr(fac["linv"]),
                                      b_off.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(b_flat), fac["prec"]))
        return b_flat

    def window_spectra(self, f, t0, dt, H, k_first, count):
        f = f if isinstance(f, torch.Tensor) else torch.as_tensor(np.asarray(f, dtype=np.float64), device=self.device)
        sg = fhw_signal(float(t0), float(dt), int(f.numel()), _ptr(f).value)
        wn = fhw_windows(float(H), 0.0)
        B = torch.empty((count, 2 * self.F), dtype=torch.complex128, device=self.device)
        self._check(_lib.fhw_window_spectra(self._h, C.byref(sg), C.byref(wn), int(k_first), int(count), _ptr(B)))
        return B

    def fourier_coefficients(self, B, V, tau0):
        count, Nr = B.shape[0], V.shape[0]
        c = torch.empty((count, Nr, 2 * self.F), dtype=torch.complex128, device=self.device)
        self._check(_lib.fhw_fourier_coefficients(self._h, _ptr(B), count, _ptr(V), Nr, float(tau0), _ptr(c)))
        return c

    def profile(self, enable=True):
        self._check(_lib.fhw_profile(self._h, int(bool(enable))))

    def profile_read(self):
        """{stage: (milliseconds, launches)} since the last read; clears the counters."""
        ms = np.zeros(len(STAGES))
        n = np.zeros(len(STAGES), dtype=np.int64)
        self._check(_lib.fhw_profile_read(self._h, ms.ctypes.data_as(_dp), n.ctypes.data_as(C.POINTER(C.c_int64))))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(STAGES)}

    def hankel01(self, z):
        z = z if isinstance(z, torch.Tensor) else torch.as_tensor(np.asarray(z, dtype=np.float64), device=self.device)
        h = torch.empty((z.numel(), 2), dtype=torch.complex128, device=self.device)
        self._check(_lib.fhw_hankel01(self._h, _ptr(z), int(z.numel()), _ptr(h)))
        return h


class Server:
    """fhw_server: continuous batching of solve requests over worker slots,
    each with its own stream and workspace (see include/fhw.h)."""

    def __init__(self, curves, precision="fp32_refine", refine_tol=1e-12, refine_max=10, c=1.0, slots=2,
                 hbm_budget_bytes=0, queue_limit_bytes=0, device=None):
        if device is not None:
            torch.cuda.set_device(device)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._cv = [[np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (cv.cx, cv.sx, cv.cy, cv.sy)]
                    for cv in curves]
        arr = (fhw_curve * len(curves))()
        for k, vs in enumerate(self._cv):
            arr[k] = fhw_curve(len(vs[0]) - 1, *[v.ctypes.data_as(_dp) for v in vs])
        pr = fhw_problem()
        pr.c = float(c)
        pr.precision = {"fp64": FHW_FP64, "fp32_refine": FHW_FP32_REFINE}[precision]
        pr.refine_tol, pr.refine_max = float(refine_tol), int(refine_max)
        h = C.c_void_p()
        rc = _lib.fhw_server_create(C.byref(h), arr, len(curves), C.byref(pr), int(slots), int(hbm_budget_bytes),
                                    int(queue_limit_bytes))
        if rc != FHW_OK:
            raise FhwError(rc, "fhw_server_create failed")
        self._h = h
        self._keep = {}   # ticket -> buffers that must outlive the request

    def submit(self, curve, omegas, N, incidences, psi=None):
        """Queue a request; returns (ticket, psi [n_inc, n_freq N], resid
        [n_inc, n_freq], sweeps) with psi and resid filled on completion, or
        raises FhwError (code FHW_E_BUSY when the queue is full)."""
        om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
        kinds = {"plane": FHW_INC_PLANE, "point": FHW_INC_POINT}
        n = len(incidences)
        inc = (fhw_incidence * max(n, 1))()
        for q, (kind, v) in enumerate(incidences):
            inc[q].kind = kinds[kind] if isinstance(kind, str) else int(kind)
            inc[q].v[0], inc[q].v[1] = float(v[0]), float(v[1])
        if psi is None:
            psi = torch.empty((max(n, 1), len(om) * int(N)), dtype=torch.complex128, device=self.device)
        resid = np.zeros((max(n, 1), len(om)))
        sweeps = np.zeros((max(n, 1), len(om)), dtype=np.int32)
        req = fhw_request(int(curve), len(om), om.ctypes.data_as(_dp), int(N), n, inc, _ptr(psi).value,
                          resid.ctypes.data_as(_dp), sweeps.ctypes.data_as(C.POINTER(C.c_int32)))
        t = C.c_int64()
        rc = _lib.fhw_server_submit(self._h, C.byref(req), C.byref(t))
        if rc != FHW_OK:
            raise FhwError(rc, "fhw_server_submit refused the request" if rc == FHW_E_BUSY else "bad request")
        self._keep[t.value] = (psi, resid, sweeps)
        return t.value, psi, resid, sweeps

    def poll(self, ticket, wait=False):
        """1 while pending, else the request's result code (reported once)."""
        st = C.c_int32()
        rc = _lib.fhw_server_poll(self._h, int(ticket), int(bool(wait)), C.byref(st))
        if rc != FHW_OK:
            raise FhwError(rc, "unknown ticket")
        if st.value != 1:
            self._keep.pop(int(ticket), None)
        return st.value

    def stats(self):
        counts = np.zeros(6, dtype=np.int64)
        busy = C.c_double()
        _lib.fhw_server_stats(self._h, counts.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(busy))
        return dict(rounds=int(counts[0]), done=int(counts[1]), refused=int(counts[2]), systems=int(counts[3]),
                    waiting=int(counts[4]), cache_hits=int(counts[5]), busy_s=busy.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.fhw_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fhw_version():
    return _lib.fhw_version()


def library():
    """The loaded ctypes library (for symbol checks)."""
    return _lib
