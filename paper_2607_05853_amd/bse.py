"""ctypes binding of libbse.so, the gfx950 dual-k-mesh TDA-BSE library.

Argument marshalling only: tensors are checked for device, dtype, shape and
contiguity, their device pointers and torch's current HIP stream are passed
to the C ABI, and status codes become exceptions.  Every step of the
computation runs in the library's HIP kernels; there is no CPU fallback, and
importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BSE_LIB", os.path.join(_HERE, "libbse.so"))

PREC = {"f64": 0, "f32": 1, "bf16x3": 2}
BSE_OK, BSE_INFO_BREAKDOWN, BSE_INFO_NOT_CONVERGED = 0, 100, 101
CHECK_HERMITIAN = 1
ALL_PAIRS = 2
CONDUCTION = {None: 0, "mc": 4, "u": 8}


class BSEError(RuntimeError):
    def __init__(self, where, status, msg):
        super().__init__("%s: status %d (%s): %s" % (where, status, _status_string(status), msg))
        self.status = status


class _Dims(ctypes.Structure):
    _fields_ = [("nk", ctypes.c_int32 * 3), ("n_ao", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("nc", ctypes.c_int32), ("n_aux", ctypes.c_int32), ("alpha", ctypes.c_double)]


_lib = None
_vp, _i32, _f64p, _i32p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)

_SIGS = {
    "bse_interpolate_W": [_i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, ctypes.c_int, _vp],
    "bse_interpolate_W_adjoint": [_i32, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _vp],
    "bse_interpolate_W_noalloc": [_i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, ctypes.c_int, _vp],
    "bse_plan_create": [ctypes.POINTER(_Dims), _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _i32, ctypes.c_uint32, _vp,
                        ctypes.POINTER(_vp)],
    "bse_plan_create_2c": [ctypes.POINTER(_Dims), _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _i32,
                           ctypes.c_uint32, _vp, ctypes.POINTER(_vp)],
    "bse_plan_destroy": [_vp],
    "bse_plan_set_R": [_vp, _i32, _vp, _vp],
    "bse_plan_set_eps": [_vp, _vp, _vp],
    "bse_plan_bytes": [_vp, ctypes.POINTER(ctypes.c_uint64)],
    "bse_plan_pairs": [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "bse_plan_conduction": [_vp, ctypes.POINTER(ctypes.c_int32)],
    "bse_plan_fused": [_vp, ctypes.POINTER(ctypes.c_int32)],
    "bse_plan_frag": [_vp, ctypes.POINTER(ctypes.c_int32)],
    "bse_offset_spectrum": [_vp, _vp, _vp, _i32, _i32, _i32, _vp, _i32, ctypes.c_double, _vp, _vp, _vp],
    "bse_offset_set": [ctypes.POINTER(ctypes.c_int32), _vp, _vp],
    "bse_apply": [_vp, _vp, _vp, _i32, _vp],
    "bse_apply_adjoint": [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp],
    "bse_velocity_start": [_vp, _vp, _vp, _i32, _vp, _vp, _vp],
    "bse_density_start": [_vp, _vp, _vp, _vp],
    "bse_haydock_spectrum": [_vp, _vp, _i32, _i32, _vp, _i32, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, _vp],
    "bse_lowest_excitons": [_vp, _i32, _i32, ctypes.c_double, _vp, _vp, _vp, _vp, _vp],
    "bse_apply_coupling": [_vp, _vp, _vp, _i32, _vp],
    "bse_apply_full": [_vp, _vp, _vp, _i32, _vp],
    "bse_full_spectrum": [_vp, _vp, _i32, _i32, _vp, _i32, ctypes.c_double, _vp, _vp, _vp, _vp, _vp],
    "bse_full_lowest": [_vp, _i32, _i32, ctypes.c_double, _vp, _vp, _vp, _vp, _vp],
    "bse_haydock_vjp": [_vp, _vp, _vp, _vp, _vp, _i32, _i32, _vp, _i32, ctypes.c_double, _vp, _vp, _vp, _vp, _vp],
    "bse_plan_set_timing": [_vp, ctypes.c_int],
    "bse_plan_stage_times": [_vp, _vp, _vp, ctypes.c_int],
    "bse_status_string": [ctypes.c_int],
    "bse_last_error": [],
    "bse_version": [],
}
EXPORTS = tuple(_SIGS)


def lib():
    """Load libbse.so once; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbse.so not built at %s: run python paper_2607_05853_amd/build_lib.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name in ("bse_status_string", "bse_last_error", "bse_version") else ctypes.c_int
        _lib = L
    return _lib


def _status_string(s):
    try:
        return lib().bse_status_string(int(s)).decode()
    except Exception:
        return "?"


def _check(where, s, allow_breakdown=False):
    if s == BSE_OK or (allow_breakdown and s == BSE_INFO_BREAKDOWN):
        return s
    raise BSEError(where, s, lib().bse_last_error().decode())


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _dev(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    if shape is not None and a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), a.shape))
    return a


def version():
    return lib().bse_version().decode()


def interpolate_W(W_R, R, w_R, q_frac, out_prec="f64"):
    """W_q[q] = sum_R w_R W_R[R] exp(+2 pi i q.R) on the device (c128 or c64 output)."""
    n_R, na, _ = W_R.shape
    R = _host(R, np.int32, (n_R, 3))
    w_R = _host(w_R, np.float64, (n_R,))
    q = _host(q_frac, np.float64)
    q = q.reshape(-1, 3)
    out = torch.empty((len(q), na, na), dtype=torch.complex128 if out_prec == "f64" else torch.complex64,
                      device=W_R.device)
    s = lib().bse_interpolate_W(na, n_R, _dev(W_R, torch.complex128, (n_R, na, na), "W_R"),
                                R.ctypes.data, w_R.ctypes.data, len(q), q.ctypes.data,
                                _dev(out, out.dtype, None, "W_q"), PREC[out_prec], _stream(W_R.device))
    _check("bse_interpolate_W", s)
    return out


def interpolate_W_noalloc(W_R, R, w_R, q_frac, out, out_prec="f64"):
    """interpolate_W into a caller-provided W_q, with the library's static device workspace (no device
    allocation by the library)."""
    n_R, na, _ = W_R.shape
    R = _host(R, np.int32, (n_R, 3))
    w_R = _host(w_R, np.float64, (n_R,))
    q = _host(q_frac, np.float64).reshape(-1, 3)
    dt = torch.complex128 if out_prec == "f64" else torch.complex64
    s = lib().bse_interpolate_W_noalloc(na, n_R, _dev(W_R, torch.complex128, (n_R, na, na), "W_R"),
                                        R.ctypes.data, w_R.ctypes.data, len(q), q.ctypes.data,
                                        _dev(out, dt, (len(q), na, na), "W_q"), PREC[out_prec],
                                        _stream(W_R.device))
    _check("bse_interpolate_W_noalloc", s)
    return out


def interpolate_W_adjoint(g_Wq, R, w_R, q_frac):
    """g_WR[R] = w_R sum_q exp(-2 pi i q.R) g_Wq[q] on the device."""
    n_q, na, _ = g_Wq.shape
    R = _host(R, np.int32)
    R = R.reshape(-1, 3)
    w_R = _host(w_R, np.float64, (len(R),))
    q = _host(q_frac, np.float64, (n_q, 3))
    out = torch.empty((len(R), na, na), dtype=torch.complex128, device=g_Wq.device)
    s = lib().bse_interpolate_W_adjoint(na, len(R), R.ctypes.data, w_R.ctypes.data, n_q, q.ctypes.data,
                                        _dev(g_Wq, torch.complex128, None, "g_Wq"),
                                        _dev(out, torch.complex128, None, "g_WR"), _stream(g_Wq.device))
    _check("bse_interpolate_W_adjoint", s)
    return out


class Plan:
    """A TDA-BSE problem resident on one GPU (halves, rho, W_q and workspaces)."""

    def __init__(self, nk, n_ao, nv, nc, n_aux, eps_qp, psi, C, Vbar, W_q, alpha=2.0, prec="f64",
                 max_nb=8, check_hermitian=False, all_pairs=False, conduction=None, two_centre=None):
        """C: k-independent LRI coefficients (device c128 [n_aux][n_ao][n_ao]), or None with
        two_centre = (C_R, RC, k_frac): real two-centre coefficients C^mu_st(R) (device f64
        [n_RC][n_aux][n_ao][n_ao]), their lattice vectors (int [n_RC][3]) and the fractional k of the
        valence and of the conduction bands ([2][Nk][3])."""
        self.nk = tuple(int(x) for x in nk)
        self.Nk = int(np.prod(self.nk))
        self.n_ao, self.nv, self.nc, self.n_aux = int(n_ao), int(nv), int(nc), int(n_aux)
        self.N = self.Nk * self.nv * self.nc
        self.prec, self.max_nb, self.alpha = prec, int(max_nb), float(alpha)
        self.device = psi.device
        d = _Dims((ctypes.c_int32 * 3)(*self.nk), self.n_ao, self.nv, self.nc, self.n_aux, self.alpha)
        nb_ = self.nv + self.nc
        h = ctypes.c_void_p()
        self._ptr = None
        flags = (CHECK_HERMITIAN if check_hermitian else 0) | (ALL_PAIRS if all_pairs else 0) | CONDUCTION[conduction]
        self.two_centre = two_centre is not None
        if two_centre is None:
            s = lib().bse_plan_create(
                ctypes.byref(d),
                _dev(eps_qp, torch.float64, (self.Nk, nb_), "eps_qp"),
                _dev(psi, torch.complex128, (self.Nk, nb_, self.n_ao), "psi"),
                _dev(C, torch.complex128, (self.n_aux, self.n_ao, self.n_ao), "C"),
                _dev(Vbar, torch.complex128, (self.n_aux, self.n_aux), "Vbar"),
                _dev(W_q, torch.complex128, (self.Nk, self.n_aux, self.n_aux), "W_q"),
                PREC[prec], self.max_nb, flags, _stream(self.device), ctypes.byref(h))
            _check("bse_plan_create", s)
        else:
            if C is not None:
                raise ValueError("give either C or two_centre")
            C_R, RC, kf = two_centre
            RC = _host(RC, np.int32).reshape(-1, 3)
            kf = _host(kf, np.float64, (2, self.Nk, 3))
            s = lib().bse_plan_create_2c(
                ctypes.byref(d),
                _dev(eps_qp, torch.float64, (self.Nk, nb_), "eps_qp"),
                _dev(psi, torch.complex128, (self.Nk, nb_, self.n_ao), "psi"),
                len(RC), RC.ctypes.data,
                _dev(C_R, torch.float64, (len(RC), self.n_aux, self.n_ao, self.n_ao), "C_R"),
                kf.ctypes.data,
                _dev(Vbar, torch.complex128, (self.n_aux, self.n_aux), "Vbar"),
                _dev(W_q, torch.complex128, (self.Nk, self.n_aux, self.n_aux), "W_q"),
                PREC[prec], self.max_nb, flags, _stream(self.device), ctypes.byref(h))
            _check("bse_plan_create_2c", s)
        self._ptr = h

    def close(self):
        if self._ptr is not None and _lib is not None:
            _lib.bse_plan_destroy(self._ptr)
        self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def pairs(self):
        """(q whose direct blocks an apply forms, N_k): about N_k / 2 under the pair symmetry."""
        f, t = ctypes.c_int64(), ctypes.c_int64()
        _check("bse_plan_pairs", lib().bse_plan_pairs(self._ptr, ctypes.byref(f), ctypes.byref(t)))
        return int(f.value), int(t.value)

    @property
    def conduction(self):
        """'mc' when the direct term forms the conduction pair densities, 'u' for the B_c(k) contraction."""
        v = ctypes.c_int32()
        _check("bse_plan_conduction", lib().bse_plan_conduction(self._ptr, ctypes.byref(v)))
        return "mc" if v.value else "u"

    @property
    def fused(self):
        """True when an apply forms the W step and the direct block in one kernel (P kept on chip)."""
        v = ctypes.c_int32()
        _check("bse_plan_fused", lib().bse_plan_fused(self._ptr, ctypes.byref(v)))
        return bool(v.value)

    @property
    def frag(self):
        """True when the plan keeps its BF16x3 halves in the pair-density kernel's fragment order."""
        v = ctypes.c_int32()
        _check("bse_plan_frag", lib().bse_plan_frag(self._ptr, ctypes.byref(v)))
        return bool(v.value)

    @property
    def bytes(self):
        v = ctypes.c_uint64()
        _check("bse_plan_bytes", lib().bse_plan_bytes(self._ptr, ctypes.byref(v)))
        return int(v.value)

    def set_R(self, R, w_R):
        R = _host(R, np.int32).reshape(-1, 3)
        w_R = _host(w_R, np.float64, (len(R),))
        self._R, self._wR = R, w_R
        _check("bse_plan_set_R", lib().bse_plan_set_R(self._ptr, len(R), R.ctypes.data, w_R.ctypes.data))

    def set_eps(self, eps_qp):
        _check("bse_plan_set_eps", lib().bse_plan_set_eps(
            self._ptr, _dev(eps_qp, torch.float64, (self.Nk, self.nv + self.nc), "eps_qp"), _stream(self.device)))

    def apply(self, X, out=None):
        """Y = A X for X [N][nb] complex128 on the device."""
        nb = X.shape[1]
        Y = torch.empty_like(X) if out is None else out
        s = lib().bse_apply(self._ptr, _dev(X, torch.complex128, (self.N, nb), "X"),
                            _dev(Y, torch.complex128, (self.N, nb), "Y"), nb, _stream(self.device))
        _check("bse_apply", s)
        return Y

    def apply_coupling(self, X, out=None):
        """Y = B X (coupling block of the full BSE) for X [N][nb] complex128 on the device."""
        nb = X.shape[1]
        Y = torch.empty_like(X) if out is None else out
        s = lib().bse_apply_coupling(self._ptr, _dev(X, torch.complex128, (self.N, nb), "X"),
                                     _dev(Y, torch.complex128, (self.N, nb), "Y"), nb, _stream(self.device))
        _check("bse_apply_coupling", s)
        return Y

    def apply_full(self, XY, out=None):
        """[[A, B], [-B*, -A*]] [X; Y] for XY [2N][nb] (X rows first); needs 2 nb <= max_nb."""
        nb = XY.shape[1]
        R = torch.empty_like(XY) if out is None else out
        s = lib().bse_apply_full(self._ptr, _dev(XY, torch.complex128, (2 * self.N, nb), "XY"),
                                 _dev(R, torch.complex128, (2 * self.N, nb), "out"), nb, _stream(self.device))
        _check("bse_apply_full", s)
        return R

    def full_spectrum(self, P, n_steps, omega, eta):
        """Full-BSE spectrum of the columns of P over the positive excitations (structure-preserving
        Lanczos, n_steps steps); returns S [nb][n_w], a, b, steps, breakdown."""
        nb = P.shape[1]
        omega = _host(omega, np.float64).ravel()
        S = np.zeros((nb, len(omega)))
        a = np.zeros((nb, n_steps))
        b = np.zeros((nb, n_steps + 1))
        steps = np.zeros(nb, dtype=np.int32)
        s = lib().bse_full_spectrum(self._ptr, _dev(P, torch.complex128, (self.N, nb), "P"), nb, int(n_steps),
                                    omega.ctypes.data, len(omega), float(eta), S.ctypes.data, a.ctypes.data,
                                    b.ctypes.data, steps.ctypes.data, _stream(self.device))
        _check("bse_full_spectrum", s, allow_breakdown=True)
        return {"S": S, "a": a, "b": b, "steps": steps, "breakdown": s == BSE_INFO_BREAKDOWN}

    def full_lowest(self, n_block=2, max_iter=200, tol=1e-10, X0=None, want_vectors=True, allow_unconverged=False):
        """Smallest positive full-BSE excitations: (omega ascending, [X; Y] [2N][n_block] with
        X^H X - Y^H Y = 1, iterations)."""
        omega = np.zeros(n_block)
        iters = np.zeros(1, dtype=np.int32)
        z = torch.empty((2 * self.N, n_block), dtype=torch.complex128, device=self.device) if want_vectors else None
        s = lib().bse_full_lowest(self._ptr, n_block, max_iter, tol,
                                  _dev(X0, torch.complex128, (2 * self.N, n_block), "X0") if X0 is not None else None,
                                  omega.ctypes.data, _dev(z, torch.complex128, None, "xy") if want_vectors else None,
                                  iters.ctypes.data, _stream(self.device))
        if not (allow_unconverged and s == BSE_INFO_NOT_CONVERGED):
            _check("bse_full_lowest", s)
        return omega, z, int(iters[0])

    def apply_adjoint(self, Ybar, X, want_WR=True, want_Wq=False, want_eps=True):
        """Gradients of Re <Ybar, A X> w.r.t. W(R) (or W(q)) and the energies."""
        nb = X.shape[1]
        gWR = torch.empty((len(self._wR), self.n_aux, self.n_aux), dtype=torch.complex128,
                          device=self.device) if want_WR else None
        gWq = torch.empty((self.Nk, self.n_aux, self.n_aux), dtype=torch.complex128,
                          device=self.device) if want_Wq else None
        geps = torch.empty((self.Nk, self.nv + self.nc), dtype=torch.float64,
                           device=self.device) if want_eps else None
        s = lib().bse_apply_adjoint(
            self._ptr, _dev(Ybar, torch.complex128, (self.N, nb), "Ybar"),
            _dev(X, torch.complex128, (self.N, nb), "X"), nb,
            _dev(gWR, torch.complex128, None, "g_WR") if want_WR else None,
            _dev(gWq, torch.complex128, None, "g_Wq") if want_Wq else None,
            _dev(geps, torch.float64, None, "g_eps") if want_eps else None, _stream(self.device))
        _check("bse_apply_adjoint", s)
        return {"W_R": gWR, "W_q": gWq, "eps": geps}

    STAGES = ("pairdens_v", "wstep", "dblock", "tx", "exchange", "diag", "lanczos", "adjoint", "pairdens_c",
              "tables", "coupling")

    def set_timing(self, enable=True):
        _check("bse_plan_set_timing", lib().bse_plan_set_timing(self._ptr, 1 if enable else 0))

    def stage_times(self, reset=True):
        """{stage: (milliseconds, launches)} accumulated since the last reset (synchronises)."""
        ms = np.zeros(len(self.STAGES))
        n = np.zeros(len(self.STAGES), dtype=np.int64)
        _check("bse_plan_stage_times", lib().bse_plan_stage_times(self._ptr, ms.ctypes.data, n.ctypes.data,
                                                                   1 if reset else 0))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.STAGES)}

    def velocity_start(self, vel, eps_ks, pol):
        pol = _host(pol, np.float64).reshape(-1, 3)
        nb = len(pol)
        P = torch.empty((self.N, nb), dtype=torch.complex128, device=self.device)
        s = lib().bse_velocity_start(self._ptr, _dev(vel, torch.complex128, (3, self.Nk, self.nc, self.nv), "vel"),
                                     _dev(eps_ks, torch.float64, (self.Nk, self.nv + self.nc), "eps_ks"), nb,
                                     pol.ctypes.data, _dev(P, torch.complex128, None, "P"), _stream(self.device))
        _check("bse_velocity_start", s)
        return P

    def density_start(self, psi):
        """<c k+Q| e^{iQ.r} |v k> for the plan's band arrays (conduction bands at k + Q): [N][1]."""
        P = torch.empty((self.N, 1), dtype=torch.complex128, device=self.device)
        s = lib().bse_density_start(self._ptr, _dev(psi, torch.complex128, (self.Nk, self.nv + self.nc, self.n_ao),
                                                    "psi"), _dev(P, torch.complex128, None, "P"),
                                    _stream(self.device))
        _check("bse_density_start", s)
        return P

    def haydock(self, P, n_steps, omega, eta, keep_basis=False):
        nb = P.shape[1]
        omega = _host(omega, np.float64).ravel()
        S = np.zeros((nb, len(omega)))
        a = np.zeros((nb, n_steps))
        b = np.zeros((nb, n_steps + 1))
        steps = np.zeros(nb, dtype=np.int32)
        basis = torch.empty((nb, n_steps, self.N), dtype=torch.complex128, device=self.device) if keep_basis else None
        s = lib().bse_haydock_spectrum(self._ptr, _dev(P, torch.complex128, (self.N, nb), "P"), nb, int(n_steps),
                                       omega.ctypes.data, len(omega), float(eta), S.ctypes.data, a.ctypes.data,
                                       b.ctypes.data, steps.ctypes.data,
                                       _dev(basis, torch.complex128, None, "basis") if keep_basis else None,
                                       _stream(self.device))
        _check("bse_haydock_spectrum", s, allow_breakdown=True)
        return {"S": S, "a": a, "b": b, "steps": steps, "basis": basis, "breakdown": s == BSE_INFO_BREAKDOWN}

    def lowest_excitons(self, n_block=4, max_iter=200, tol=1e-10, X0=None, want_vectors=True,
                        allow_unconverged=False):
        """Lowest n_block eigenpairs by block LOBPCG: (omega ascending, x [N][n_block], iterations)."""
        omega = np.zeros(n_block)
        iters = np.zeros(1, dtype=np.int32)
        x = torch.empty((self.N, n_block), dtype=torch.complex128, device=self.device) if want_vectors else None
        s = lib().bse_lowest_excitons(self._ptr, n_block, max_iter, tol,
                                      _dev(X0, torch.complex128, (self.N, n_block), "X0") if X0 is not None else None,
                                      omega.ctypes.data, _dev(x, torch.complex128, None, "x") if want_vectors else None,
                                      iters.ctypes.data, _stream(self.device))
        if not (allow_unconverged and s == BSE_INFO_NOT_CONVERGED):
            _check("bse_lowest_excitons", s)
        return omega, x, int(iters[0])

    def haydock_vjp(self, hay, omega, eta, gamma, want_WR=True, want_Wq=False, want_eps=True):
        """Gradient of sum gamma[b][w] S_b(w) through a Haydock run made with keep_basis=True."""
        if hay.get("basis") is None:
            raise ValueError("haydock_vjp needs the Lanczos basis (haydock(..., keep_basis=True))")
        basis = hay["basis"]
        nb, m, _ = basis.shape
        omega = _host(omega, np.float64).ravel()
        gamma = _host(gamma, np.float64, (nb, len(omega)))
        a = _host(hay["a"], np.float64, (nb, m))
        b = _host(hay["b"], np.float64, (nb, m + 1))
        steps = _host(hay["steps"], np.int32, (nb,))
        gWR = torch.empty((len(self._wR), self.n_aux, self.n_aux), dtype=torch.complex128,
                          device=self.device) if want_WR else None
        gWq = torch.empty((self.Nk, self.n_aux, self.n_aux), dtype=torch.complex128,
                          device=self.device) if want_Wq else None
        geps = torch.empty((self.Nk, self.nv + self.nc), dtype=torch.float64, device=self.device) if want_eps else None
        s = lib().bse_haydock_vjp(self._ptr, _dev(basis, torch.complex128, None, "basis"), a.ctypes.data,
                                  b.ctypes.data, steps.ctypes.data, nb, m, omega.ctypes.data, len(omega),
                                  float(eta), gamma.ctypes.data,
                                  _dev(gWR, torch.complex128, None, "g_WR") if want_WR else None,
                                  _dev(gWq, torch.complex128, None, "g_Wq") if want_Wq else None,
                                  _dev(geps, torch.float64, None, "g_eps") if want_eps else None,
                                  _stream(self.device))
        _check("bse_haydock_vjp", s)
        return {"W_R": gWR, "W_q": gWq, "eps": geps}


def offset_set():
    """The paper's k-offsets (units of the dense-mesh spacing) and weights: ([4][3], [4])."""
    n = ctypes.c_int32()
    off, w = np.zeros((4, 3)), np.zeros(4)
    _check("bse_offset_set", lib().bse_offset_set(ctypes.byref(n), off.ctypes.data, w.ctypes.data))
    return off[:n.value], w[:n.value]


def offset_spectrum(plans, Ps, weights, n_steps, omega, eta):
    """sum_j weights[j] * (Haydock spectrum of plans[j] from start block Ps[j]): k-offset averaging."""
    n = len(plans)
    if len(Ps) != n or len(weights) != n:
        raise ValueError("offset_spectrum: one start block and one weight per plan")
    nb = Ps[0].shape[1]
    omega = _host(omega, np.float64).ravel()
    weights = _host(weights, np.float64, (n,))
    S = np.zeros((nb, len(omega)))
    steps = np.zeros((n, nb), dtype=np.int32)
    hp = (ctypes.c_void_p * n)(*[pl._ptr for pl in plans])
    hP = (ctypes.c_void_p * n)(*[_dev(P, torch.complex128, (plans[j].N, nb), "P") for j, P in enumerate(Ps)])
    s = lib().bse_offset_spectrum(hp, hP, weights.ctypes.data, n, nb, int(n_steps), omega.ctypes.data, len(omega),
                                  float(eta), S.ctypes.data, steps.ctypes.data, _stream(plans[0].device))
    _check("bse_offset_spectrum", s, allow_breakdown=True)
    return {"S": S, "steps": steps, "breakdown": s == BSE_INFO_BREAKDOWN}


def plan_from_problem(prob, W_q, prec="f64", max_nb=8, device="cuda:0", check_hermitian=False, all_pairs=False,
                      conduction=None):
    """Build a Plan from a synthetic crystal (inputs copied host -> device); a crystal with two-centre
    coefficients (prob.C_R) gets a two-centre plan with the k of its valence and conduction bands."""
    dev = torch.device(device)
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
    if getattr(prob, "C_R", None) is not None:
        C, tc = None, (t(prob.C_R, torch.float64), prob.RC, np.stack(prob.band_k()))
    else:
        C, tc = t(prob.C, torch.complex128), None
    return Plan(prob.nk, prob.n_ao, prob.nv, prob.nc, prob.n_aux, t(prob.eps_qp, torch.float64),
                t(prob.psi, torch.complex128), C, t(prob.Vbar, torch.complex128),
                W_q, alpha=prob.alpha, prec=prec, max_nb=max_nb, check_hermitian=check_hermitian,
                all_pairs=all_pairs, conduction=conduction, two_centre=tc)
