"""FP64 CPU oracle for non-gridding MEM imaging (Carcamo et al.).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  The heavy sums
live in uvmem_oracle.c (plain direct sums, FP64, compensated); this module
marshals numpy arrays and composes the objective of Eq. phi2/phi3:

    Phi(I) = chi^2(I) + lambda * S(I),
    chi^2  = 1/2 sum_k w_k |V^m_k(I) - V^o_k|^2,          (Eq. phi2)
    S      = sum_p I_p ln(I_p / M),                        (regulariser; its
             gradient ln(I/M) + 1 is Eq. Sgradient)
    grad Phi = A o Re F^H (w o R) + lambda (ln(I/M) + 1)   (Eq. chi2gradient,
             with the beam factor of the exact derivative).

Readings taken where the paper is ambiguous, on which this file depends:
the 1/2 in chi^2 (Eq. phi2), S written with M in place of G and without the
1/G prefactor (so that Eq. Sgradient is its exact gradient), the sign
Phi = chi^2 + lambda S (the paper's S carries the opposite sign), the beam
factor A_ij kept in the chi^2 gradient, and, for one image fitted to several
channels, the entropy term counted once (Eq. chi2-multi sums only chi^2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uvmem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_beam.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        L.or_forward.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, dp, dp, dp, dp]
        L.or_forward_sel.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, i64p,
                                     dp, dp, dp, dp, dp]
        L.or_adjoint.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, dp, dp, dp,
                                 ctypes.c_int64, i64p, dp]
        L.or_forward_pix.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, dp, dp,
                                     ctypes.c_int64, i64p, dp, dp]
        L.or_chi2.argtypes = [ctypes.c_int64, dp, dp, dp, dp]
        L.or_chi2.restype = ctypes.c_double
        L.or_entropy.argtypes = [ctypes.c_int64, dp, ctypes.c_double, dp]
        L.or_entropy.restype = ctypes.c_double
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _cplx(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def beam(n: int, cell: float, fwhm: float) -> np.ndarray:
    """A_ij = exp(-4 ln 2 (x_j^2 + y_i^2) / FWHM^2) (Sec. 2.4, item 1)."""
    A = np.empty((n, n))
    lib().or_beam(n, cell, fwhm, _d(A))
    return A


def forward(n: int, cell: float, u, v, A: Optional[np.ndarray], I) -> np.ndarray:
    """V^m_k = sum_ij A_ij I_ij exp(-2 pi i (u_k x_j + v_k y_i)) (Eq. fft)."""
    u, v, I = _f64(u), _f64(v), _f64(I)
    assert I.shape == (n, n)
    Ak = None if A is None else _f64(A)
    V = np.empty(u.shape[0], dtype=np.complex128)
    lib().or_forward(n, cell, u.shape[0], _d(u), _d(v), _d(Ak) if Ak is not None else None,
                     _d(I), _d(V.view(np.float64)))
    return V


def forward_sel(n: int, cell: float, idx, u, v, A, I) -> np.ndarray:
    """Forward model at the listed visibility indices only."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    u, v, I = _f64(u), _f64(v), _f64(I)
    Ak = None if A is None else _f64(A)
    V = np.empty(idx.shape[0], dtype=np.complex128)
    lib().or_forward_sel(n, cell, idx.shape[0], idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         _d(u), _d(v), _d(Ak) if Ak is not None else None, _d(I),
                         _d(V.view(np.float64)))
    return V


def forward_pix(n: int, cell: float, u, v, A: Optional[np.ndarray], pix, vals) -> np.ndarray:
    """Forward model (Eq. fft) of an image that is zero except vals[q] at
    linear pixel pix[q]: V_k = sum_q A[pix_q] vals_q exp(-2 pi i (u_k x + v_k y))."""
    u, v = _f64(u), _f64(v)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    vals = _f64(vals)
    assert pix.shape == vals.shape and pix.ndim == 1
    Ak = None if A is None else _f64(A)
    V = np.empty(u.shape[0], dtype=np.complex128)
    lib().or_forward_pix(n, cell, u.shape[0], _d(u), _d(v), _d(Ak) if Ak is not None else None,
                         pix.shape[0], pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _d(vals),
                         _d(V.view(np.float64)))
    return V


def phi_at_pixel_steps(n, cell, u, v, A, I, V_I, Vo, w, M, lam, pix, h):
    """Phi (Eq. phi3) at the images I + h_q e_{p_q}, one pixel changed at a
    time, for q = 0..len(pix)-1: the model visibilities are V(I) + h_q V(e_p)
    (the forward model is linear), chi^2 and S are then evaluated from their
    definitions.  V_I = forward(I) is passed in so that it is computed once."""
    I = _f64(I)
    out = np.empty(len(pix))
    for q, (p, hq) in enumerate(zip(pix, h)):
        Vp = forward_pix(n, cell, u, v, A, [p], [hq])
        x2, _ = chi2(V_I + Vp, Vo, w)
        Ip = I.copy()
        Ip.flat[p] += hq
        S, _ = entropy(Ip, M)
        out[q] = x2 + lam * S
    return out


def adjoint(n: int, cell: float, u, v, A: Optional[np.ndarray], c, pix=None) -> np.ndarray:
    """G_ij = A_ij sum_k Re(c_k exp(+2 pi i (u_k x_j + v_k y_i))).

    With c = w * R this is the chi^2 gradient (Eq. chi2gradient, Alg. 3).
    `pix` (optional) lists linear pixel indices N*i + j to evaluate."""
    u, v = _f64(u), _f64(v)
    c = _cplx(c)
    Ak = None if A is None else _f64(A)
    if pix is None:
        G = np.empty((n, n))
        lib().or_adjoint(n, cell, u.shape[0], _d(u), _d(v), _d(Ak) if Ak is not None else None,
                         _d(c.view(np.float64)), -1, None, _d(G))
        return G
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    G = np.empty(pix.shape[0])
    lib().or_adjoint(n, cell, u.shape[0], _d(u), _d(v), _d(Ak) if Ak is not None else None,
                     _d(c.view(np.float64)), pix.shape[0],
                     pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _d(G))
    return G


def chi2(V, Vo, w):
    """chi^2 = 1/2 sum_k w_k |V_k - Vo_k|^2 (Eq. phi2); returns (chi2, R)."""
    V, Vo = _cplx(V), _cplx(Vo)
    w = _f64(w)
    R = np.empty_like(V)
    x = lib().or_chi2(V.shape[0], _d(V.view(np.float64)), _d(Vo.view(np.float64)), _d(w),
                      _d(R.view(np.float64)))
    return float(x), R


def entropy(I, M: float):
    """S = sum I ln(I/M), grad = ln(I/M) + 1 (Eq. Sgradient).  S is NaN if
    any pixel is <= 0."""
    I = _f64(I)
    g = np.empty_like(I)
    s = lib().or_entropy(I.size, _d(I), M, _d(g))
    return float(s), g


def phi_grad(n, cell, u, v, A, I, Vo, w, M, lam):
    """Phi = chi^2 + lambda S and its gradient for one channel (Eq. phi2/phi3,
    Eq. Sgradient, Eq. chi2gradient)."""
    V = forward(n, cell, u, v, A, I)
    x2, R = chi2(V, Vo, w)
    S, gS = entropy(I, M)
    gchi = adjoint(n, cell, u, v, A, _f64(w) * R)
    grad = gchi + lam * gS
    return dict(phi=x2 + lam * S, chi2=x2, S=S, grad=grad, gchi2=gchi, V=V, R=R)


def phi_grad_shared(n, cell, chans, I, M, lam):
    """Phi and grad Phi of ONE image seen by several channels (Eq. chi2-multi).

    chi^2 is the sum over the channels of Eq. phi2, each channel with its own
    (u, v), weights and attenuation image A_c (Sec. 2.4 item 1: one
    attenuation matrix per channel); grad chi^2 is the sum of the channels'
    gradients of Eq. chi2gradient (the per-channel gradients that the
    multi-channel gradient function of Sec. 2.7 adds into one image); S and
    its gradient are counted once.  `chans` is a sequence of dicts with keys
    u, v, A, vis, w."""
    I = _f64(I)
    x2 = 0.0
    gchi = np.zeros((n, n))
    Vs, Rs = [], []
    for ch in chans:
        V = forward(n, cell, ch["u"], ch["v"], ch["A"], I)
        x, R = chi2(V, ch["vis"], ch["w"])
        gchi += adjoint(n, cell, ch["u"], ch["v"], ch["A"], _f64(ch["w"]) * R)
        x2 += x
        Vs.append(V)
        Rs.append(R)
    S, gS = entropy(I, M)
    return dict(phi=x2 + lam * S, chi2=x2, S=S, grad=gchi + lam * gS, gchi2=gchi,
                V=np.concatenate(Vs) if Vs else np.zeros(0, np.complex128),
                R=np.concatenate(Rs) if Rs else np.zeros(0, np.complex128))


def beam_at(n: int, cell: float, fwhm: float, x0: float, y0: float) -> np.ndarray:
    """Gaussian attenuation image centred on a pointing at (x0, y0) radians
    from the image centre (Sec. 2.4 item 1: for a mosaic, each pointing's
    attenuation image is centred on its field)."""
    c = (np.arange(n) - n // 2) * cell
    dx2 = (c - x0) ** 2
    dy2 = (c - y0) ** 2
    return np.exp(-4.0 * np.log(2.0) * (dy2[:, None] + dx2[None, :]) / (fwhm * fwhm))


def phi_grad_mosaic(n, cell, pointings, I, M, lam):
    """One image fitted to several pointings (Sec. 1, mosaic support;
    Sec. 2.4 items 1 and 3).  Pointing p (keys u, v, A, vis, w, x0, y0) sees
    the image through its attenuation image A (centred on its field) with
    its phase-tracking centre at (x0, y0):
        V_k = e^{+2 pi i (u_k x0 + v_k y0)} sum_ij A_ij I_ij e^{-2 pi i (u_k x_j + v_k y_i)}
    (the exponent of Eq. fft measured from the pointing's centre).  chi^2 is
    summed over pointings (as over channels in Eq. chi2-multi); differentiating
    1/2 w |V - V^o|^2 gives the pointing's gradient
        A o Re sum_k w_k R_k e^{-2 pi i (u_k x0 + v_k y0)} e^{+2 pi i (u_k x_j + v_k y_i)},
    the adjoint of the phase-shifted coefficients.  S counted once."""
    I = _f64(I)
    x2 = 0.0
    gchi = np.zeros((n, n))
    Vs, Rs = [], []
    for p in pointings:
        u, v = _f64(p["u"]), _f64(p["v"])
        shift = np.exp(2j * np.pi * (u * p["x0"] + v * p["y0"]))
        V = shift * forward(n, cell, u, v, p["A"], I)
        x, R = chi2(V, p["vis"], p["w"])
        gchi += adjoint(n, cell, u, v, p["A"], _f64(p["w"]) * R * np.conj(shift))
        x2 += x
        Vs.append(V)
        Rs.append(R)
    S, gS = entropy(I, M)
    return dict(phi=x2 + lam * S, chi2=x2, S=S, grad=gchi + lam * gS, gchi2=gchi,
                V=np.concatenate(Vs) if Vs else np.zeros(0, np.complex128),
                R=np.concatenate(Rs) if Rs else np.zeros(0, np.complex128))
