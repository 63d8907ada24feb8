"""Gridded forward model of the paper's GPU objective (Sec. 2.4, Alg. 1), FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper approximates the model visibilities by
  1. attenuation      B = A o I                                   (item 1)
  2. 2-D DFT          V^F = F_2D{B} on the uniform uv grid         (item 2)
  3. modulation       Vhat^F(u, v) = V^F(u, v) exp{2 pi i (u x_c + v y_c)}
                      (the phase-tracking centre, item 3)
  4. bilinear interpolation of Vhat^F at (u_k / du, v_k / dv)     (item 4)
and then forms the residuals as before.  Written here in that order with the
geometry of the exact model: pixel (i, j) at x_j = (j - N/2) dx,
y_i = (i - N/2) dx, so (x_c, y_c) is pixel (N/2, N/2).  The image may be
zero-padded to Ng = s N before the transform (s = 1 is the paper's grid;
a finer Fourier grid is the paper's remedy for aliasing): du = 1/(Ng dx).
Grid index p covers frequency p du for p < Ng/2 and (p - Ng) du above
(the FFT's periodic layout); interpolation wraps modulo Ng.

gridded_adjoint is the exact adjoint (transpose, real part) of that linear
map, in reverse order: the transposed bilinear interpolation scatters each
coefficient onto its four grid nodes, the conjugate modulation and the
inverse (unnormalised, e^{+}) 2-D DFT bring it back to the padded image, the
first N rows and columns are kept, and the real part is multiplied by A.
"""
from __future__ import annotations

import numpy as np


def _grid_coords(u, v, cell, Ng):
    """Fractional grid coordinates (u_k / du, v_k / du) = (u_k dx Ng, v_k dx Ng),
    the lower grid node (mod Ng) and the bilinear fractions."""
    gx = np.asarray(u, np.float64) * cell * Ng
    gy = np.asarray(v, np.float64) * cell * Ng
    px, py = np.floor(gx), np.floor(gy)
    fx, fy = gx - px, gy - py
    return (px.astype(np.int64) % Ng, py.astype(np.int64) % Ng, fx, fy)


def _modulation(N, Ng):
    """exp{+2 pi i (p + q)(N/2)/Ng} over grid indices (q rows, p columns):
    the phase centre at pixel N/2 of both axes.  N/2 is an integer, so the
    factor is the same for p and p - Ng."""
    k = np.arange(Ng)
    ph = np.exp(2j * np.pi * k * (N // 2) / Ng)
    return ph[:, None] * ph[None, :]


def grid_spectrum(n, A, I, oversample=1):
    """Steps 1-3: Vhat^F on the Ng x Ng grid, rows q (v), columns p (u)."""
    Ng = oversample * n
    B = np.zeros((Ng, Ng))
    B[:n, :n] = (np.ones((n, n)) if A is None else np.asarray(A, np.float64)) * np.asarray(I, np.float64)
    return np.fft.fft2(B) * _modulation(n, Ng)


def gridded_forward(n, cell, u, v, A, I, oversample=1):
    """V^m_k by bilinear interpolation of the modulated grid spectrum (step 4)."""
    Ng = oversample * n
    G = grid_spectrum(n, A, I, oversample)
    px, py, fx, fy = _grid_coords(u, v, cell, Ng)
    qx, qy = (px + 1) % Ng, (py + 1) % Ng
    return ((1 - fx) * (1 - fy) * G[py, px] + fx * (1 - fy) * G[py, qx]
            + (1 - fx) * fy * G[qy, px] + fx * fy * G[qy, qx])


def gridded_adjoint(n, cell, u, v, A, c, oversample=1):
    """A o Re(F_grid^H c): the exact adjoint of gridded_forward."""
    Ng = oversample * n
    px, py, fx, fy = _grid_coords(u, v, cell, Ng)
    qx, qy = (px + 1) % Ng, (py + 1) % Ng
    c = np.asarray(c, np.complex128)
    H = np.zeros((Ng, Ng), np.complex128)
    np.add.at(H, (py, px), (1 - fx) * (1 - fy) * c)
    np.add.at(H, (py, qx), fx * (1 - fy) * c)
    np.add.at(H, (qy, px), (1 - fx) * fy * c)
    np.add.at(H, (qy, qx), fx * fy * c)
    H *= np.conj(_modulation(n, Ng))
    img = np.fft.ifft2(H) * (Ng * Ng)
    G = img[:n, :n].real
    return G if A is None else G * np.asarray(A, np.float64)


def gridded_phi_grad(n, cell, u, v, A, I, Vo, w, M, lam, oversample=1, grad="adjoint"):
    """Phi = chi^2 + lambda S with the gridded model visibilities; grad Phi
    from the exact adjoint of the gridded map (grad="adjoint") or from the
    exact-DFT gradient of Eq. chi2gradient at the gridded residuals
    (grad="dft", the paper's combination)."""
    from . import adjoint, chi2, entropy
    V = gridded_forward(n, cell, u, v, A, I, oversample)
    x2, R = chi2(V, Vo, w)
    S, gS = entropy(I, M)
    wR = np.asarray(w, np.float64) * R
    if grad == "adjoint":
        gchi = gridded_adjoint(n, cell, u, v, A, wR, oversample)
    else:
        gchi = adjoint(n, cell, u, v, A, wR)
    return dict(phi=x2 + lam * S, chi2=x2, S=S, grad=gchi + lam * gS, gchi2=gchi, V=V, R=R)
