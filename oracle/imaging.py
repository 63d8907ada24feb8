"""Imaging utilities of the paper's appendices, FP64 (App. A and B).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* natural-weight dirty image (Eq. dirty) and PSF (Eq. PSF), with the
  normalised weights omega_k = w_k / sum w:
      I^D(X) = Re sum_k omega_k V^o_k e^{+2 pi i U_k . X},
      PSF(X) = sum_k omega_k cos(2 pi U_k . X)
  (R18: the 2 pi of the exponent also in the cosine), no attenuation;
* thermal noise sigma_D = 1 / sqrt(sum_k w_k) (App. B);
* the clean beam: an elliptical Gaussian fitted to the PSF's main lobe
  (App. A leaves the fit open; reading taken: the pixels with PSF >= 1/2
  connected to the centre pixel through edge neighbours, least squares of
  -ln PSF as a quadratic form in the pixel offsets, the peak being 1).
  BMAJ, BMIN are the FWHM along the axes; BPA is the angle of the major axis
  from +y towards +x in degrees, in (-90, 90].
"""
from __future__ import annotations

import math

import numpy as np
import scipy.ndimage

from . import adjoint


def dirty_and_psf(n, cell, chans):
    """chans: dicts with u, v, vis, w (one image seen by all of them)."""
    wsum = sum(float(np.sum(np.asarray(c["w"], np.float64))) for c in chans)
    dirty = np.zeros((n, n))
    psf = np.zeros((n, n))
    for c in chans:
        w = np.asarray(c["w"], np.float64)
        dirty += adjoint(n, cell, c["u"], c["v"], None, w * np.asarray(c["vis"], np.complex128))
        psf += adjoint(n, cell, c["u"], c["v"], None, w.astype(np.complex128))
    return dirty / wsum, psf / wsum


def sigma_d(chans) -> float:
    return 1.0 / math.sqrt(sum(float(np.sum(np.asarray(c["w"], np.float64))) for c in chans))


def fit_beam(psf, cell):
    """(bmaj, bmin, bpa) of the elliptical Gaussian fitted to the main lobe."""
    psf = np.asarray(psf, np.float64)
    n = psf.shape[0]
    c0 = n // 2
    lab, _ = scipy.ndimage.label(psf >= 0.5)
    lobe = (lab == lab[c0, c0]) & (lab > 0)
    lobe[c0, c0] = False
    ii, jj = np.nonzero(lobe)
    dx, dy = (jj - c0).astype(np.float64), (ii - c0).astype(np.float64)
    X = np.stack([dx * dx, dx * dy, dy * dy], axis=1)
    coef, *_ = np.linalg.lstsq(X, -np.log(psf[ii, jj]), rcond=None)
    A, B, C = coef
    evals, evecs = np.linalg.eigh(np.array([[A, B / 2], [B / 2, C]]))
    lmin, lmax = evals
    ex, ey = evecs[:, 0]
    bmaj = 2.0 * math.sqrt(math.log(2.0) / lmin) * cell
    bmin = 2.0 * math.sqrt(math.log(2.0) / lmax) * cell
    ang = math.degrees(math.atan2(ex, ey))
    while ang > 90.0:
        ang -= 180.0
    while ang <= -90.0:
        ang += 180.0
    return bmaj, bmin, ang
