"""Pins of the oracle's imaging utilities (App. A dirty image, PSF and clean
beam; App. B thermal noise) and of the focus-of-attention CG (Sec. 6).

Checked against: the PSF's value and symmetry, a point-source data set whose
dirty image is the flux times the PSF, a library FFT on grid-aligned uv,
a Monte Carlo estimate of the dirty image's noise, exact elliptical
Gaussians whose parameters the fit must return, and a CG whose fixed pixels
must not move while the free ones reach the bound-constrained minimum of
the reduced problem.
"""
import math

import numpy as np
import pytest
import scipy.optimize

import oracle
from oracle import cg as ocg
from oracle import imaging as oim
from paper_1703_02920_amd import synth

N, CELL = 32, 1.0e-6


def _chans(seed, sizes=(150, 90)):
    out = []
    for k, z in enumerate(sizes):
        u, v, vis, w = synth.random_problem(N, z, seed + k, cell=CELL)
        out.append(dict(u=u, v=v, vis=vis, w=w))
    return out


def test_psf_is_one_at_the_centre_and_symmetric():
    _, psf = oim.dirty_and_psf(N, CELL, _chans(70))
    c0 = N // 2
    assert abs(psf[c0, c0] - 1.0) < 1e-14
    a = psf[c0 - 10:c0 + 11, c0 - 10:c0 + 11]
    assert np.allclose(a, a[::-1, ::-1], rtol=0, atol=1e-14)


def test_point_source_data_dirty_image_is_flux_times_psf():
    ch = _chans(71)
    for c in ch:
        c["vis"] = np.full(len(c["u"]), 0.6 + 0j)
    d, p = oim.dirty_and_psf(N, CELL, ch)
    assert np.allclose(d, 0.6 * p, rtol=0, atol=1e-14)


def test_psf_on_grid_aligned_uv_matches_numpy_fft():
    """u = p du, v = q du (du = 1/(N dx)): PSF_ij = sum omega cos(2 pi (p (j - N/2) + q (i - N/2)) / N)
    equals the real part of N^2 ifft2 of the grid of weights times (-1)^(p+q)
    (the phase centre at pixel N/2 shifts each frequency's phase by pi (p+q))."""
    rng = np.random.default_rng(72)
    p = rng.integers(-N // 2, N // 2, 300)
    q = rng.integers(-N // 2, N // 2, 300)
    w = rng.uniform(0.5, 2.0, 300)
    du = 1.0 / (N * CELL)
    _, psf = oim.dirty_and_psf(N, CELL, [dict(u=p * du, v=q * du, vis=np.zeros(300), w=w)])
    Wg = np.zeros((N, N))
    np.add.at(Wg, (q % N, p % N), w * (-1.0) ** (p + q))
    ref = np.real(np.fft.ifft2(Wg)) * N * N
    assert np.allclose(psf, ref / w.sum(), rtol=0, atol=1e-13)


def test_dirty_image_noise_matches_sigma_d_monte_carlo():
    """Noise-only data, Re and Im ~ N(0, 1/w_k): the dirty image's variance at
    any pixel is 1 / sum w (App. B)."""
    ch = _chans(73, sizes=(120,))[0]
    w = ch["w"].astype(np.float64)
    rng = np.random.default_rng(74)
    pix = np.array([N // 2 * N + N // 2, 3 * N + 7, 20 * N + 29])
    samples = []
    for _ in range(3000):
        vis = (rng.standard_normal(len(w)) + 1j * rng.standard_normal(len(w))) / np.sqrt(w)
        samples.append(oracle.adjoint(N, CELL, ch["u"], ch["v"], None, w * vis, pix=pix) / w.sum())
    var = np.var(np.array(samples), axis=0)
    sd2 = oim.sigma_d([ch]) ** 2
    assert np.all(np.abs(var / sd2 - 1.0) < 0.1), var / sd2


@pytest.mark.parametrize("bpa", [0.0, 30.0, -60.0, 89.0])
def test_beam_fit_recovers_an_exact_elliptical_gaussian(bpa):
    n, cell = 64, 2e-6
    bmaj, bmin = 9.3 * cell, 4.1 * cell
    yy, xx = (np.mgrid[0:n, 0:n] - n // 2).astype(np.float64) * cell
    t = math.radians(bpa)
    # major axis along (sin t, cos t): angle t from +y towards +x
    a = xx * math.sin(t) + yy * math.cos(t)
    b = xx * math.cos(t) - yy * math.sin(t)
    psf = np.exp(-4 * math.log(2) * (a * a / bmaj ** 2 + b * b / bmin ** 2))
    fa, fb, fp = oim.fit_beam(psf, cell)
    assert abs(fa / bmaj - 1) < 1e-9 and abs(fb / bmin - 1) < 1e-9
    assert abs(((fp - bpa + 90) % 180) - 90) < 1e-7


def test_focus_of_attention_cg_keeps_fixed_pixels_and_minimises_the_rest():
    n, cell = 8, 4e-6
    u, v, vis, w = synth.random_problem(n, 90, 75, cell=cell)
    A = oracle.beam(n, cell, 6 * cell)
    prob = ocg.Problem(n, cell, u, v, vis, w, A, 1e-2, 0.05)
    free = np.zeros((n, n), bool)
    free[2:6, 1:7] = True
    I, traj = ocg.projected_cg(prob, 300, free=free)
    assert np.all(I[~free] == prob.M)
    phis = [t["phi"] for t in traj]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(phis, phis[1:]))

    def fun(x):
        J = np.full((n, n), prob.M)
        J[free] = x
        e = prob.evaluate(J)
        return e["phi"], e["g"][free]

    opt = scipy.optimize.minimize(fun, np.full(int(free.sum()), 0.1), jac=True, method="L-BFGS-B",
                                  bounds=[(prob.M, None)] * int(free.sum()),
                                  options=dict(maxiter=5000, ftol=1e-15, gtol=1e-12))
    phi_cg = prob.evaluate(I)["phi"]
    assert abs(phi_cg - opt.fun) < 1e-7 * abs(opt.fun)
