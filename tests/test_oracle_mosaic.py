"""Pins of the oracle's mosaic objective (one image, several pointings, each
with its attenuation image centred on its field and its own phase-tracking
centre; Sec. 1 mosaic support, Sec. 2.4 items 1 and 3).

Checked against: the C oracle's beam, a point source at a pointing centre
(whose visibilities are the constant flux exactly), the shared-image
objective when every centre is at the origin, brute-force finite
differences with two pointings, and the CG reaching the L-BFGS-B minimum.
"""
import numpy as np
import scipy.optimize

import oracle
from oracle import cg as ocg
from paper_1703_02920_amd import synth


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _pointing(n, cell, nvis, seed, fwhm, x0, y0):
    u, v, vis, w = synth.random_problem(n, nvis, seed, cell=cell)
    return dict(u=u, v=v, vis=vis, w=w, x0=x0, y0=y0, A=oracle.beam_at(n, cell, fwhm, x0, y0))


def test_beam_at_origin_is_the_c_beam_and_shifts_by_whole_pixels():
    n, cell, fw = 32, 1e-6, 9e-6
    assert np.allclose(oracle.beam_at(n, cell, fw, 0.0, 0.0), oracle.beam(n, cell, fw), rtol=1e-14, atol=0)
    sh = oracle.beam_at(n, cell, fw, 3 * cell, -2 * cell)
    ref = np.roll(np.roll(oracle.beam(n, cell, fw), 3, axis=1), -2, axis=0)
    assert np.allclose(sh[4:-4, 4:-4], ref[4:-4, 4:-4], rtol=1e-12, atol=0)


def test_point_source_at_a_pointing_centre_gives_the_flux():
    """A pixel of flux F at the pointing centre: the beam is 1 there and the
    phase is measured from there, so V_k = F for every k of that pointing."""
    n, cell = 16, 2e-6
    x0, y0 = 5 * cell, -3 * cell
    p = _pointing(n, cell, 70, 40, 6 * cell, x0, y0)
    I = np.zeros((n, n))
    I[n // 2 - 3, n // 2 + 5] = 0.75
    out = oracle.phi_grad_mosaic(n, cell, [p], I, 1.0, 0.0)
    assert np.allclose(out["V"], 0.75, rtol=0, atol=1e-14)


def test_centres_at_origin_reduce_to_shared_image():
    n, cell = 16, 2e-6
    ps = [_pointing(n, cell, 60, 41, 8 * cell, 0.0, 0.0), _pointing(n, cell, 45, 42, 5 * cell, 0.0, 0.0)]
    img = synth.random_image(n, 41, lo=0.05, hi=1.0)[0]
    a = oracle.phi_grad_mosaic(n, cell, ps, img, 1e-2, 0.2)
    b = oracle.phi_grad_shared(n, cell, ps, img, 1e-2, 0.2)
    assert abs(a["phi"] - b["phi"]) <= 1e-14 * abs(b["phi"])
    assert rel(a["grad"], b["grad"]) < 1e-14


def test_mosaic_gradient_matches_central_differences_two_pointings():
    n, cell = 8, 4e-6
    ps = [_pointing(n, cell, 50, 43, 3 * cell, 1.5 * cell, -1.0 * cell),
          _pointing(n, cell, 40, 44, 4 * cell, -2.0 * cell, 0.5 * cell)]
    img = synth.random_image(n, 43, lo=0.05, hi=1.0)[0]
    M, lam = 1e-2, 0.3
    out = oracle.phi_grad_mosaic(n, cell, ps, img, M, lam)
    fd = np.zeros((n, n))
    for pix in range(n * n):
        i, j = divmod(pix, n)
        h = 1e-4 * img[i, j]
        a = img.copy(); a[i, j] += h
        b = img.copy(); b[i, j] -= h
        fd[i, j] = (oracle.phi_grad_mosaic(n, cell, ps, a, M, lam)["phi"]
                    - oracle.phi_grad_mosaic(n, cell, ps, b, M, lam)["phi"]) / (2 * h)
    assert rel(out["grad"], fd) < 1e-7


def test_mosaic_problem_matches_objective_and_reaches_minimum():
    n, cell = 8, 4e-6
    ps = [_pointing(n, cell, 60, 45, 4 * cell, 1.0 * cell, 1.0 * cell),
          _pointing(n, cell, 60, 46, 4 * cell, -1.5 * cell, -0.5 * cell)]
    prob = ocg.MosaicProblem(n, cell, ps, 1e-2, 0.05)
    img = synth.random_image(n, 45, lo=0.05, hi=1.0)[0]
    ev, ref = prob.evaluate(img), oracle.phi_grad_mosaic(n, cell, ps, img, 1e-2, 0.05)
    assert abs(ev["phi"] - ref["phi"]) < 1e-13 * abs(ref["phi"]) and rel(ev["g"], ref["grad"]) < 1e-13
    I, traj = ocg.projected_cg(prob, 300)
    phis = [t["phi"] for t in traj]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(phis, phis[1:]))

    def fun(x):
        e = prob.evaluate(x.reshape(n, n))
        return e["phi"], e["g"].ravel()

    opt = scipy.optimize.minimize(fun, np.full(n * n, 0.1), jac=True, method="L-BFGS-B",
                                  bounds=[(prob.M, None)] * (n * n),
                                  options=dict(maxiter=5000, ftol=1e-15, gtol=1e-12))
    phi_cg = prob.evaluate(I)["phi"]
    assert phi_cg <= opt.fun + 1e-8 * abs(opt.fun)
    assert abs(phi_cg - opt.fun) < 1e-7 * abs(opt.fun)
