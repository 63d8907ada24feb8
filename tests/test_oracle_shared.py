"""Pins of the oracle's shared-image (multi-frequency) objective, Eq. chi2-multi.

One image is seen by every channel through the channel's own uv, weights and
attenuation image.  Each test checks the oracle against something other than
itself: a closed form with explicit per-channel beams, the single-channel
objective on the same visibilities (a channel split in two is the same data),
brute-force finite differences, and a library bound-constrained minimiser.
"""
import numpy as np
import scipy.optimize

import oracle
from oracle import cg as ocg
from paper_1703_02920_amd import synth


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _chan(n, cell, nvis, seed, fwhm_cells, uv_scale=1.0):
    u, v, vis, w = synth.random_problem(n, nvis, seed, cell=cell)
    return dict(u=u * uv_scale, v=v * uv_scale, vis=vis, w=w, A=oracle.beam(n, cell, fwhm_cells * cell))


def test_point_source_closed_form_per_channel_beams():
    """A single pixel of value a at p, one visibility per channel at
    (u, v) = (0, 0) with V^o = 0 and w = 1: V_c = a A_c[p], so
    chi^2 = 1/2 sum_c a^2 A_c[p]^2 and grad chi^2[q] = a sum_c A_c[q] A_c[p].
    Arbitrary beam images make a beam taken from the wrong channel visible."""
    n, cell = 8, 3.0e-6
    rng = np.random.default_rng(31)
    As = [rng.uniform(0.1, 1.0, (n, n)) for _ in range(3)]
    chans = [dict(u=np.zeros(1), v=np.zeros(1), vis=np.zeros(1, np.complex128), w=np.ones(1), A=A)
             for A in As]
    a, (pi, pj) = 2.5, (3, 6)
    I = np.zeros((n, n))
    I[pi, pj] = a
    out = oracle.phi_grad_shared(n, cell, chans, I, 1.0, 0.0)
    chi2 = 0.5 * sum((a * A[pi, pj]) ** 2 for A in As)
    g = a * sum(A * A[pi, pj] for A in As)
    assert abs(out["chi2"] - chi2) < 1e-13 * chi2
    assert rel(out["gchi2"], g) < 1e-13
    assert np.allclose(out["V"], [a * A[pi, pj] for A in As], rtol=1e-14, atol=0)


def test_channel_split_in_two_equals_one_channel():
    """Splitting one channel's visibilities into two channels with the same
    beam leaves the data unchanged, so Phi, chi^2 and grad Phi of the shared
    image equal the single-channel objective on all the visibilities."""
    n, cell = 16, 2.0e-6
    c = _chan(n, cell, 300, 32, 9)
    img = synth.random_image(n, 32, lo=0.05, hi=1.0)[0]
    M, lam = 1e-2, 0.2
    one = oracle.phi_grad(n, cell, c["u"], c["v"], c["A"], img, c["vis"], c["w"], M, lam)
    k = 117
    halves = [dict(u=c["u"][s], v=c["v"][s], vis=c["vis"][s], w=c["w"][s], A=c["A"])
              for s in (slice(0, k), slice(k, None))]
    two = oracle.phi_grad_shared(n, cell, halves, img, M, lam)
    assert abs(two["phi"] - one["phi"]) < 1e-12 * abs(one["phi"])
    assert abs(two["chi2"] - one["chi2"]) < 1e-12 * one["chi2"]
    assert abs(two["S"] - one["S"]) == 0.0
    assert rel(two["grad"], one["grad"]) < 1e-12
    assert rel(two["R"], one["R"]) < 1e-13


def test_shared_gradient_matches_central_differences_two_beams():
    """Brute-force central differences of the shared Phi at every pixel of
    an 8x8 image, with two channels of different beams and uv scales (the
    frequency scaling of Sec. 2.4), reproduce the analytic gradient."""
    n, cell = 8, 4.0e-6
    chans = [_chan(n, cell, 50, 33, 3), _chan(n, cell, 70, 34, 7, uv_scale=1.1)]
    img = synth.random_image(n, 33, lo=0.05, hi=1.0)[0]
    M, lam = 1e-2, 0.3
    out = oracle.phi_grad_shared(n, cell, chans, img, M, lam)

    def phi(x):
        return oracle.phi_grad_shared(n, cell, chans, x, M, lam)["phi"]

    fd = np.zeros((n, n))
    for p in range(n * n):
        i, j = divmod(p, n)
        h = 1e-4 * img[i, j]
        a = img.copy(); a[i, j] += h
        b = img.copy(); b[i, j] -= h
        fd[i, j] = (phi(a) - phi(b)) / (2 * h)
    assert rel(out["grad"], fd) < 1e-7


def test_shared_problem_forward_adjoint_pair():
    """The shared problem's forward and adjoint are adjoint to each other:
    <F I, c>_w-free real inner product equals <I, F^H c> for random I, c."""
    n, cell = 8, 4.0e-6
    chans = [_chan(n, cell, 40, 35, 4), _chan(n, cell, 30, 36, 6, uv_scale=0.9)]
    prob = ocg.SharedProblem(n, cell, chans, 1e-2, 0.1)
    rng = np.random.default_rng(35)
    I = rng.standard_normal((n, n))
    c = rng.standard_normal(70) + 1j * rng.standard_normal(70)
    lhs = float(np.sum((prob.F(I) * np.conj(c)).real))
    rhs = float(np.sum(I * prob.FH(c)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_shared_cg_on_split_channel_follows_single_channel_cg():
    """The projected CG on the shared image of a channel split in two takes
    the same iterates as on the single channel."""
    n, cell = 8, 4.0e-6
    c = _chan(n, cell, 90, 37, 6)
    M, lam = 1e-2, 0.1
    single = ocg.Problem(n, cell, c["u"], c["v"], c["vis"], c["w"], c["A"], M, lam)
    halves = [dict(u=c["u"][s], v=c["v"][s], vis=c["vis"][s], w=c["w"][s], A=c["A"])
              for s in (slice(0, 41), slice(41, None))]
    shared = ocg.SharedProblem(n, cell, halves, M, lam)
    I1, t1 = ocg.projected_cg(single, 12)
    I2, t2 = ocg.projected_cg(shared, 12)
    assert len(t1) == len(t2) == 12
    for a, b in zip(t1, t2):
        assert abs(a["phi"] - b["phi"]) < 1e-10 * abs(a["phi"])
    assert rel(I2, I1) < 1e-9


def test_shared_cg_reaches_bound_constrained_minimum():
    """Two channels with different beams: Phi is non-increasing, I >= M, and
    after many iterations Phi equals the minimum found by L-BFGS-B."""
    n, cell = 8, 4.0e-6
    chans = [_chan(n, cell, 60, 38, 5), _chan(n, cell, 60, 39, 8, uv_scale=1.2)]
    prob = ocg.SharedProblem(n, cell, chans, 1e-2, 0.05)
    I, traj = ocg.projected_cg(prob, 300)
    phis = [t["phi"] for t in traj]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(phis, phis[1:]))
    assert np.all(I >= prob.M)

    def fun(x):
        ev = prob.evaluate(x.reshape(n, n))
        return ev["phi"], ev["g"].ravel()

    ref = scipy.optimize.minimize(fun, np.full(n * n, 0.1), jac=True, method="L-BFGS-B",
                                  bounds=[(prob.M, None)] * (n * n),
                                  options=dict(maxiter=5000, ftol=1e-15, gtol=1e-12))
    phi_cg = prob.evaluate(I)["phi"]
    assert phi_cg <= ref.fun + 1e-8 * abs(ref.fun)
    assert abs(phi_cg - ref.fun) < 1e-7 * abs(ref.fun)
