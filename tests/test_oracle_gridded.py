"""Pins of the oracle's gridded forward model (Sec. 2.4, Alg. 1) and its adjoint.

The gridded model uses a library FFT; it is pinned to the independent direct
DFT of the C oracle: on grid-aligned uv points it must equal the exact model,
and off the grid it must equal the bilinear blend of the exact model at the
four surrounding grid frequencies (which also pins the modulation by the
phase centre, the wrap-around of negative frequencies and the zero padding).
The adjoint is pinned by the dot test and by finite differences of the
gridded objective.
"""
import numpy as np
import pytest

import oracle
from oracle import gridded as og
from paper_1703_02920_amd import synth


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


CELL = 1.0e-6


@pytest.mark.parametrize("n,s", [(16, 1), (16, 2), (32, 1), (8, 4)])
def test_grid_aligned_uv_equals_exact_dft(n, s):
    """u_k = p_k du, v_k = q_k du with integer p, q in [-Ng/2, Ng/2): no
    interpolation, so the gridded model is the exact DFT (Eq. fft)."""
    Ng = s * n
    rng = np.random.default_rng(60 + n + s)
    p = rng.integers(-Ng // 2, Ng // 2, 200)
    q = rng.integers(-Ng // 2, Ng // 2, 200)
    du = 1.0 / (Ng * CELL)
    u, v = p * du, q * du
    A = oracle.beam(n, CELL, 0.7 * n * CELL)
    img = synth.random_image(n, 61)[0]
    got = og.gridded_forward(n, CELL, u, v, A, img, s)
    ref = oracle.forward(n, CELL, u, v, A, img)
    assert rel(got, ref) < 1e-13


@pytest.mark.parametrize("n,s", [(16, 1), (16, 2), (32, 1)])
def test_off_grid_is_bilinear_blend_of_exact_dft(n, s):
    """At (p + f) du, (q + g) du the gridded value is
    (1-f)(1-g) V(p,q) + f(1-g) V(p+1,q) + (1-f) g V(p,q+1) + f g V(p+1,q+1)
    with V the exact DFT at those grid frequencies (computed by the C
    oracle), including cells that straddle the +-Ng/2 wrap."""
    Ng = s * n
    rng = np.random.default_rng(62 + n + s)
    nv = 300
    p = rng.integers(-Ng // 2, Ng // 2, nv)
    q = rng.integers(-Ng // 2, Ng // 2, nv)
    p[:5] = Ng // 2 - 1          # cells whose upper node wraps to -Ng/2
    q[5:10] = Ng // 2 - 1
    f = rng.uniform(0, 1, nv)
    g = rng.uniform(0, 1, nv)
    du = 1.0 / (Ng * CELL)
    u, v = (p + f) * du, (q + g) * du
    A = oracle.beam(n, CELL, 0.6 * n * CELL)
    img = synth.random_image(n, 63)[0]
    got = og.gridded_forward(n, CELL, u, v, A, img, s)

    def ex(pp, qq):
        return oracle.forward(n, CELL, pp * du, qq * du, A, img)

    ref = ((1 - f) * (1 - g) * ex(p, q) + f * (1 - g) * ex(p + 1, q)
           + (1 - f) * g * ex(p, q + 1) + f * g * ex(p + 1, q + 1))
    assert rel(got, ref) < 1e-12


def test_gridded_adjoint_dot_test():
    """<F_g I, c> (real part) = <I, A o Re F_g^H c> for random I, c, s = 2."""
    n, s = 16, 2
    u, v, _, _ = synth.random_problem(n, 250, 64, cell=CELL)
    A = oracle.beam(n, CELL, 0.8 * n * CELL)
    rng = np.random.default_rng(64)
    I = rng.standard_normal((n, n))
    c = rng.standard_normal(250) + 1j * rng.standard_normal(250)
    lhs = float(np.sum((og.gridded_forward(n, CELL, u, v, A, I, s) * np.conj(c)).real))
    rhs = float(np.sum(I * og.gridded_adjoint(n, CELL, u, v, A, c, s)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gridded_gradient_matches_central_differences_8x8():
    """With grad="adjoint" the gradient is the exact gradient of the gridded
    objective: central differences at every pixel of an 8x8 image."""
    n, cell = 8, 4.0e-6
    u, v, vis, w = synth.random_problem(n, 60, 65, cell=cell)
    A = oracle.beam(n, cell, 5 * cell)
    img = synth.random_image(n, 65, lo=0.05, hi=1.0)[0]
    M, lam = 1e-2, 0.3
    out = og.gridded_phi_grad(n, cell, u, v, A, img, vis, w, M, lam, oversample=2)
    fd = np.zeros((n, n))
    for pix in range(n * n):
        i, j = divmod(pix, n)
        h = 1e-4 * img[i, j]
        a = img.copy(); a[i, j] += h
        b = img.copy(); b[i, j] -= h
        fa = og.gridded_phi_grad(n, cell, u, v, A, a, vis, w, M, lam, oversample=2)["phi"]
        fb = og.gridded_phi_grad(n, cell, u, v, A, b, vis, w, M, lam, oversample=2)["phi"]
        fd[i, j] = (fa - fb) / (2 * h)
    assert rel(out["grad"], fd) < 1e-7


def test_gridded_objective_on_grid_aligned_data_equals_exact():
    """Grid-aligned uv: the gridded Phi, R and both gradient choices equal
    the exact objective."""
    n, s = 16, 1
    Ng = s * n
    rng = np.random.default_rng(66)
    du = 1.0 / (Ng * CELL)
    u = rng.integers(-Ng // 2, Ng // 2, 120) * du
    v = rng.integers(-Ng // 2, Ng // 2, 120) * du
    vis = rng.standard_normal(120) + 1j * rng.standard_normal(120)
    w = rng.uniform(0.5, 2, 120)
    A = oracle.beam(n, CELL, 0.7 * n * CELL)
    img = synth.random_image(n, 66, lo=0.05, hi=1.0)[0]
    ex = oracle.phi_grad(n, CELL, u, v, A, img, vis, w, 1e-2, 0.1)
    for grad in ("adjoint", "dft"):
        gr = og.gridded_phi_grad(n, CELL, u, v, A, img, vis, w, 1e-2, 0.1, oversample=s, grad=grad)
        assert abs(gr["phi"] - ex["phi"]) < 1e-12 * abs(ex["phi"])
        assert rel(gr["R"], ex["R"]) < 1e-12
        assert rel(gr["grad"], ex["grad"]) < 1e-11


def test_interpolation_error_shrinks_with_oversampling():
    """A compact source observed at random uv: the gridded model's error
    against the exact DFT falls roughly fourfold per doubling of the Fourier
    grid (bilinear interpolation is second order in the grid step)."""
    n = 32
    u, v, _, _ = synth.random_problem(n, 400, 67, cell=CELL, fill=0.4)
    A = oracle.beam(n, CELL, 0.8 * n * CELL)
    yy, xx = np.mgrid[0:n, 0:n] - n // 2
    img = np.exp(-(xx ** 2 + yy ** 2) / (2 * 2.0 ** 2))
    ref = oracle.forward(n, CELL, u, v, A, img)
    errs = [rel(og.gridded_forward(n, CELL, u, v, A, img, s), ref) for s in (1, 2, 4, 8)]
    for a, b in zip(errs, errs[1:]):
        assert 2.5 < a / b < 6.0, errs
