"""Positively-constrained projected conjugate gradient, FP64 reference.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper minimises Phi over I >= G (Eq. minproblem) with a positively
constrained CG whose loop runs on the host (Sec. 2.6); its CPU version is
built on the Numerical Recipes frprmn routine with line minimisation and
bracketing (Sec. 3.2).  The variant below is the reading taken here, step by
step, in plain numpy on top of the direct-sum forward/adjoint of the C
oracle:

  init:  I <- M everywhere; V = F(I), R = V - V^o, g = grad Phi(I);
         active set  Act = {p : I_p <= M(1 + 1e-12) and g_p > 0};
         projected gradient gt = g with gt_p = 0 on Act;  d = -gt.
  each iteration:
    1. project the direction: d_p = 0 on Act; d_p = max(d_p, 0) on the other
       pixels at the bound.
    2. if gt.d >= 0 restart with d = -gt;  stop if gt = 0.
    3. Vd = F(d) (no data term).
    4. a = sum w |Vd|^2, b = sum w Re(conj(R) Vd): chi^2(I + alpha d) =
       chi^2 + b alpha + a alpha^2 / 2 exactly (F is linear).
    5. alpha_max = min over d_p < 0 of (I_p - M) / (-d_p)  (inf if none).
    6. phi(alpha) = chi^2(alpha) + lambda sum (I + alpha d) ln((I + alpha d)/M)
       is convex on [0, alpha_max] with
       phi'(alpha)  = b + a alpha + lambda sum d (ln((I + alpha d)/M) + 1),
       phi''(alpha) = a + lambda sum d^2 / (I + alpha d).
    7. alpha* = alpha_max if phi'(alpha_max) <= 0, else the root of phi' by
       Newton steps kept inside a shrinking bisection bracket.
    8. I <- max(I + alpha* d, M); V, R, Phi, g, gt, Act recomputed from scratch.
    9. beta = max(0, gt_new.(gt_new - gt_old) / gt_old.gt_old) (Polak-Ribiere
       with restart at zero); d <- -gt_new + beta d.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import adjoint, chi2, entropy, forward

BOUND_TOL = 1e-12


class Problem:
    """One channel: image side n, cell, uv, data, weights, beam image A."""

    def __init__(self, n, cell, u, v, vis, w, A, M, lam):
        self.n = n
        self.cell = cell
        self.u = np.asarray(u, np.float64)
        self.v = np.asarray(v, np.float64)
        self.vis = np.asarray(vis, np.complex128)
        self.w = np.asarray(w, np.float64)
        self.A = None if A is None else np.asarray(A, np.float64)
        self.M = float(M)
        self.lam = float(lam)

    def F(self, img):
        return forward(self.n, self.cell, self.u, self.v, self.A, img)

    def FH(self, c):
        return adjoint(self.n, self.cell, self.u, self.v, self.A, c)

    def evaluate(self, img):
        V = self.F(img)
        x2, R = chi2(V, self.vis, self.w)
        S, gS = entropy(img, self.M)
        g = self.FH(self.w * R) + self.lam * gS
        return dict(V=V, R=R, chi2=x2, S=S, phi=x2 + self.lam * S, g=g)


class SharedProblem(Problem):
    """One image fitted to several channels (Eq. chi2-multi): the forward
    model is the concatenation of the channels' visibilities, each channel
    with its own uv, weights and beam; the adjoint of concatenated
    coefficients is the sum of the channels' adjoint images.  The CG below
    then runs unchanged on the one image."""

    def __init__(self, n, cell, chans, M, lam):
        self.n = n
        self.cell = cell
        self.chans = [dict(u=np.asarray(c["u"], np.float64), v=np.asarray(c["v"], np.float64),
                           A=None if c["A"] is None else np.asarray(c["A"], np.float64))
                      for c in chans]
        self.sizes = [int(c["u"].shape[0]) for c in self.chans]
        self.vis = np.concatenate([np.asarray(c["vis"], np.complex128) for c in chans])
        self.w = np.concatenate([np.asarray(c["w"], np.float64) for c in chans])
        self.M = float(M)
        self.lam = float(lam)

    def F(self, img):
        return np.concatenate([forward(self.n, self.cell, c["u"], c["v"], c["A"], img) for c in self.chans])

    def FH(self, coef):
        out = np.zeros((self.n, self.n))
        o = 0
        for c, z in zip(self.chans, self.sizes):
            out += adjoint(self.n, self.cell, c["u"], c["v"], c["A"], coef[o:o + z])
            o += z
        return out


class MosaicProblem(SharedProblem):
    """One image fitted to several pointings (oracle.phi_grad_mosaic): each
    pointing's forward model carries the phase factor of its phase-tracking
    centre (keys x0, y0) and the adjoint its conjugate."""

    def __init__(self, n, cell, pointings, M, lam):
        super().__init__(n, cell, pointings, M, lam)
        self.shifts = [np.exp(2j * np.pi * (np.asarray(p["u"], np.float64) * p["x0"]
                                            + np.asarray(p["v"], np.float64) * p["y0"])) for p in pointings]

    def F(self, img):
        return np.concatenate([s * forward(self.n, self.cell, c["u"], c["v"], c["A"], img)
                               for c, s in zip(self.chans, self.shifts)])

    def FH(self, coef):
        out = np.zeros((self.n, self.n))
        o = 0
        for c, s, z in zip(self.chans, self.shifts, self.sizes):
            out += adjoint(self.n, self.cell, c["u"], c["v"], c["A"], coef[o:o + z] * np.conj(s))
            o += z
        return out


class GriddedProblem(Problem):
    """One channel with the gridded forward model of Sec. 2.4 / Alg. 1
    (oracle.gridded) on a grid oversample times finer than the image.
    grad="adjoint" uses that model's exact adjoint; grad="dft" the exact-DFT
    gradient of Eq. chi2gradient at the gridded residuals (the paper's
    combination)."""

    def __init__(self, n, cell, u, v, vis, w, A, M, lam, oversample=1, grad="adjoint"):
        super().__init__(n, cell, u, v, vis, w, A, M, lam)
        self.oversample = int(oversample)
        self.grad = grad

    def F(self, img):
        from .gridded import gridded_forward
        return gridded_forward(self.n, self.cell, self.u, self.v, self.A, img, self.oversample)

    def FH(self, c):
        if self.grad == "dft":
            return adjoint(self.n, self.cell, self.u, self.v, self.A, c)
        from .gridded import gridded_adjoint
        return gridded_adjoint(self.n, self.cell, self.u, self.v, self.A, c, self.oversample)


def line_search(a, b, I, d, M, lam, alpha_max, max_steps=100, rtol=1e-13):
    """Exact minimiser of phi on [0, alpha_max] (steps 6-7)."""
    def dphi(al):
        x = I + al * d
        return b + a * al + lam * float(np.sum(d * (np.log(x / M) + 1.0)))

    def d2phi(al):
        x = I + al * d
        return a + lam * float(np.sum(d * d / x))

    d0 = dphi(0.0)
    if not d0 < 0.0:
        return 0.0, 0
    lo, hi = 0.0, alpha_max
    if math.isfinite(alpha_max):
        if dphi(alpha_max) <= 0.0:
            return alpha_max, 0
    else:
        # bracket the root: grow an upper end until phi' > 0
        hi = -b / a if a > 0 else 1.0
        if not (hi > 0 and math.isfinite(hi)):
            hi = 1.0
        n_grow = 0
        while dphi(hi) <= 0.0:
            lo = hi
            hi *= 2.0
            n_grow += 1
            if n_grow > 2000:
                raise FloatingPointError("line search: no upper bracket")
    al = 0.5 * (lo + hi)
    if a > 0:
        guess = -b / a
        if lo < guess < hi:
            al = guess
    steps = 0
    for steps in range(1, max_steps + 1):
        f = dphi(al)
        if f > 0:
            hi = al
        else:
            lo = al
        h = d2phi(al)
        nxt = al - f / h if h > 0 else 0.5 * (lo + hi)
        if not (lo < nxt < hi):
            nxt = 0.5 * (lo + hi)
        delta = abs(nxt - al)
        al = nxt
        if delta <= rtol * abs(al):
            break
    return al, steps


def projected_cg(prob: Problem, iters: int, I0: Optional[np.ndarray] = None, free: Optional[np.ndarray] = None):
    """Run `iters` iterations; returns the final image and the trajectory
    (per iteration: phi, chi2, S, alpha, beta, |gt|^2 after the step).
    `free` (optional boolean image) is a focus-of-attention region (Sec. 6):
    pixels outside it are not free parameters and join the active set, so
    they keep their value."""
    M, lam = prob.M, prob.lam
    fixed = np.zeros((prob.n, prob.n), bool) if free is None else ~np.asarray(free, bool)
    I = np.full((prob.n, prob.n), M) if I0 is None else np.array(I0, np.float64)
    ev = prob.evaluate(I)
    at_bound = I <= M * (1 + BOUND_TOL)
    act = (at_bound & (ev["g"] > 0)) | fixed
    gt = np.where(act, 0.0, ev["g"])
    d = -gt
    traj = []
    for _ in range(iters):
        at_bound = I <= M * (1 + BOUND_TOL)
        d = np.where(act, 0.0, d)
        d = np.where(at_bound & ~act, np.maximum(d, 0.0), d)
        gg = float(np.sum(gt * gt))
        if gg == 0.0:
            break
        if float(np.sum(gt * d)) >= 0.0:
            d = -gt
        Vd = prob.F(d)
        R = ev["R"]
        a = float(np.sum(prob.w * (Vd.real ** 2 + Vd.imag ** 2)))
        b = float(np.sum(prob.w * (R.real * Vd.real + R.imag * Vd.imag)))
        neg = d < 0
        alpha_max = float(np.min((I[neg] - M) / (-d[neg]))) if np.any(neg) else math.inf
        alpha, _ = line_search(a, b, I, d, M, lam, alpha_max)
        if alpha == 0.0:
            break
        I = np.maximum(I + alpha * d, M)
        ev = prob.evaluate(I)
        at_bound = I <= M * (1 + BOUND_TOL)
        act = (at_bound & (ev["g"] > 0)) | fixed
        gt_new = np.where(act, 0.0, ev["g"])
        beta = max(0.0, float(np.sum(gt_new * (gt_new - gt))) / gg)
        d = -gt_new + beta * d
        gt = gt_new
        traj.append(dict(phi=ev["phi"], chi2=ev["chi2"], S=ev["S"], alpha=alpha, beta=beta,
                         gnorm2=float(np.sum(gt * gt)), alpha_max=alpha_max))
    return I, traj
