"""Parity at the full workload sizes, in the launch configuration the
benchmark uses.

256^2 x 99,840 visibilities: Phi, chi^2, V^m, R and grad Phi compared element
by element with the FP64 oracle over every visibility and pixel.
512^2 x 999,600, 64 x 256^2 (uneven channels) and 1024^2 x 5,000,250: the
model visibilities at seeded samples of visibilities and the adjoint at
seeded samples of pixels (each computed one by one by the oracle), plus
properties that fix the full-size reductions exactly: an image that is a
single point of flux F at the phase centre has V_k = F for every k, so chi^2
and the residuals are known in closed form, and the chi^2 gradient is the
adjoint of those residuals.
"""
import functools

import numpy as np
import pytest

import oracle
from _common import TOL, Problem, flush, rel, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@functools.lru_cache(maxsize=None)
def _ds(c):
    flush(f"  generating workload c{c}")
    return synth.make_config(c)


@functools.lru_cache(maxsize=None)
def _oracle_c2_P3():
    ds = _ds(2)
    prob = Problem.from_dataset(ds)
    img = synth.eval_images(ds, "P3")[0].astype(np.float32).astype(np.float64)
    return img, prob.oracle_phi_grad(0, img)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_c2_full_phi_grad(prec):
    """Every visibility and pixel of the 256^2 x 99,840 workload at P3."""
    _cuda()
    flush(f"c2 full parity {prec}")
    ds = _ds(2)
    img, ref = _oracle_c2_P3()
    prob = Problem.from_dataset(ds)
    ctx = prob.context(prec)
    I = torch.tensor(img[None], dtype=torch.float32, device="cuda")
    scal, grad = ctx.phi_and_grad(I)
    scal = scal.cpu().numpy()
    e = dict(phi=abs(scal[0, 0] - ref["phi"]) / abs(ref["phi"]),
             chi2=abs(scal[0, 1] - ref["chi2"]) / abs(ref["chi2"]),
             S=abs(scal[0, 2] - ref["S"]) / abs(ref["S"]),
             R=rel(ctx.residual().cpu().numpy(), ref["R"]),
             grad=rel(grad.cpu().numpy()[0], ref["grad"]))
    flush("  " + " ".join(f"{k} {v:.2e}" for k, v in e.items()))
    for k, v in e.items():
        assert v < TOL[prec], (k, v)


def _sampled(prec, c, n_vis=96, n_pix=96, channels=None):
    _cuda()
    ds = _ds(c)
    prob = Problem.from_dataset(ds)
    ctx = prob.context(prec)
    rng = np.random.default_rng(1000 + c)
    img = synth.eval_images(ds, "P3").astype(np.float32)
    I = torch.tensor(img, dtype=torch.float32, device="cuda")
    V = ctx.forward(I).cpu().numpy()
    offs = prob.offsets()
    chans = range(prob.n_chan) if channels is None else channels
    worst = 0.0
    for ch in chans:
        nv = len(prob.chans[ch]["u"])
        if nv == 0:
            continue
        idx = np.sort(rng.choice(nv, size=min(n_vis, nv), replace=False))
        A = prob.beam(ch)
        ref = oracle.forward_sel(ds.n, ds.cell, idx, prob.chans[ch]["u"], prob.chans[ch]["v"], A,
                                 img[ch].astype(np.float64))
        got = V[offs[ch] + idx]
        worst = max(worst, rel(got, ref))
    flush(f"  forward, sampled visibilities: worst channel rel err {worst:.2e}")
    assert worst < TOL[prec]
    # adjoint of a fixed coefficient vector at sampled pixels
    coef = np.concatenate([prob.chans[ch]["w"].astype(np.float64) * prob.chans[ch]["vis"].astype(np.complex128)
                           for ch in range(prob.n_chan)])
    G = ctx.adjoint(torch.tensor(coef, dtype=torch.complex128, device="cuda")).cpu().numpy()
    worst = 0.0
    for ch in chans:
        pix = np.sort(rng.choice(ds.n * ds.n, size=n_pix, replace=False))
        ref = prob.oracle_adjoint(ch, coef[offs[ch]:offs[ch + 1]], pix=pix)
        worst = max(worst, rel(G[ch].ravel()[pix], ref))
    flush(f"  adjoint, sampled pixels: worst channel rel err {worst:.2e}")
    assert worst < TOL[prec]
    return ds, prob, ctx


def _point_source_property(ds, prob, ctx, prec):
    """Point of flux F at the phase centre: V_k = F exactly (A = 1 there), so
    R = F - V^o, chi^2 = 1/2 sum w |F - V^o|^2 over all visibilities, and
    grad chi^2 = A o Re F^H(w R) at sampled pixels."""
    F = 0.75
    img = np.full((prob.n_chan, ds.n, ds.n), 1e-30, dtype=np.float32)
    img[:, ds.n // 2, ds.n // 2] = F
    I = torch.tensor(img, dtype=torch.float32, device="cuda")
    scal, grad = ctx.phi_and_grad(I)
    scal = scal.cpu().numpy()
    grad = grad.cpu().numpy()
    offs = prob.offsets()
    rng = np.random.default_rng(7)
    worst_x2 = worst_g = 0.0
    for ch in range(prob.n_chan):
        vo = prob.chans[ch]["vis"].astype(np.complex128)
        w = prob.chans[ch]["w"].astype(np.float64)
        if len(vo) == 0:
            continue
        # model visibilities of the image: F exactly plus the 1e-30 floor's
        # contribution (bounded by N^2 1e-30, far below any tolerance)
        x2, R = oracle.chi2(np.full(len(vo), F + 0j), vo, w)
        worst_x2 = max(worst_x2, abs(scal[ch, 1] - x2) / x2)
        pix = np.sort(rng.choice(ds.n * ds.n, size=48, replace=False))
        gref = prob.oracle_adjoint(ch, w * R, pix=pix)
        lam_part = ds.lam * (np.log(img[ch].ravel()[pix].astype(np.float64) / ds.prior_m) + 1.0)
        worst_g = max(worst_g, rel(grad[ch].ravel()[pix] - lam_part, gref))
    flush(f"  point-source property: chi2 rel err {worst_x2:.2e}, grad chi2 rel err {worst_g:.2e}")
    assert worst_x2 < TOL[prec] and worst_g < TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_c3_sampled_and_point_source(prec):
    flush(f"c3 512^2 x 999,600 sampled parity {prec}")
    ds, prob, ctx = _sampled(prec, 3)
    _point_source_property(ds, prob, ctx, prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_c4_batched_sampled_and_point_source(prec):
    flush(f"c4 64 x 256^2 batched sampled parity {prec}")
    ds, prob, ctx = _sampled(prec, 4, n_vis=48, n_pix=32, channels=[0, 17, 40, 63])
    _point_source_property(ds, prob, ctx, prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_c5_sampled_and_point_source(prec):
    flush(f"c5 1024^2 x 5,000,250 sampled parity {prec}")
    ds, prob, ctx = _sampled(prec, 5, n_vis=48, n_pix=48)
    _point_source_property(ds, prob, ctx, prec)


def test_all_channels_empty():
    """A context whose every channel has no visibilities: chi^2 = 0 and
    grad Phi is the entropy gradient alone."""
    _cuda()
    prob = Problem.random(64, [0, 0], seed=5, lam=0.3)
    ctx = prob.context("fp32")
    I = torch.full((2, 64, 64), 2e-3, dtype=torch.float32, device="cuda")
    scal, grad = ctx.phi_and_grad(I)
    s = scal.cpu().numpy()
    assert np.all(s[:, 1] == 0.0)
    expect = 0.3 * (np.log(np.float32(2e-3).astype(np.float64) / 1e-3) + 1.0)
    assert np.allclose(grad.cpu().numpy(), expect, rtol=1e-6)
    ctx.cg_init(I, init_to_floor=True)
    ctx.cg_step(I)
    ctx.check()


def test_zero_weights_channel():
    """All weights zero (a fully flagged channel): chi^2 = 0, grad chi^2 = 0."""
    _cuda()
    prob = Problem.random(64, [500], seed=6, lam=0.1)
    prob.chans[0]["w"] = np.zeros(500, np.float32)
    ctx = prob.context("fp32")
    I = torch.tensor(synth.random_image(64, 6), dtype=torch.float32, device="cuda")
    scal, grad = ctx.phi_and_grad(I)
    assert float(scal[0, 1]) == 0.0
    expect = 0.1 * (np.log(I.cpu().numpy().astype(np.float64) / 1e-3) + 1.0)
    assert rel(grad.cpu().numpy(), expect) < 1e-6


@pytest.mark.parametrize("n", [2, 2048])
def test_extreme_image_sizes(n):
    """Smallest legal image (2 x 2, padded to one tile) and a large 2048^2
    image with few visibilities: forward and adjoint against the oracle."""
    _cuda()
    nv = 300 if n > 2 else 40
    prob = Problem.random(n, [nv], seed=n, fwhm_px=max(2, n // 2))
    ctx = prob.context("fp32")
    img = synth.random_image(n, n)[0].astype(np.float32)
    V = ctx.forward(torch.tensor(img[None], device="cuda")).cpu().numpy()
    if n <= 64:
        ref = prob.oracle_forward(0, img.astype(np.float64))
        assert rel(V, ref) < TOL["fp32"]
    else:
        idx = np.arange(0, nv, 7)
        ch = prob.chans[0]
        ref = oracle.forward_sel(n, prob.cell, idx, ch["u"], ch["v"], prob.beam(0), img.astype(np.float64))
        assert rel(V[idx], ref) < TOL["fp32"]
    coef = np.random.default_rng(n).standard_normal(nv) + 0j
    G = ctx.adjoint(torch.tensor(coef, dtype=torch.complex128, device="cuda")).cpu().numpy()[0]
    pix = np.arange(0, n * n, max(1, (n * n) // 97))
    ref = prob.oracle_adjoint(0, coef, pix=pix)
    assert rel(G.ravel()[pix], ref) < TOL["fp32"]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_c4_shared_sampled_and_point_source(prec):
    """The 64-channel 256^2 workload fitted with ONE image (Eq. chi2-multi):
    model visibilities at seeded samples of four channels, the adjoint summed
    over all 64 channels at seeded pixels, and the point-source property
    (chi^2 is the sum of the channels' closed forms; grad chi^2 the sum of
    their adjoints)."""
    _cuda()
    flush(f"c4 shared image 64 channels sampled parity {prec}")
    ds = _ds(4)
    prob = Problem.from_dataset(ds)
    ctx = prob.context(prec, mode="shared")
    rng = np.random.default_rng(2004)
    img = synth.eval_images(ds, "P3")[:1].astype(np.float32)
    V = ctx.forward(torch.tensor(img, device="cuda")).cpu().numpy()
    offs = prob.offsets()
    # the bar applies to the relative l2 error of the whole V^m vector; it is
    # estimated on 160 seeded visibilities from each of four channels pooled
    got, refs, per = [], [], []
    for ch in (0, 17, 40, 63):
        nv = len(prob.chans[ch]["u"])
        idx = np.sort(rng.choice(nv, size=min(160, nv), replace=False))
        ref = oracle.forward_sel(ds.n, ds.cell, idx, prob.chans[ch]["u"], prob.chans[ch]["v"], prob.beam(ch),
                                 img[0].astype(np.float64))
        got.append(V[offs[ch] + idx])
        refs.append(ref)
        per.append(rel(got[-1], ref))
    pooled = rel(np.concatenate(got), np.concatenate(refs))
    flush(f"  forward, sampled visibilities: pooled rel err {pooled:.2e}, per channel "
          + " ".join(f"{x:.2e}" for x in per))
    assert pooled < TOL[prec]
    coef = np.concatenate([prob.chans[ch]["w"].astype(np.float64) * prob.chans[ch]["vis"].astype(np.complex128)
                           for ch in range(prob.n_chan)])
    G = ctx.adjoint(torch.tensor(coef, dtype=torch.complex128, device="cuda")).cpu().numpy()
    pix = np.sort(rng.choice(ds.n * ds.n, size=32, replace=False))
    gref = sum(prob.oracle_adjoint(ch, coef[offs[ch]:offs[ch + 1]], pix=pix) for ch in range(prob.n_chan))
    e_a = rel(G[0].ravel()[pix], gref)
    flush(f"  adjoint summed over 64 channels, sampled pixels: rel err {e_a:.2e}")
    assert e_a < TOL[prec]
    F = 0.75
    pimg = np.full((1, ds.n, ds.n), 1e-30, dtype=np.float32)
    pimg[0, ds.n // 2, ds.n // 2] = F
    scal, grad = ctx.phi_and_grad(torch.tensor(pimg, device="cuda"))
    scal, grad = scal.cpu().numpy(), grad.cpu().numpy()
    x2 = 0.0
    gref = np.zeros(len(pix))
    for ch in range(prob.n_chan):
        vo = prob.chans[ch]["vis"].astype(np.complex128)
        w = prob.chans[ch]["w"].astype(np.float64)
        if len(vo) == 0:
            continue
        x, R = oracle.chi2(np.full(len(vo), F + 0j), vo, w)
        x2 += x
        gref += prob.oracle_adjoint(ch, w * R, pix=pix)
    lam_part = ds.lam * (np.log(pimg[0].ravel()[pix].astype(np.float64) / ds.prior_m) + 1.0)
    e_x2 = abs(scal[0, 1] - x2) / x2
    e_g = rel(grad[0].ravel()[pix] - lam_part, gref)
    flush(f"  point-source property: chi2 rel err {e_x2:.2e}, grad chi2 rel err {e_g:.2e}")
    assert e_x2 < TOL[prec] and e_g < TOL[prec]
