"""Imaging utilities and focus of attention on the GPU against the oracle:
natural-weight dirty image and PSF (App. A), thermal noise (App. B), the
clean-beam fit, and CG restricted to a region (Sec. 6)."""
import functools

import numpy as np
import pytest

import oracle
from oracle import cg as ocg
from oracle import imaging as oim
from _common import CG_TOL, TOL, Problem, flush, rel, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRECS = ["fp64", "fp32", "bf16x3", "fp16x3"]


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ochans(prob, idx):
    return [dict(u=prob.chans[c]["u"], v=prob.chans[c]["v"], vis=prob.chans[c]["vis"], w=prob.chans[c]["w"])
            for c in idx]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("mode", ["cube", "shared"])
def test_dirty_image_and_psf_parity(prec, mode):
    _cuda()
    prob = Problem.random(100, [900, 1333], seed=80, lam=0.05)
    ctx = prob.context(prec, mode=mode)
    d, p = ctx.dirty_image()
    d, p = d.cpu().numpy(), p.cpu().numpy()
    groups = [[0], [1]] if mode == "cube" else [[0, 1]]
    errs = []
    for m, g in enumerate(groups):
        rd, rp = oim.dirty_and_psf(prob.n, prob.cell, _ochans(prob, g))
        errs += [rel(d[m], rd), rel(p[m], rp)]
        assert abs(p[m][prob.n // 2, prob.n // 2] - 1.0) < 10 * TOL[prec]
    flush(f"dirty/psf {prec} {mode}: " + " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) < TOL[prec]
    sd = ctx.noise()
    for m, g in enumerate(groups):
        assert abs(sd[m] / oim.sigma_d(_ochans(prob, g)) - 1.0) < 1e-14


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fit_beam_matches_oracle_fit_on_the_same_psf(prec):
    """The library's fit on the oracle's PSF of the 256^2 x 99,840 workload
    (rounded to the context's precision) equals the oracle's fit of that PSF;
    the library's own PSF gives the same beam to the PSF's accuracy."""
    _cuda()
    ds = synth.make_config(2)
    prob = Problem.from_dataset(ds)
    ctx = prob.context(prec)
    _, rp = oim.dirty_and_psf(ds.n, ds.cell, _ochans(prob, [0]))
    dt = torch.float64 if prec == "fp64" else torch.float32
    rp_t = torch.tensor(rp[None], dtype=dt, device="cuda")
    a, b, pa = ctx.fit_beam(rp_t)
    oa, ob, opa = oim.fit_beam(rp_t.cpu().numpy()[0].astype(np.float64), ds.cell)
    flush(f"fit_beam {prec}: bmaj {a[0] / ds.cell:.4f} px bmin {b[0] / ds.cell:.4f} px bpa {pa[0]:.3f} deg")
    assert abs(a[0] / oa - 1) < 1e-9 and abs(b[0] / ob - 1) < 1e-9 and abs(pa[0] - opa) < 1e-7
    _, p = ctx.dirty_image(dirty=False)
    a2, b2, pa2 = ctx.fit_beam(p)
    assert abs(a2[0] / oa - 1) < 1e-4 and abs(b2[0] / ob - 1) < 1e-4 and abs(pa2[0] - opa) < 1e-2


def test_dirty_image_full_size_sampled():
    """1024^2 x 5,000,250: the dirty image at seeded pixels, each computed by
    the oracle as a direct sum over all visibilities."""
    _cuda()
    ds = synth.make_config(5)
    prob = Problem.from_dataset(ds)
    ctx = prob.context("fp32")
    d, _ = ctx.dirty_image(psf=False)
    ch = prob.chans[0]
    w = ch["w"].astype(np.float64)
    pix = np.sort(np.random.default_rng(81).choice(ds.n * ds.n, size=24, replace=False))
    ref = oracle.adjoint(ds.n, ds.cell, ch["u"], ch["v"], None, w * ch["vis"].astype(np.complex128), pix=pix) / w.sum()
    e = rel(d.cpu().numpy()[0].ravel()[pix], ref)
    flush(f"dirty image c5 sampled: {e:.2e}")
    assert e < TOL["fp32"]


def _region(n):
    free = np.zeros((n, n), bool)
    free[n // 4:3 * n // 4 + 3, n // 4 - 5:3 * n // 4] = True
    return free


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_focus_of_attention_phi_grad_and_cg(prec):
    """64^2 x 5,130 workload restricted to a region: grad Phi is the oracle's
    inside and 0 outside; the CG follows the oracle's region-restricted CG and
    leaves the pixels outside at the floor."""
    _cuda()
    ds = synth.make_config(1)
    prob = Problem.from_dataset(ds)
    free = _region(ds.n)
    from paper_1703_02920_amd.uvmem import Context
    ctx = Context(ds.n, 1, prec)
    ch = prob.chans[0]
    ctx.set_uv(0, ch["u"], ch["v"], ds.cell)
    ctx.set_vis(0, ch["vis"])
    ctx.set_weights(0, ch["w"])
    ctx.set_beam(0, ch["fwhm"])
    ctx.set_mask(0, free)
    ctx.set_prior(ds.prior_m, ds.lam)
    ctx.finalize()
    I = torch.tensor(synth.eval_images(ds, "P3"), dtype=ctx.dtype, device="cuda")
    scal, g = ctx.phi_and_grad(I)
    ref = prob.oracle_phi_grad(0, I.cpu().numpy()[0].astype(np.float64))
    gg = g.cpu().numpy()[0]
    assert np.all(gg[~free] == 0.0)
    assert rel(gg[free], ref["grad"][free]) < TOL[prec]
    assert abs(float(scal[0, 0]) - ref["phi"]) < TOL[prec] * abs(ref["phi"])
    op = ocg.Problem(ds.n, ds.cell, ch["u"], ch["v"], ch["vis"], ch["w"], prob.beam(0), ds.prior_m, ds.lam)
    I_ref, traj = ocg.projected_cg(op, ds.cg_iters, free=free)
    J = ctx.image()
    ctx.cg_init(J, init_to_floor=True)
    hist = ctx.cg_run(J, ds.cg_iters, graph=True).cpu().numpy()
    ctx.check()
    Jn = J.cpu().numpy()[0]
    assert np.all(Jn[~free] == Jn[0, 0])
    phis = hist[:, 0, 0]
    ref_phis = np.array([t["phi"] for t in traj])
    e_phis = np.abs(phis - ref_phis) / np.abs(ref_phis)
    e_img = rel(Jn, I_ref)
    flush(f"focus of attention cg {prec}: max rel phi {e_phis.max():.2e}, final image {e_img:.2e}")
    bar = {"fp64": CG_TOL["fp64"]["phi"], "fp32": 5e-5}[prec]
    assert e_phis.max() < bar and e_img < CG_TOL[prec]["img"] and e_phis[0] < CG_TOL[prec]["first"]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_focus_region_visits_fewer_tiles(prec):
    """256^2 image, region inside one quarter: the CG's direction forward and
    gradient adjoint visit only the region's blocks and tiles; Phi, the
    gradient inside the region and the CG trajectory match the oracle's
    region-restricted results, and the pixels outside stay at the floor."""
    _cuda()
    prob = Problem.random(256, [1800], seed=82, lam=0.02)
    free = np.zeros((256, 256), bool)
    free[20:100, 30:120] = True
    from paper_1703_02920_amd.uvmem import Context
    ctx = Context(256, 1, prec)
    ch = prob.chans[0]
    ctx.set_uv(0, ch["u"], ch["v"], prob.cell)
    ctx.set_vis(0, ch["vis"])
    ctx.set_weights(0, ch["w"])
    ctx.set_beam(0, ch["fwhm"])
    ctx.set_mask(0, free)
    ctx.set_prior(prob.M, prob.lam)
    ctx.finalize()
    info = ctx.info()
    flush(f"region lists {prec}: forward {info['n_fwd_wgs_region']} of {info['n_fwd_wgs']} workgroups, "
          f"adjoint {info['n_adj_wgs_region']} of {info['n_adj_items']}")
    assert info["n_fwd_wgs_region"] > 0 and info["n_adj_wgs_region"] > 0
    I = torch.tensor(synth.random_image(256, 83, lo=1e-3, hi=1.0), dtype=ctx.dtype, device="cuda")
    scal, g = ctx.phi_and_grad(I)
    ref = prob.oracle_phi_grad(0, I.cpu().numpy()[0].astype(np.float64))
    gg = g.cpu().numpy()[0]
    assert np.all(gg[~free] == 0.0)
    e_g = rel(gg[free], ref["grad"][free])
    assert e_g < TOL[prec] and abs(float(scal[0, 0]) - ref["phi"]) < TOL[prec] * abs(ref["phi"])
    op = ocg.Problem(256, prob.cell, ch["u"], ch["v"], ch["vis"], ch["w"], prob.beam(0), prob.M, prob.lam)
    iters = 8
    I_ref, traj = ocg.projected_cg(op, iters, free=free)
    J = ctx.image()
    ctx.cg_init(J, init_to_floor=True)
    hist = ctx.cg_run(J, iters, graph=True).cpu().numpy()
    ctx.check()
    Jn = J.cpu().numpy()[0]
    assert np.all(Jn[~free] == Jn[0, 0])
    e_phis = np.abs(hist[:, 0, 0] - [t["phi"] for t in traj]) / np.abs([t["phi"] for t in traj])
    e_img = rel(Jn, I_ref)
    flush(f"  grad {e_g:.2e}, cg max rel phi {e_phis.max():.2e}, final image {e_img:.2e}")
    bar = {"fp64": CG_TOL["fp64"]["phi"], "fp32": 5e-5, "bf16x3": CG_TOL["bf16x3"]["phi"]}[prec]
    assert e_phis.max() < bar and e_img < CG_TOL[prec]["img"]
