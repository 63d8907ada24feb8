"""Shared-image (multi-frequency) mode: one image seen by every channel
through the channel's own uv, weights and beam (Eq. chi2-multi), against the
oracle's objective, forward/adjoint and projected CG."""
import functools

import numpy as np
import pytest

import oracle
from oracle import cg as ocg
from _common import CG_TOL, TOL, Problem, flush, rel, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRECS = ["fp64", "fp32", "bf16x3", "fp16x3"]


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@functools.lru_cache(maxsize=None)
def _continuum(n_chan=3, seed=51):
    """The 64^2 one-channel workload's sky observed at n_chan frequencies:
    channel c scales the uv coordinates by s_c = 1 + 0.03 c and the beam FWHM
    by 1/s_c (the beam scales with frequency, Sec. 2.4 item 1), keeps a
    seeded 70% of the baselines (uneven channel sizes) and carries the
    oracle's model visibilities of the sky through its beam plus seeded
    Gaussian noise of 1% of the peak (w = 1/sigma^2)."""
    ds = synth.make_config(1)
    sky = ds.sky[0].astype(np.float64)
    base = ds.channels[0]
    rng = np.random.default_rng(seed)
    sig = 0.01 * float(sky.max())
    chans = []
    for c in range(n_chan):
        s = 1.0 + 0.03 * c
        keep = rng.uniform(size=len(base.u)) < 0.7
        u, v = base.u[keep] * s, base.v[keep] * s
        fwhm = base.fwhm / s
        V = oracle.forward(ds.n, ds.cell, u, v, oracle.beam(ds.n, ds.cell, fwhm), sky)
        noise = sig * (rng.standard_normal(len(u)) + 1j * rng.standard_normal(len(u)))
        chans.append(dict(u=u, v=v, vis=(V + noise).astype(np.complex64),
                          w=np.full(len(u), 1.0 / sig ** 2, np.float32), fwhm=fwhm))
    return Problem(ds.n, ds.cell, chans, ds.prior_m, ds.lam)


def _ragged(seed=41):
    """100^2 (a ragged tile edge), three channels of different sizes, uv
    scales and beams, one of them empty."""
    prob = Problem.random(100, [700, 0, 1234], seed=seed, lam=0.05)
    for c, (s, f) in enumerate([(1.0, 0.9), (1.1, 0.7), (0.85, 0.5)]):
        prob.chans[c]["u"] = prob.chans[c]["u"] * s
        prob.chans[c]["v"] = prob.chans[c]["v"] * s
        prob.chans[c]["fwhm"] = f * prob.n * prob.cell
    return prob


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("which", ["continuum", "ragged"])
def test_shared_phi_grad_parity(prec, which):
    _cuda()
    flush(f"shared phi/grad parity {prec} {which}")
    prob = _continuum() if which == "continuum" else _ragged()
    ctx = prob.context(prec, mode="shared")
    assert ctx.n_img == 1 and ctx.info()["n_img"] == 1
    img = synth.random_image(prob.n, 52, lo=1e-3, hi=1.0)
    I = torch.tensor(img, dtype=ctx.dtype, device="cuda")
    scal, grad = ctx.phi_and_grad(I)
    scal = scal.cpu().numpy()
    assert scal.shape == (1, 8) and tuple(grad.shape) == (1, prob.n, prob.n)
    ref = prob.oracle_phi_grad_shared(I.cpu().numpy()[0].astype(np.float64))
    e = dict(phi=abs(scal[0, 0] - ref["phi"]) / abs(ref["phi"]),
             chi2=abs(scal[0, 1] - ref["chi2"]) / abs(ref["chi2"]),
             S=abs(scal[0, 2] - ref["S"]) / abs(ref["S"]),
             grad=rel(grad.cpu().numpy()[0], ref["grad"]),
             R=rel(ctx.residual().cpu().numpy(), ref["R"]))
    flush("  " + " ".join(f"{k} {v:.2e}" for k, v in e.items()))
    for k, v in e.items():
        assert v < TOL[prec], (k, v)


@pytest.mark.parametrize("prec", PRECS)
def test_shared_forward_adjoint_parity(prec):
    """Forward of the one image = each channel's model visibilities through
    its own beam, concatenated; adjoint = the sum over channels."""
    _cuda()
    flush(f"shared forward/adjoint parity {prec}")
    prob = _ragged(seed=42)
    ctx = prob.context(prec, mode="shared")
    img = synth.random_image(prob.n, 53, lo=1e-3, hi=1.0)
    I = torch.tensor(img, dtype=ctx.dtype, device="cuda")
    V = ctx.forward(I).cpu().numpy()
    Ih = I.cpu().numpy()[0].astype(np.float64)
    ref = np.concatenate([prob.oracle_forward(c, Ih) for c in range(prob.n_chan)])
    e_f = rel(V, ref)
    rng = np.random.default_rng(54)
    offs = prob.offsets()
    coef = rng.standard_normal(offs[-1]) + 1j * rng.standard_normal(offs[-1])
    G = ctx.adjoint(torch.tensor(coef, dtype=torch.complex128, device="cuda")).cpu().numpy()
    assert G.shape == (1, prob.n, prob.n)
    gref = sum(prob.oracle_adjoint(c, coef[offs[c]:offs[c + 1]]) for c in range(prob.n_chan))
    e_a = rel(G[0], gref)
    flush(f"  forward {e_f:.2e} adjoint {e_a:.2e}")
    assert e_f < TOL[prec] and e_a < TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_shared_single_channel_is_cube_bitwise(prec):
    """With one channel the two modes are the same problem and run the same
    kernels on the same schedule: identical bits."""
    _cuda()
    prob = Problem.random(64, [900], seed=43, lam=0.05)
    img = synth.random_image(64, 55, lo=1e-3, hi=1.0)
    out = []
    for mode in ("cube", "shared"):
        ctx = prob.context(prec, mode=mode)
        I = torch.tensor(img, dtype=ctx.dtype, device="cuda")
        s, g = ctx.phi_and_grad(I)
        ctx.cg_init(I)
        h = ctx.cg_run(I, 3, graph=False)
        out.append((s.clone(), g.clone(), h.clone(), I.clone()))
    for a, b in zip(*out):
        assert torch.equal(a, b)


def test_shared_split_channel_equals_one_channel_fp64():
    """A channel split in two channels with the same beam is the same data:
    shared-mode Phi, grad Phi and CG iterates equal those of the one channel
    (up to FP64 rounding of the different split-K chunking)."""
    _cuda()
    one = Problem.random(64, [1500], seed=44, lam=0.02)
    ch = one.chans[0]
    halves = [dict(u=ch["u"][s], v=ch["v"][s], vis=ch["vis"][s], w=ch["w"][s], fwhm=ch["fwhm"])
              for s in (slice(0, 611), slice(611, None))]
    two = Problem(one.n, one.cell, halves, one.M, one.lam)
    img = synth.random_image(64, 56, lo=1e-3, hi=1.0)
    res = []
    for prob, mode in ((one, "cube"), (two, "shared")):
        ctx = prob.context("fp64", mode=mode)
        I = torch.tensor(img, dtype=torch.float64, device="cuda")
        s, g = ctx.phi_and_grad(I)
        ctx.cg_init(I)
        h = ctx.cg_run(I, 5, graph=False)
        res.append((s.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy(), I.cpu().numpy()))
    (s1, g1, h1, I1), (s2, g2, h2, I2) = res
    assert np.allclose(s1[:, :3], s2[:, :3], rtol=1e-12, atol=0)
    assert rel(g2, g1) < 1e-12
    assert np.allclose(h1[:, 0, :6], h2[:, 0, :6], rtol=1e-9, atol=1e-300)
    assert rel(I2, I1) < 1e-10


@pytest.mark.parametrize("prec", PRECS)
def test_shared_cg_trajectory(prec):
    """Projected CG on the one image of a three-channel continuum problem
    against the oracle's CG on the same objective."""
    _cuda()
    prob = _continuum()
    iters = 20
    flush(f"shared cg trajectory {prec} {iters} iterations")
    oprob = ocg.SharedProblem(prob.n, prob.cell, prob.oracle_chans(), prob.M, prob.lam)
    I_ref, traj = ocg.projected_cg(oprob, iters)
    ctx = prob.context(prec, mode="shared")
    I = ctx.image()
    ctx.cg_init(I, init_to_floor=True)
    hist = ctx.cg_run(I, iters, graph=True).cpu().numpy()
    ctx.check()
    assert len(traj) == iters
    phis = hist[:, 0, 0]
    ref_phis = np.array([t["phi"] for t in traj])
    e_phi = np.max(np.abs(phis - ref_phis) / np.abs(ref_phis))
    e_img = rel(I.cpu().numpy()[0], I_ref)
    flush(f"  max rel phi {e_phi:.2e}, final image {e_img:.2e}")
    flush("  phi rel err: " + " ".join(f"{x:.1e}" for x in np.abs(phis - ref_phis) / np.abs(ref_phis)))
    assert np.all(np.diff(phis) <= 1e-12 * np.abs(phis[:-1]))
    assert float(I.min()) >= prob.M * (1 - 1e-7)
    assert np.all(hist[:, 0, 4] >= 0)
    assert e_phi < CG_TOL[prec]["phi"] and e_img < CG_TOL[prec]["img"]
    assert abs(phis[0] - ref_phis[0]) < CG_TOL[prec]["first"] * abs(ref_phis[0])


def test_shared_graph_replay_and_checkpoint_bitwise():
    """Graph replays equal eager steps, and a checkpoint taken mid-run
    resumes to the same bits, in shared mode."""
    _cuda()
    prob = _ragged(seed=45)
    ctx = prob.context("bf16x3", mode="shared")
    I = ctx.image()
    ctx.cg_init(I)
    ctx.cg_run(I, 2, graph=False)
    blob = ctx.get_state()
    I_mid = I.clone()
    h_eager = ctx.cg_run(I, 3, graph=False).clone()
    I_eager = I.clone()
    I.copy_(I_mid)
    ctx.set_state(blob)
    h_graph = ctx.cg_run(I, 3, graph=True).clone()
    torch.cuda.synchronize()
    assert torch.equal(h_eager, h_graph)
    assert torch.equal(I_eager, I)


def test_shared_rejects_cube_shaped_image():
    _cuda()
    prob = _ragged(seed=46)
    ctx = prob.context("fp32", mode="shared")
    with pytest.raises(ValueError):
        ctx.phi_and_grad(torch.ones((3, prob.n, prob.n), dtype=torch.float32, device="cuda"))
