"""Projected CG on the GPU against the oracle's CG, graph replay, checkpoint
and resume, determinism, channel batching with uneven and empty channels."""
import numpy as np
import pytest

import oracle
from oracle import cg as ocg
from _common import CG_TOL, TOL, Problem, flush, rel, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle_cg(prob, c, iters, I0):
    ch = prob.chans[c]
    p = ocg.Problem(prob.n, prob.cell, ch["u"], ch["v"], ch["vis"], ch["w"], prob.beam(c), prob.M, prob.lam)
    return ocg.projected_cg(p, iters, I0=I0)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3"])
def test_cg_trajectory_c1(prec):
    _cuda()
    ds = synth.make_config(1)
    iters = ds.cg_iters
    flush(f"cg trajectory c1 {prec} {iters} iterations")
    prob = Problem.from_dataset(ds)
    I_ref, traj = _oracle_cg(prob, 0, iters, None)
    ctx = prob.context(prec)
    I = ctx.image()
    ctx.cg_init(I, init_to_floor=True)
    hist = ctx.cg_run(I, iters, graph=False).cpu().numpy()
    ctx.check()
    phis = hist[:, 0, 0]
    ref_phis = np.array([t["phi"] for t in traj])
    assert len(traj) == iters
    e_phi = np.max(np.abs(phis - ref_phis) / np.abs(ref_phis))
    e_img = rel(I.cpu().numpy()[0], I_ref)
    alphas = hist[:, 0, 3]
    e_alpha = np.max(np.abs(alphas - [t["alpha"] for t in traj]) / np.abs([t["alpha"] for t in traj]))
    flush(f"  max rel phi {e_phi:.2e}, final image {e_img:.2e}, alpha {e_alpha:.2e}")
    flush("  alpha gpu/oracle: " + " ".join(f"{x:.4f}" for x in alphas / np.array([t["alpha"] for t in traj])))
    flush("  phi rel err: " + " ".join(f"{x:.1e}" for x in np.abs(phis - ref_phis) / np.abs(ref_phis)))
    flush("  alpha_max hit oracle: " + "".join("1" if t["alpha"] == t["alpha_max"] else "0" for t in traj))
    flush("  alpha_max hit gpu:    " + "".join("1" if x == y else "0" for x, y in zip(alphas, hist[:, 0, 6])))
    assert np.all(np.diff(phis) <= 1e-12 * np.abs(phis[:-1]))
    assert float(I.min()) >= ds.prior_m * (1 - 1e-7)
    assert np.all(hist[:, 0, 4] >= 0)
    assert e_phi < CG_TOL[prec]["phi"] and e_img < CG_TOL[prec]["img"]
    assert abs(phis[0] - ref_phis[0]) < CG_TOL[prec]["first"] * abs(ref_phis[0])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cg_trajectory_without_entropy(prec):
    """lambda = 0 (no entropy term: positivity-constrained least squares,
    phi'' from the chi^2 part alone, so the line search's entropy sums are
    zero): the c1 trajectory against the oracle's CG, same bars as with the
    entropy."""
    _cuda()
    ds = synth.make_config(1)
    iters = 12
    flush(f"cg trajectory c1 lambda=0 {prec} {iters} iterations")
    prob = Problem.from_dataset(ds)
    prob.lam = 0.0
    I_ref, traj = _oracle_cg(prob, 0, iters, None)
    ctx = prob.context(prec)
    I = ctx.image()
    ctx.cg_init(I, init_to_floor=True)
    hist = ctx.cg_run(I, iters, graph=True).cpu().numpy()
    phis = hist[:, 0, 0]
    ref_phis = np.array([t["phi"] for t in traj])
    n = min(len(traj), iters)
    e_phi = np.max(np.abs(phis[:n] - ref_phis[:n]) / np.abs(ref_phis[:n]))
    e_img = rel(I.cpu().numpy()[0], I_ref)
    flush(f"  {len(traj)} oracle steps; max rel phi {e_phi:.2e}, final image {e_img:.2e}")
    assert len(traj) == iters
    assert np.all(np.diff(phis) <= 1e-12 * np.abs(phis[:-1]))
    assert float(I.min()) >= ds.prior_m * (1 - 1e-7)
    assert e_phi < CG_TOL[prec]["phi"] and e_img < CG_TOL[prec]["img"]


def test_graph_replay_equals_eager():
    """Each graph replay, with eager work and synchronisation in between,
    gives the same bits as the eager step."""
    _cuda()
    flush("graph replay vs eager, c1 fp32")
    ds = synth.make_config(1)
    prob = Problem.from_dataset(ds)
    a = prob.context("fp32")
    b = prob.context("fp32")
    Ia, Ib = a.image(), b.image()
    a.cg_init(Ia)
    b.cg_init(Ib)
    for t in range(6):
        sa = a.cg_step(Ia)
        hb = b.cg_run(Ib, 1, graph=True)
        torch.cuda.synchronize()
        junk = (Ib * 2.0).sum().item()   # eager work between replays
        assert np.isfinite(junk)
        assert torch.equal(Ia, Ib), f"replay {t}"
        assert torch.equal(sa, hb[0]), f"replay {t} scalars"
    hb = b.cg_run(Ib, 3, graph=True)
    for t in range(3):
        sa = a.cg_step(Ia)
        assert torch.equal(sa, hb[t])
    assert torch.equal(Ia, Ib)


def test_graph_replay_without_history_buffer():
    """cg_run in graph mode with no history buffer (NULL): the replays still
    advance the image exactly as eager steps do, and a later run with a
    buffer starts its rows at 0."""
    _cuda()
    flush("graph replay without a history buffer, c1 fp32")
    ds = synth.make_config(1)
    prob = Problem.from_dataset(ds)
    a = prob.context("fp32")
    b = prob.context("fp32")
    Ia, Ib = a.image(), b.image()
    a.cg_init(Ia)
    b.cg_init(Ib)
    b._call("uvmem_cg_run", b._img(Ib).data_ptr(), 3, None, 1)
    torch.cuda.synchronize()
    for _ in range(3):
        a.cg_step(Ia)
    assert torch.equal(Ia, Ib)
    hb = b.cg_run(Ib, 2, graph=True)
    for t in range(2):
        sa = a.cg_step(Ia)
        assert torch.equal(sa, hb[t]), t
    assert torch.equal(Ia, Ib)


def test_graph_replay_equals_eager_several_images():
    """Cube mode with three channels (one empty): each graph replay writes
    the same history rows, bit for bit, as the eager steps (with one image
    the gradient pass writes the history row itself; with several a
    separate copy follows the step)."""
    _cuda()
    flush("graph replay vs eager, three-channel cube fp32")
    prob = Problem.random(64, [1500, 0, 777], seed=41, lam=0.05)
    a = prob.context("fp32")
    b = prob.context("fp32")
    Ia, Ib = a.image(), b.image()
    a.cg_init(Ia)
    b.cg_init(Ib)
    hb = b.cg_run(Ib, 4, graph=True)
    torch.cuda.synchronize()
    for t in range(4):
        sa = a.cg_step(Ia)
        assert torch.equal(sa, hb[t]), f"replay {t} scalars"
    assert torch.equal(Ia, Ib)
    hb2 = b.cg_run(Ib, 2, graph=True)   # a second run restarts the history rows
    for t in range(2):
        sa = a.cg_step(Ia)
        assert torch.equal(sa, hb2[t]), f"second run, replay {t} scalars"


def test_checkpoint_resume_bitwise():
    _cuda()
    flush("checkpoint/resume c1 fp32")
    ds = synth.make_config(1)
    prob = Problem.from_dataset(ds)
    ctx = prob.context("fp32")
    I = ctx.image()
    ctx.cg_init(I)
    ctx.cg_run(I, 4, graph=False)
    blob = ctx.get_state()
    I_save = I.clone()
    ctx.cg_run(I, 4, graph=False)
    I_straight = I.clone()
    I.copy_(I_save)
    ctx.set_state(blob)
    ctx.cg_run(I, 4, graph=False)
    assert torch.equal(I, I_straight)


def test_phi_grad_deterministic():
    _cuda()
    ds = synth.make_config(1)
    prob = Problem.from_dataset(ds)
    ctx = prob.context("fp32")
    I = torch.tensor(synth.eval_images(ds, "P3"), dtype=torch.float32, device="cuda")
    s1, g1 = ctx.phi_and_grad(I)
    s2, g2 = ctx.phi_and_grad(I)
    assert torch.equal(s1, s2) and torch.equal(g1, g2)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3"])
def test_channel_batching_uneven_and_empty(prec):
    """Several channels of different sizes and one empty channel in one set
    of launches: each channel equals its own oracle evaluation; the empty one
    has chi^2 = 0 and grad = lambda (ln(I/M) + 1)."""
    _cuda()
    flush(f"batching {prec}")
    prob = Problem.random(64, [1500, 0, 333, 4097], seed=11, lam=0.05)
    ctx = prob.context(prec)
    img = synth.random_image(64, 12, lo=1e-3, hi=1.0, n_chan=4)
    I = torch.tensor(img, dtype=ctx.dtype, device="cuda")
    scal, grad = ctx.phi_and_grad(I)
    scal, grad = scal.cpu().numpy(), grad.cpu().numpy()
    Ih = I.cpu().numpy().astype(np.float64)
    offs = prob.offsets()
    R = ctx.residual().cpu().numpy()
    for c in range(4):
        ref = prob.oracle_phi_grad(c, Ih[c])
        if c == 1:
            assert scal[c, 1] == 0.0
        else:
            assert abs(scal[c, 1] - ref["chi2"]) < TOL[prec] * ref["chi2"]
            assert rel(R[offs[c]:offs[c + 1]], ref["R"]) < TOL[prec]
        assert abs(scal[c, 0] - ref["phi"]) < TOL[prec] * abs(ref["phi"])
        assert rel(grad[c], ref["grad"]) < TOL[prec], c


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_many_small_uneven_channels(prec):
    """384 channels of 0 to 40 visibilities on a 32^2 image in one set of
    launches (work tables far longer than the chip is wide): Phi, chi^2,
    the gradients and the residuals of all channels match their oracle
    evaluations, and graph-replayed CG steps equal the eager ones bit for
    bit."""
    _cuda()
    rng = np.random.default_rng(77)
    nv = [int(x) for x in rng.integers(0, 41, 384)]
    nv[5] = 0
    flush(f"many small channels {prec}: {len(nv)} channels, {sum(nv)} visibilities")
    prob = Problem.random(32, nv, seed=61, lam=0.05)
    ctx = prob.context(prec)
    img = synth.random_image(32, 62, lo=1e-3, hi=1.0, n_chan=len(nv))
    I = torch.tensor(img, dtype=ctx.dtype, device="cuda")
    scal, grad = ctx.phi_and_grad(I)
    scal, grad = scal.cpu().numpy(), grad.cpu().numpy()
    R = ctx.residual().cpu().numpy()
    Ih = I.cpu().numpy().astype(np.float64)
    # norm-wise over all channels at the parity bar, as the other parity
    # tests; each channel within ten times it (a channel with a handful of
    # visibilities inherits the cancellation in R = V - V_o, but a channel
    # mixed up with another would be off by order one)
    refs = [prob.oracle_phi_grad(c, Ih[c]) for c in range(len(nv))]
    phi_ref = np.array([r["phi"] for r in refs])
    chi_ref = np.array([r["chi2"] for r in refs])
    g_ref = np.stack([r["grad"] for r in refs])
    R_ref = np.concatenate([r["R"] for r in refs])
    e_phi, e_chi, e_g, e_R = rel(scal[:, 0], phi_ref), rel(scal[:, 1], chi_ref), rel(grad, g_ref), rel(R, R_ref)
    worst = max(max(abs(scal[c, 0] - phi_ref[c]) / abs(phi_ref[c]), rel(grad[c], g_ref[c])) for c in range(len(nv)))
    flush(f"  phi {e_phi:.2e} chi2 {e_chi:.2e} grad {e_g:.2e} R {e_R:.2e}; worst channel {worst:.2e}")
    assert max(e_phi, e_chi, e_g, e_R) < TOL[prec]
    assert worst < 10 * TOL[prec]
    assert all(scal[c, 1] == 0.0 for c in range(len(nv)) if nv[c] == 0)
    a, b = prob.context(prec), prob.context(prec)
    Ia, Ib = a.image(), b.image()
    a.cg_init(Ia)
    b.cg_init(Ib)
    hb = b.cg_run(Ib, 3, graph=True)
    torch.cuda.synchronize()
    for t in range(3):
        sa = a.cg_step(Ia)
        assert torch.equal(sa, hb[t]), t
    assert torch.equal(Ia, Ib)


def test_cg_batched_channels_match_single_channel_runs():
    """Cube mode: channels are independent, so a batched CG equals separate
    single-channel CG runs of each channel (up to the split-K chunking of the
    adjoint, which depends on the total visibility count)."""
    _cuda()
    prob = Problem.random(64, [900, 2500, 0], seed=21, lam=0.02)
    ctx = prob.context("fp64")
    I = ctx.image()
    ctx.cg_init(I)
    hb = ctx.cg_run(I, 5, graph=False).cpu().numpy()
    for c in (0, 1, 2):
        single = Problem(prob.n, prob.cell, [prob.chans[c]], prob.M, prob.lam).context("fp64")
        Is = single.image()
        single.cg_init(Is)
        hs = single.cg_run(Is, 5, graph=False).cpu().numpy()
        assert rel(Is[0].cpu().numpy(), I[c].cpu().numpy()) < 1e-10, c
        assert np.allclose(hs[:, 0, :6], hb[:, c, :6], rtol=1e-9, atol=1e-300), c


def test_phi_function_autograd_fd_fp64():
    """PhiFunction backward vs central differences of the GPU FP64 Phi."""
    _cuda()
    from paper_1703_02920_amd.uvmem import PhiFunction
    prob = Problem.random(16, [200], seed=31, lam=0.1, fwhm_px=6)
    ctx = prob.context("fp64")
    I = torch.tensor(synth.random_image(16, 31, lo=0.05, hi=1.0), dtype=torch.float64, device="cuda",
                     requires_grad=True)
    phi = PhiFunction.apply(I, ctx)
    phi.backward()
    g = I.grad.detach().cpu().numpy()[0]
    x0 = I.detach().clone()
    fd = np.zeros((16, 16))
    for p in range(0, 256, 7):
        i, j = divmod(p, 16)
        h = 1e-5 * float(x0[0, i, j])
        xp = x0.clone(); xp[0, i, j] += h
        xm = x0.clone(); xm[0, i, j] -= h
        fp = float(ctx.phi_and_grad(xp)[0][0, 0])
        fm = float(ctx.phi_and_grad(xm)[0][0, 0])
        fd[i, j] = (fp - fm) / (2 * h)
        assert abs(fd[i, j] - g[i, j]) < 1e-6 * max(1.0, abs(g[i, j])), (i, j, fd[i, j], g[i, j])


def test_domain_flag_and_errors():
    _cuda()
    from paper_1703_02920_amd.uvmem import EDOMAIN, ESTATE, UvmemError
    prob = Problem.random(64, [300], seed=41)
    ctx = prob.context("fp32")
    I = ctx.image(fill=1e-3)
    I[0, 3, 4] = 0.0
    ctx.phi_and_grad(I)
    with pytest.raises(UvmemError) as ei:
        ctx.check()
    assert ei.value.code == EDOMAIN
    ctx.check()          # flag cleared
    with pytest.raises(UvmemError) as ei:
        ctx.set_prior(1e-3, 0.1)
    assert ei.value.code == ESTATE
    with pytest.raises(UvmemError) as ei:
        ctx.cg_step(I)
    assert ei.value.code == ESTATE
    # u beyond 4096 cycles per pixel is rejected before anything reaches the GPU
    from paper_1703_02920_amd.uvmem import EINVAL, Context
    c2 = Context(64, 1, "fp32")
    ch = prob.chans[0]
    u = ch["u"].copy()
    u[7] = 4097.0 / prob.cell
    with pytest.raises(UvmemError) as ei:
        c2.set_uv(0, u, ch["v"], prob.cell)
    assert ei.value.code == EINVAL and "cycles per pixel" in str(ei.value)
    u[7] = 4095.0 / prob.cell
    c2.set_uv(0, u, ch["v"], prob.cell)


@pytest.mark.parametrize("case", ["c1-fp64", "c1-fp32", "cube3-fp32", "shared3-fp32", "shared3-bf16x3"])
def test_restart_when_direction_is_not_descent(case):
    """The CG's restart (steepest descent when the projected direction does
    not descend, R13): a checkpoint whose direction is +gt with beta = 1 makes
    the next direction -gt + gt = 0, so gt . d = 0 >= 0 and the step must
    restart with d = -gt.  That is the direction of the first step after
    cg_init (d = -gt, beta = 0), so both steps give the same bits.  Cases:
    the 64^2 workload, and three uneven channels (96^2) as three images or
    one shared image (the restart rewrites every channel's B = A o d)."""
    import struct
    from paper_1703_02920_amd.uvmem import NSCAL, S_BETA
    _cuda()
    name, prec = case.split("-")
    flush(f"restart path {case}")
    if name == "c1":
        ds = synth.make_config(1)
        prob, mode = Problem.from_dataset(ds), "cube"
    else:
        prob = Problem.random(96, [1500, 700, 2300], seed=37)
        mode = "shared" if name.startswith("shared") else "cube"
    n_img = 1 if mode == "shared" else prob.n_chan
    ctx = prob.context(prec, mode=mode)
    I = ctx.image()
    ctx.cg_init(I, init_to_floor=True)
    blob = bytearray(ctx.get_state())
    I0 = I.clone()
    s_a = ctx.cg_step(I).clone()
    I_a = I.clone()
    # blob: 48-byte header, d, gt, g (n_img x N x N of the real type),
    # R (complex128 per visibility), scalars, CG flags (uvmem.h)
    hdr, elem = 48, (8 if prec == "fp64" else 4)
    img = n_img * prob.n * prob.n * elem
    ztot = sum(len(ch["u"]) for ch in prob.chans)
    blob[hdr:hdr + img] = blob[hdr + img:hdr + 2 * img]          # d := +gt
    for m in range(n_img):                                        # beta := 1
        struct.pack_into("=d", blob, hdr + 3 * img + 16 * ztot + 8 * (m * NSCAL + S_BETA), 1.0)
    I.copy_(I0)
    ctx.set_state(bytes(blob))
    s_b = ctx.cg_step(I).clone()
    ctx.check()
    flush(f"  plain first step phi {float(s_a[0, 0]):.12e}, restarted {float(s_b[0, 0]):.12e}")
    assert bool((s_a[:, 3] > 0.0).all())
    assert torch.equal(I, I_a)
    assert torch.equal(s_a, s_b)
