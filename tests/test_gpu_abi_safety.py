"""Error paths of the C ABI on the GPU: a finalize whose device allocation
fails leaves a context that can still be destroyed (every buffer released
once), rejected set_* calls leave the staged inputs unchanged, and the
binding refuses arrays whose length does not match the channel."""
import os

import numpy as np
import pytest

from _common import TOL, Problem, flush, rel, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("fail_at", [0, 7, 16, 29])
def test_failed_allocation_then_destroy(fail_at):
    """UVMEM_TEST_FAIL_ALLOC=k makes the k-th allocation of finalize fail: the
    call returns UVMEM_ENOMEM, the context is then destroyed (no buffer freed
    twice), and torch's allocator and a fresh context still work."""
    _cuda()
    from paper_1703_02920_amd.uvmem import ENOMEM, UvmemError
    flush(f"failed allocation {fail_at}, then destroy")
    from paper_1703_02920_amd.uvmem import Context
    prob = Problem.random(64, [700, 300], seed=51)
    bad = Context(64, 2, "fp32")
    for c, ch in enumerate(prob.chans):
        bad.set_uv(c, ch["u"], ch["v"], prob.cell)
        bad.set_vis(c, ch["vis"])
        bad.set_weights(c, ch["w"])
        bad.set_beam(c, ch["fwhm"])
    bad.set_prior(prob.M, prob.lam)
    os.environ["UVMEM_TEST_FAIL_ALLOC"] = str(fail_at)
    try:
        with pytest.raises(UvmemError) as ei:
            bad.finalize()
        code = ei.value.code
        del ei
    finally:
        del os.environ["UVMEM_TEST_FAIL_ALLOC"]
    assert code == ENOMEM
    bad.close()                       # destroy after the failed finalize
    junk = [torch.randn(1 << 20, device="cuda") for _ in range(8)]
    torch.cuda.synchronize()
    ctx = prob.context("fp32")
    img = synth.random_image(64, 51, n_chan=2)
    I = torch.tensor(img, dtype=torch.float32, device="cuda")
    scal, grad = ctx.phi_and_grad(I)
    ref = prob.oracle_phi_grad(1, I.cpu().numpy()[1].astype(np.float64))
    assert rel(grad.cpu().numpy()[1], ref["grad"]) < TOL["fp32"]
    assert all(float(t.sum()) == float(t.sum()) for t in junk)
    ctx.close()
    ctx.close()                       # a second close is a no-op


def test_rejected_set_uv_keeps_the_staged_channel():
    """A set_uv rejected for a non-finite coordinate (with a different
    length) leaves the channel's previous coordinates, data and weights in
    place: finalize then builds the same problem as without the bad call."""
    _cuda()
    from paper_1703_02920_amd.uvmem import EINVAL, Context, UvmemError
    prob = Problem.random(64, [500], seed=52)
    ch = prob.chans[0]
    ctx = Context(64, 1, "fp32")
    ctx.set_uv(0, ch["u"], ch["v"], prob.cell)
    ctx.set_vis(0, ch["vis"])
    ctx.set_weights(0, ch["w"])
    bad_u = np.concatenate([ch["u"], [np.nan, 1.0]])
    bad_v = np.concatenate([ch["v"], [0.0, 1.0]])
    with pytest.raises(UvmemError) as ei:
        ctx.set_uv(0, bad_u, bad_v, prob.cell)
    assert ei.value.code == EINVAL
    with pytest.raises(UvmemError) as ei:
        ctx.set_weights(0, -ch["w"])
    assert ei.value.code == EINVAL
    ctx.set_beam(0, ch["fwhm"])
    ctx.set_prior(prob.M, prob.lam)
    ctx.finalize()
    img = synth.random_image(64, 52)
    I = torch.tensor(img, dtype=torch.float32, device="cuda")
    scal, grad = ctx.phi_and_grad(I)
    ref = prob.oracle_phi_grad(0, I.cpu().numpy()[0].astype(np.float64))
    assert rel(grad.cpu().numpy()[0], ref["grad"]) < TOL["fp32"]
    assert abs(float(scal[0, 1]) - ref["chi2"]) < TOL["fp32"] * ref["chi2"]


def test_new_coordinates_require_new_data():
    """New coordinates of another length invalidate the channel's
    visibilities and weights: finalize refuses until they are set again."""
    _cuda()
    from paper_1703_02920_amd.uvmem import ESTATE, Context, UvmemError
    prob = Problem.random(64, [400], seed=53)
    ch = prob.chans[0]
    ctx = Context(64, 1, "fp32")
    ctx.set_uv(0, ch["u"], ch["v"], prob.cell)
    ctx.set_vis(0, ch["vis"])
    ctx.set_weights(0, ch["w"])
    ctx.set_uv(0, ch["u"][:300], ch["v"][:300], prob.cell)
    ctx.set_beam(0, ch["fwhm"])
    ctx.set_prior(prob.M, prob.lam)
    with pytest.raises(UvmemError) as ei:
        ctx.finalize()
    assert ei.value.code == ESTATE
    ctx.set_vis(0, ch["vis"][:300])
    ctx.set_weights(0, ch["w"][:300])
    ctx.finalize()


def test_binding_checks_array_lengths():
    _cuda()
    from paper_1703_02920_amd.uvmem import Context
    prob = Problem.random(32, [100], seed=54)
    ch = prob.chans[0]
    ctx = Context(32, 2, "fp32")
    with pytest.raises(ValueError):
        ctx.set_uv(0, ch["u"], ch["v"][:50], prob.cell)
    ctx.set_uv(0, ch["u"], ch["v"], prob.cell)
    with pytest.raises(ValueError):
        ctx.set_vis(0, ch["vis"][:99])
    with pytest.raises(ValueError):
        ctx.set_weights(0, np.ones(101, np.float32))
    with pytest.raises(ValueError):
        ctx.set_beam_image(0, np.ones((32, 31), np.float32))
    with pytest.raises(ValueError):
        ctx.set_vis(2, ch["vis"])
    ctx.set_vis(0, ch["vis"])
    ctx.set_weights(0, ch["w"])
    ctx.close()
