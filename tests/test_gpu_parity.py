"""Parity of the HIP path with the FP64 oracle, element by element, on small
seeded problems that span several tiles and a ragged tail."""
import numpy as np
import pytest

from _common import TOL, Problem, flush, rel, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


PRECS = ["fp64", "fp32", "bf16x3", "fp16x3"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,nvis", [(64, 1000), (128, 777), (100, 321), (256, 1203)])
def test_forward_parity(prec, n, nvis):
    _cuda()
    flush(f"forward parity {prec} n={n} nvis={nvis}")
    prob = Problem.random(n, [nvis], seed=n + nvis)
    ctx = prob.context(prec)
    img = synth.random_image(n, 5, lo=1e-3, hi=1.0)[0]
    I = torch.tensor(img[None], dtype=ctx.dtype, device="cuda")
    V = ctx.forward(I).cpu().numpy()
    ref = prob.oracle_forward(0, I.cpu().numpy()[0].astype(np.float64))
    err = rel(V, ref)
    flush(f"  rel err {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,nvis", [(64, 1000), (128, 777), (100, 321), (256, 1203)])
def test_adjoint_parity(prec, n, nvis):
    _cuda()
    flush(f"adjoint parity {prec} n={n} nvis={nvis}")
    prob = Problem.random(n, [nvis], seed=3 * n + nvis)
    ctx = prob.context(prec)
    rng = np.random.default_rng(n + nvis)
    coef = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
    G = ctx.adjoint(torch.tensor(coef, dtype=torch.complex128, device="cuda")).cpu().numpy()[0]
    ref = prob.oracle_adjoint(0, coef)
    err = rel(G, ref)
    flush(f"  rel err {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("which", ["P1", "P3"])
def test_phi_grad_parity_c1(prec, which):
    _cuda()
    flush(f"phi/grad parity c1 {prec} {which}")
    ds = synth.make_config(1)
    prob = Problem.from_dataset(ds)
    ctx = prob.context(prec)
    img = synth.eval_images(ds, which)
    I = torch.tensor(img, dtype=ctx.dtype, device="cuda")
    scal, grad = ctx.phi_and_grad(I)
    scal = scal.cpu().numpy()
    ref = prob.oracle_phi_grad(0, I.cpu().numpy()[0].astype(np.float64))
    e_phi = abs(scal[0, 0] - ref["phi"]) / abs(ref["phi"])
    e_chi = abs(scal[0, 1] - ref["chi2"]) / abs(ref["chi2"])
    e_g = rel(grad.cpu().numpy()[0], ref["grad"])
    e_r = rel(ctx.residual().cpu().numpy(), ref["R"])
    flush(f"  phi {e_phi:.2e} chi2 {e_chi:.2e} grad {e_g:.2e} R {e_r:.2e}")
    assert e_phi < TOL[prec] and e_chi < TOL[prec] and e_g < TOL[prec] and e_r < TOL[prec]
    S_ref = ref["S"]
    assert abs(scal[0, 2] - S_ref) <= TOL[prec] * max(abs(S_ref), 1e-300) + 1e-12 * ds.n ** 2 * ds.prior_m


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_forward_parity_short_last_round(prec):
    """256^2: the persistent forward's last round of wave tiles (16
    visibilities for FP32, 32 for the split precisions) is short, at most two
    tiles per workgroup, so its tiles are split across the waves of their
    workgroups (row slices for FP32, column slices for the split forward);
    the visibilities of that round, a ragged last tile among them, match the
    oracle like the rest."""
    _cuda()
    n = 256
    tv = 16 if prec == "fp32" else 32
    # visibility counts tried in order until the schedule leaves a short last round
    for nvis in (20001, 35961, 28001, 44001):
        prob = Problem.random(n, [nvis], seed=91)
        ctx = prob.context(prec)
        info = ctx.info()
        nwg = info["n_fwd_wgs"] // info["n_fwd_parts"]
        ntiles = -(-nvis // tv)
        nfull = ntiles // (8 * nwg) * (8 * nwg)
        if 0 < ntiles - nfull <= 2 * nwg:
            break
        ctx.close()
    else:
        pytest.fail("no tried size leaves a short last round")
    flush(f"forward short last round {prec} n={n} nvis={nvis} nwg={nwg} leftover tiles={ntiles - nfull}")
    img = synth.random_image(n, 6, lo=1e-3, hi=1.0)[0]
    I = torch.tensor(img[None], dtype=ctx.dtype, device="cuda")
    V = ctx.forward(I).cpu().numpy()
    ref = prob.oracle_forward(0, I.cpu().numpy()[0].astype(np.float64))
    tail = slice(nfull * tv, nvis)
    e_all, e_tail = rel(V, ref), rel(V[tail], ref[tail])
    flush(f"  rel err {e_all:.3e}, last round ({nvis - nfull * tv} visibilities) {e_tail:.3e}")
    assert e_all < TOL[prec] and e_tail < TOL[prec]
