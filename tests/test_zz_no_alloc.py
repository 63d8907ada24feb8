"""The allocation-free forward model (uvmem_forward_noalloc) against the
context's uvmem_forward on the same inputs, through the C ABI: two calls in
a row, the second with a smaller problem (the fixed scratch keeps the first
call's contents), plus the oracle and the size limits."""
import numpy as np
import pytest

import oracle
from _common import TOL, flush, rel, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(n, nvis, seed):
    cell = 1.0e-6
    u, v, vis, w = synth.random_problem(n, nvis, seed, cell=cell)
    A = oracle.beam(n, cell, 0.6 * n * cell).astype(np.float32)
    img = synth.random_image(n, seed)[0].astype(np.float32)
    return cell, u, v, vis, w, A, img


def _context_forward(n, cell, u, v, vis, w, A, img):
    from paper_1703_02920_amd.uvmem import Context
    ctx = Context(n, 1, "fp32")
    ctx.set_uv(0, u, v, cell)
    ctx.set_vis(0, vis)
    ctx.set_weights(0, w)
    ctx.set_beam_image(0, A)
    ctx.set_prior(1e-3, 0.01)
    ctx.finalize()
    out = ctx.forward(torch.tensor(img[None], device="cuda")).cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("first,second", [((256, 40000), (200, 3001)), ((128, 9000), (64, 777))])
def test_noalloc_forward_matches_context_forward(first, second):
    _cuda()
    from paper_1703_02920_amd.uvmem import forward_noalloc
    outs = []
    for k, (n, nvis) in enumerate((first, second)):
        flush(f"noalloc forward call {k}: n {n}, {nvis} visibilities")
        cell, u, v, vis, w, A, img = _case(n, nvis, 300 + 17 * n + k)
        ud = torch.tensor(u, dtype=torch.float64, device="cuda")
        vd = torch.tensor(v, dtype=torch.float64, device="cuda")
        Ad = torch.tensor(A, device="cuda")
        Id = torch.tensor(img, device="cuda")
        got = forward_noalloc(n, cell, ud, vd, Id, beam=Ad)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        ref = _context_forward(n, cell, u, v, vis, w, A, img)
        e_ctx = rel(got, ref)
        idx = np.arange(0, nvis, max(1, nvis // 200))
        e_or = rel(got[idx], oracle.forward_sel(n, cell, idx, u, v, A.astype(np.float64), img.astype(np.float64)))
        flush(f"  vs uvmem_forward {e_ctx:.2e} (bitwise {np.array_equal(got, ref)}), vs oracle {e_or:.2e}")
        assert e_ctx < TOL["fp32"] and e_or < TOL["fp32"]
        outs.append(got)
    assert len(outs[1]) == second[1]


def test_noalloc_limits():
    _cuda()
    from paper_1703_02920_amd.uvmem import EINVAL, ETOOBIG, UvmemError, forward_noalloc
    n = 1024
    u = torch.zeros(200000, dtype=torch.float64, device="cuda")
    I = torch.ones(n * n, dtype=torch.float32, device="cuda")
    with pytest.raises(UvmemError) as ei:
        forward_noalloc(n, 1e-6, u, u, I)
    assert ei.value.code == ETOOBIG
    with pytest.raises(UvmemError) as ei:
        forward_noalloc(63, 1e-6, u[:10], u[:10], torch.ones(63 * 63, dtype=torch.float32, device="cuda"))
    assert ei.value.code == EINVAL
    out = forward_noalloc(64, 1e-6, u[:0], u[:0], torch.ones(64 * 64, dtype=torch.float32, device="cuda"))
    assert out.numel() == 0
