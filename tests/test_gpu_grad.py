"""The library's hand-written adjoint (mpsph_grad) against the float64 autograd oracle
(oracle/grad.py, itself pinned to central differences through the C oracle).

FP32 forward and reverse passes against FP64: the loss agrees to 1e-5 relative, the gradients
normwise to 2e-3 (the reverse pass accumulates the FP32 rounding of every pair term of every
step; the per-step relative rounding is ~1e-6 of the condition scale, amplified over the steps
by the Jacobians).  The checkpoint interval only changes what is recomputed: gradients are
bit-identical for every interval.
"""
import numpy as np
import pytest

from oracle import grad as G
from paper_1906_07925_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 4
LAM = 1.0


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_07925_amd import mpsph as M
    M.lib()
    return torch


def _case(n_side=10, seed=3, scale_c=0.1, n_colours=6):
    n = n_side ** 3
    rng = np.random.Generator(np.random.PCG64(seed))
    spec = W.rbf_cube(n)
    coeff = rng.normal(0.0, scale_c, size=spec["n_rbf"])
    cfg = dict(spec=spec, seed=W.BASE_SEED + 4, init="lattice", per_axis=n_side, n_colours=n_colours)
    x, col, typ = W.make_state(cfg)
    return dict(spec, n=n), x.astype(np.float32), col, typ, coeff


def _gpu(torch, spec, x32, col, typ, coeff, steps, ckpt, want_pos=True):
    from paper_1906_07925_amd import mpsph as M
    R = M.Relaxer(dict(spec, rbf_coeff=coeff), n=x32.shape[0])
    R.load(torch.from_numpy(x32).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    loss, gc, gx = R.grad(steps, ckpt, LAM, n_rbf=spec["n_rbf"], want_pos=want_pos)
    xs, ts = R.store()
    m = R.metrics()
    R.close()
    return loss, gc, (gx.cpu().numpy().astype(np.float64) if gx is not None else None), xs.cpu().numpy(), m


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("steps", [0, 1, STEPS])
def test_gradient_matches_oracle(torch_cuda, steps):
    spec, x32, col, typ, coeff = _case()
    pr = G.Problem(spec, spec["s0"], col, typ)
    L0, gc0, gx0, _, _, _ = G.run(pr, x32.astype(np.float64), coeff, steps, LAM, want_x0_grad=True)
    L, gc, gx, _, _ = _gpu(torch_cuda, spec, x32, col, typ, coeff, steps, 2)
    print("steps", steps, "loss", L, L0, "coeff", _rel(gc, gc0), "pos", _rel(gx, gx0))
    assert abs(L - L0) <= 1e-5 * abs(L0)
    assert _rel(gc, gc0) <= 2e-3
    assert _rel(gx, gx0) <= 2e-3
    # the direction of steepest descent agrees component by component where it matters
    big = np.abs(gc0) > 0.1 * np.max(np.abs(gc0))
    assert np.all(np.sign(gc[big]) == np.sign(gc0[big]))


def test_checkpoint_interval_does_not_change_the_gradient(torch_cuda):
    spec, x32, col, typ, coeff = _case(n_side=8)
    ref = _gpu(torch_cuda, spec, x32, col, typ, coeff, 7, 1)
    for ck in (2, 3, 7, 10):
        got = _gpu(torch_cuda, spec, x32, col, typ, coeff, 7, ck)
        assert got[0] == ref[0]
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2]), ck
        assert np.array_equal(got[3], ref[3])


def test_grad_advances_the_state_like_step(torch_cuda):
    torch = torch_cuda
    from paper_1906_07925_amd import mpsph as M
    spec, x32, col, typ, coeff = _case(n_side=8)
    _, _, _, xg, mg = _gpu(torch, spec, x32, col, typ, coeff, 5, 2, want_pos=False)
    R = M.Relaxer(dict(spec, rbf_coeff=coeff), n=x32.shape[0])
    R.load(torch.from_numpy(x32).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    R.step(5)
    xs = R.store()[0].cpu().numpy()
    ms = R.metrics()
    R.close()
    assert np.array_equal(xg, xs)
    assert mg == ms


def test_set_field_coeff_matches_fresh_context(torch_cuda):
    torch = torch_cuda
    from paper_1906_07925_amd import mpsph as M
    spec, x32, col, typ, coeff = _case(n_side=8)
    b = M.Relaxer(dict(spec, rbf_coeff=coeff), n=x32.shape[0])
    # the same cell grid (the automatic choice depends on the field's smallest spacing)
    a = M.Relaxer(dict(spec, rbf_coeff=np.zeros_like(coeff)), n=x32.shape[0], cell_log2=b.cell_log2())
    a.set_field_coeff(coeff)
    for R in (a, b):
        R.load(torch.from_numpy(x32).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
        R.step(3)
    assert torch.equal(a.store()[0], b.store()[0])
    a.close()
    b.close()


def test_autograd_function(torch_cuda):
    torch = torch_cuda
    from paper_1906_07925_amd import mpsph as M
    spec, x32, col, typ, coeff = _case(n_side=8)
    R = M.Relaxer(dict(spec, rbf_coeff=coeff), n=x32.shape[0])
    F = M.relax_loss_function()
    c = torch.tensor(coeff, dtype=torch.float64, requires_grad=True)
    x0 = torch.from_numpy(x32).cuda().requires_grad_(True)
    colour = torch.from_numpy(col).cuda()
    ptype = torch.from_numpy(typ).cuda()
    loss = F.apply(c, x0, R, colour, ptype, 3, 2, LAM)
    (2.0 * loss).backward()
    R2 = M.Relaxer(dict(spec, rbf_coeff=coeff), n=x32.shape[0])
    R2.load(x0.detach(), colour, ptype)
    L, gc, gx = R2.grad(3, 2, LAM, n_rbf=len(coeff), want_pos=True)
    assert float(loss.detach()) == L
    assert np.array_equal(c.grad.numpy(), 2.0 * gc)
    assert torch.equal(x0.grad, 2.0 * gx)
    R.close()
    R2.close()
