"""mpsph_create_static: a context whose workspace is the library's static scratch array (no
device allocation) computes exactly what a context of mpsph_create computes with the same
kernels, call after call on the same array, and refuses what does not fit."""
import numpy as np
import pytest

from paper_1906_07925_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_07925_amd import mpsph as M
    M.lib()
    return torch


def _state(name, scale):
    cfg = W.config(name, scale=scale)
    x, col, typ = W.make_state(cfg)
    return dict(cfg["spec"], n=x.shape[0]), x.astype(np.float32), col, typ


def _run(torch, spec, x, col, typ, steps, static):
    from paper_1906_07925_amd import mpsph as M
    R = M.Relaxer(spec, n=x.shape[0], static=static)
    R.load(torch.from_numpy(x).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    R.step(steps)
    m = R.metrics()
    xs, ts = R.store()
    R.close()
    return xs.cpu().numpy(), ts.cpu().numpy(), m


def test_static_context_matches_allocating_context(torch_cuda):
    """Two static contexts in a row on the same array, the second with a smaller 2D input than
    the first 3D one: each ends bit-identical to an mpsph_create context of the same input."""
    torch = torch_cuda
    for name, scale, steps in (("cube_inclusion_2m", 0.05, 6), ("square_4k", 0.5, 8)):
        spec, x, col, typ = _state(name, scale)
        print(f"[no-alloc] {name} n={x.shape[0]} steps={steps}", flush=True)
        xs, ts, ms = _run(torch, spec, x, col, typ, steps, static=True)
        xr, tr, mr = _run(torch, spec, x, col, typ, steps, static=False)
        assert np.array_equal(xs, xr) and np.array_equal(ts, tr), name
        assert ms == mr, name
        assert ms["pairs"] > 0 and ms["nonfinite"] == 0


def test_static_context_limits(torch_cuda):
    """A problem whose workspace exceeds the array is refused with its own status; a second
    static context on the same device is refused while the first exists and accepted after it
    is destroyed; the gradient driver, which allocates, is refused on a static context."""
    torch = torch_cuda
    from paper_1906_07925_amd import mpsph as M
    spec, x, col, typ = _state("cube_inclusion_2m", 0.5)
    assert M.workspace_bytes(spec, x.shape[0]) > 64 << 20
    with pytest.raises(M.MpsphError) as e:
        M.Relaxer(spec, n=x.shape[0], static=True)
    assert e.value.code == 7
    spec, x, col, typ = _state("square_4k", 0.25)
    A = M.Relaxer(spec, n=x.shape[0], static=True)
    with pytest.raises(M.MpsphError) as e:
        M.Relaxer(spec, n=x.shape[0], static=True)
    assert e.value.code == 4
    A.load(torch.from_numpy(x).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    with pytest.raises(M.MpsphError) as e:
        A.grad(1)
    assert e.value.code == 6
    A.close()
    B = M.Relaxer(spec, n=x.shape[0], static=True)
    B.load(torch.from_numpy(x).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    B.step(2)
    assert B.metrics()["pairs"] > 0
    B.close()
