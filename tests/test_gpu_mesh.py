"""Level set and target field on a background mesh (multilinear interpolation of node
values, projection r <- r - phi N): the HIP path against the oracle.

A single step from identical inputs is held to the same per-quantity tolerances as every other
configuration.  Over many steps: particles stay in the positive phase or on its boundary,
surface particles sit on the zero level of the interpolated level set (to the FP32 precision
of the projection), the surface population and interface statistics stay close to the
oracle's, and no non-finite value appears.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_07925_amd import workloads as W
from tests import parity_util as PU

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_07925_amd import mpsph as M
    M.lib()
    return torch


def _state(dim, n, seed, n_colours=6):
    spec = W.levelset_ball(n, dim=dim)
    cfg = dict(spec=spec, seed=seed, init="random", n_colours=n_colours)
    x, col, typ = W.make_state(cfg)
    return dict(spec, n=x.shape[0]), x.astype(np.float32), col, typ


@pytest.mark.parametrize("dim,n", [(2, 3000), (3, 6000)])
def test_single_step_parity(torch_cuda, dim, n):
    spec, x32, col, typ = _state(dim, n, 7 + dim)
    s0 = O.OracleParams(spec).s0
    rep = {}
    errs = PU.check_single_step(spec, s0, x32, col, typ, report=rep)
    print(dim, {k: f"{v:.2e}" for k, v in errs.items()}, rep["counts"])


def test_many_steps_stay_on_the_level_set(torch_cuda):
    torch = torch_cuda
    from paper_1906_07925_amd import mpsph as M
    spec, x32, col, typ = _state(3, 6000, 21)
    s0 = O.OracleParams(spec).s0
    R = M.Relaxer(spec, n=x32.shape[0], s0=s0)
    R.load(torch.from_numpy(x32).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    R.step(60)
    m = R.metrics()
    x, t = (v.cpu().numpy() for v in R.store())
    R.close()
    op = O.OracleParams(spec, s0=s0)
    phi, _ = O.grid_interp(op, "phi", x.astype(np.float64))
    surf = t > 0
    assert m["nonfinite"] == 0 and surf.sum() > 0 and np.all(t <= 1)
    # positive phase or its boundary; surface particles on the zero level (one node spacing is
    # 1/47, the FP32 projection leaves ~1e-6)
    assert np.all(phi[~surf] > -1e-6)
    assert np.max(np.abs(phi[surf])) < 1e-5
    # the oracle's own 60-step run from the same input: the surface population and interface
    # size agree to a few percent (the trajectories diverge chaotically)
    xo, to = x32.astype(np.float64), typ.copy()
    for k in range(60):
        xo, to, ro = O.step(op, xo, col, to, k, want=())
    assert abs((to > 0).sum() - surf.sum()) <= 0.05 * (to > 0).sum() + 5
    assert abs(m["interface_pairs"] - ro["interface_pairs"]) <= 0.05 * ro["interface_pairs"]
