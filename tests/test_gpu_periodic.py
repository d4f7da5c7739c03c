"""Periodic box on the GPU (no walls, minimum-image separations, positions wrapped into
[lo, hi)): the lattice invariants of the method and single-step parity with the oracle.

  * a perfect lattice with h = 1.3 dx: every particle has the density of the lattice sum the
    oracle computes (closed-form neighbourhood, all equal), and the pair force cancels by
    symmetry (|a| is rounding noise against the sum of |pair terms|);
  * random particles: the single step against the oracle at the standard tolerances, total
    momentum of the pair forces vanishing, and positions wrapped into the box.
"""
import numpy as np
import pytest

from oracle import oracle as O
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


def _spec(dim, n, **kw):
    s = dict(dim=dim, geometry="periodic", lo=(0.0,) * dim, hi=(1.0,) * dim, field="uniform", n=n)
    s.update(kw)
    return s


def _lattice(dim, per):
    ax = (np.arange(per) + 0.5) / per
    g = np.meshgrid(*([ax] * dim), indexing="ij")
    return np.stack([v.reshape(-1) for v in g], axis=1)


@pytest.mark.parametrize("dim,per", [(2, 32), (3, 16)])
def test_lattice_density_and_zero_force(torch_cuda, dim, per):
    n = per ** dim
    x = _lattice(dim, per).astype(np.float32)
    spec = _spec(dim, n, s0=1.0 / per)
    col = np.zeros(n, np.int32)
    typ = np.zeros(n, np.int32)
    m, g = PU.gpu_run(spec, 1.0 / per, x, col, typ, fields=("rho", "a", "a_abs"))
    _, _, r = O.step(O.OracleParams(spec, s0=1.0 / per), x.astype(np.float64), col, typ, 0)
    assert np.max(np.abs(g["rho"] / r["rho"][0] - 1.0)) < 2e-6
    assert m["pairs"] == r["pairs"]
    assert np.max(np.linalg.norm(g["a"], axis=1)) <= 1e-6 * np.max(g["a_abs"])


@pytest.mark.parametrize("dim,n", [(2, 1500), (3, 1200)])
def test_random_single_step_parity(torch_cuda, dim, n):
    rng = np.random.Generator(np.random.PCG64(dim * 100 + 7))
    x = rng.uniform(0.0, 1.0, size=(n, dim)).astype(np.float32)
    col = rng.integers(0, 5, size=n).astype(np.int32)
    typ = np.zeros(n, np.int32)
    spec = _spec(dim, n)
    s0 = O.OracleParams(spec).s0
    rep = {}
    errs = PU.check_single_step(spec, s0, x, col, typ, report=rep)
    print(dim, {k: f"{v:.2e}" for k, v in errs.items()}, rep["counts"])
    m, g = PU.gpu_run(spec, s0, x, col, typ, steps=20, fields=("a", "a_abs"))
    assert np.linalg.norm(g["a"].sum(0)) <= 1e-6 * g["a_abs"].sum()
    assert np.all((g["x1"] >= 0.0) & (g["x1"] < 1.0)) and m["nonfinite"] == 0
