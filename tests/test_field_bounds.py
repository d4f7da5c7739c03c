"""Bounds of the target size field that the neighbour search relies on (mpsph_field_bounds,
host-only): s_min <= s <= s_max and |s(x) - s(y)| <= L |x - y| over the region's box.  The field
values come from the oracle (h = tau s, Eq. 16) on dense seeded samples, so a bound that is not
a bound fails here; for the RBF field the bounds must also stay close to the sampled extremes
(a loose bound inflates the search radius and the candidate count)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_07925_amd import mpsph as M
from paper_1906_07925_amd import workloads as W


def rbf(scale, seed):
    spec = W.rbf_cube(1 << 20)
    rng = np.random.Generator(np.random.PCG64(seed))
    return dict(spec, rbf_coeff=rng.normal(0.0, scale, size=spec["n_rbf"]))


CASES = [
    ("uniform cube", W.unit_cube(1 << 18)),
    ("annulus, radial linear", W.annulus(262144)),
    ("cube with inclusion, sphere distance", W.cube_with_inclusion(1 << 21)),
    ("rbf cube, c ~ N(0, 0.1^2)", rbf(0.1, W.BASE_SEED + 40)),
    ("rbf cube, c ~ N(0, 0.3^2)", rbf(0.3, W.BASE_SEED + 41)),
]


def field_s(spec, s0, x):
    op = O.OracleParams(spec, s0=s0)
    _, h = O.field(op, x)
    return h / op.p.tau


@pytest.mark.parametrize("case", range(len(CASES)))
def test_bounds_hold_on_dense_samples(case):
    name, spec = CASES[case]
    if not __import__("os").path.exists(M.LIB_PATH):
        pytest.fail("libmpsph.so is not built")
    b = M.field_bounds(spec, spec["n"])
    d = spec["dim"]
    lo, hi = np.asarray(spec["lo"], dtype=np.float64), np.asarray(spec["hi"], dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(W.BASE_SEED + 70 + case))
    x = rng.uniform(lo, hi, size=(200000, d))
    s = field_s(spec, b["s0"], x)
    assert b["smin"] <= s.min() * (1 + 1e-12) and s.max() <= b["smax"] * (1 + 1e-12), name
    # slopes over short random segments kept inside the box
    u = rng.normal(size=(200000, d))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    y = np.clip(x + 1e-3 * (hi - lo).max() * u, lo, hi)
    dist = np.linalg.norm(y - x, axis=1)
    ok = dist > 0
    slope = np.abs(field_s(spec, b["s0"], y) - s)[ok] / dist[ok]
    assert slope.max() <= b["lip"] * (1 + 1e-9) + 1e-12, name
    if spec["field"] == "rbf_exp":
        assert b["smax"] <= 1.5 * s.max() and b["smin"] >= s.min() / 1.5, name
        assert b["lip"] <= 5.0 * slope.max(), name
