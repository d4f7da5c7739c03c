"""Explicitly seeded boundary features (§2.3 Eq. 5-6, §3.5) on the HIP path against the oracle.

* The library's particle budget (mpsph_feature_budget, Gauss-Legendre panels) equals the
  oracle's (midpoint rule, bisection): s0 and the per-feature masses to 1e-5, counts exactly.
* Single steps from feature-seeded states match the oracle at the single-step tolerances,
  including normal particles that cross a wall and are mirrored back (the seeded-feature
  reading: no type ever changes).
* Long runs keep every particle on its feature, relax the 1D chains of a square's sides and a
  cube's edges to even gaps, and agree with the oracle's run on the density residual.
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
    M.lib()  # raises when the library is missing: no fallback
    return torch


def oracle_budget(spec, n):
    return O.feature_budget(O.OracleParams(spec, s0=1.0), n)


BUDGET_CASES = [
    (W.unit_cube(50000), 50000),
    (W.unit_square(4096), 4096),
    (W.cube_with_inclusion(1 << 21), 1 << 21),
    (W.ball(100000), 100000),
    (W.ball(20000, dim=2), 20000),
    (W.annulus(262144), 262144),
]


@pytest.mark.parametrize("case", range(len(BUDGET_CASES)))
def test_budget_matches_oracle(torch_cuda, case):
    from paper_1906_07925_amd import mpsph as M
    spec, n = BUDGET_CASES[case]
    g = M.feature_budget(spec, n)
    o = oracle_budget(spec, n)
    assert g["s0"] == pytest.approx(o["s0"], rel=1e-5)
    assert g["mass_volume"] == pytest.approx(o["mass_volume"], rel=1e-5)
    assert np.array_equal(g["type"], o["type"])
    assert np.allclose(g["mass"], o["mass"], rtol=1e-5, atol=0)
    assert np.array_equal(g["count"], o["count"])
    assert g["n_volume"] == o["n_volume"]


def test_budget_rejects_level_set(torch_cuda):
    from paper_1906_07925_amd import mpsph as M
    with pytest.raises(M.MpsphError) as e:
        M.feature_budget(W.levelset_ball(10000), 10000)
    assert e.value.code == 6


def seeded_state(spec, n, seed, n_colours, near_wall=0):
    """Feature-seeded float32 state; near_wall normal particles are moved to 1e-6 inside a wall
    so that the step pushes some of them across it."""
    bd = oracle_budget(spec, n)
    spec = dict(spec, n=n, seeded=True)
    x, col, typ = W.feature_seeded(spec, bd, seed, n_colours)
    if near_wall:
        idx = np.nonzero(typ == 0)[0][:near_wall]
        rng = np.random.Generator(np.random.PCG64(seed + 1))
        if spec["geometry"] == "box":
            lo, hi = np.asarray(spec["lo"]), np.asarray(spec["hi"])
            for i in idx:
                a = int(rng.integers(0, spec["dim"]))
                x[i, a] = lo[a] + 1e-6 if rng.uniform() < 0.5 else hi[a] - 1e-6
        else:
            c = np.asarray(spec["centre"])
            for i in idx:
                u = (x[i] - c) / np.linalg.norm(x[i] - c)
                inner = spec["geometry"] == "annulus" and rng.uniform() < 0.5
                x[i] = c + u * (spec["r_in"] * (1 + 1e-6) if inner else spec["r_out"] * (1 - 1e-6))
    return spec, bd["s0"], x.astype(np.float32), col, typ


SEEDED_CASES = [
    (W.unit_square(4096), 4096, 4, 200),
    (W.cube_with_inclusion(30000), 30000, 8, 400),
    (W.unit_cube(20000), 20000, 4, 400),
    (W.ball(20000), 20000, 4, 400),
    (W.annulus(20000), 20000, 8, 400),
]


@pytest.mark.parametrize("case", range(len(SEEDED_CASES)))
def test_single_step_parity_seeded(torch_cuda, case):
    spec, n, nc, near = SEEDED_CASES[case]
    spec, s0, x32, col, typ = seeded_state(spec, n, W.BASE_SEED + 50 + case, nc, near_wall=near)
    rep = {}
    PU.check_single_step(spec, s0, x32, col, typ, report=rep)
    r = rep["oracle"]
    if near:
        # some displacements cross the boundary: the mirror rule was exercised by this step
        x1 = x32.astype(np.float64) + r["dr"]
        if spec["geometry"] == "box":
            out = np.any((x1 < np.asarray(spec["lo"])) | (x1 > np.asarray(spec["hi"])), axis=1)
        else:
            rr = np.linalg.norm(x1 - np.asarray(spec["centre"]), axis=1)
            out = (rr > spec["r_out"]) | (rr < spec.get("r_in", -1.0))
        assert np.sum(out & (typ == 0)) > 0
    print(spec["geometry"], spec["field"], {k: f"{v:.2e}" for k, v in rep["errs"].items()})


def _on_walls(x, spec):
    lo, hi = np.asarray(spec["lo"]), np.asarray(spec["hi"])
    return ((x == lo) | (x == hi)).sum(axis=1)


def _chain_gaps(x, typ, spec, axis_free, fixed):
    """Sorted gaps along the chain of feature particles lying on the walls given by
    fixed = {axis: value}, normalised by their mean."""
    sel = typ >= 1
    for a, v in fixed.items():
        sel &= x[:, a] == v
    t = np.sort(x[sel, axis_free])
    g = np.diff(t)
    return g / g.mean()


def _gpu_long(spec, s0, x32, col, typ, steps):
    m, g = PU.gpu_run(spec, s0, x32, col, typ, steps=steps, debug=False, fields=())
    return m, g["x1"], g["t1"]


def _oracle_long(spec, s0, x32, col, typ, steps):
    op = O.OracleParams(spec, s0=s0)
    x = x32.astype(np.float64)
    t = typ.copy()
    r = None
    for k in range(steps):
        x, t, r = O.step(op, x, col, t, k, want=())
    return r, x, t


def test_long_run_seeded_square(torch_cuda):
    """Unit square with (u + 2)^2 = 4096 particles, u = 62: 62 per side, 4 corners, 62^2
    inside; one colour (no surface-tension jumps along the sides); 300 steps."""
    spec, s0, x32, col, typ = seeded_state(W.unit_square(4096), 4096, W.BASE_SEED + 60, 1)
    assert np.bincount(typ, minlength=4).tolist() == [3844, 248, 0, 4]
    steps = 300
    m, xg, tg = _gpu_long(spec, s0, x32, col, typ, steps)
    r, xo, to = _oracle_long(spec, s0, x32, col, typ, steps)
    for x, t in ((xg, tg), (xo, to)):
        assert np.array_equal(t, typ)                         # no type ever changes
        assert np.all(_on_walls(x[typ == 1], spec) == 1) and np.all(_on_walls(x[typ == 3], spec) == 2)
        assert np.array_equal(x[typ == 3], x32[typ == 3].astype(np.float64))  # corners never move
        assert np.all((x >= 0.0) & (x <= 1.0))
        for a in range(2):
            for v in (0.0, 1.0):
                gaps = _chain_gaps(x, t, spec, 1 - a, {a: v})
                assert gaps.size == 63
                inner = gaps[2:-2]
                assert inner.max() / inner.min() < 1.05, (a, v, inner.min(), inner.max())
    assert m["nonfinite"] == 0
    assert m["residual_l2"] == pytest.approx(r["residual_l2"], rel=0.05)


def test_long_run_seeded_cube(torch_cuda):
    """Unit cube, uniform field, one colour: (u + 2)^3 = 13824 particles, u = 22: 22^2 per face,
    22 per edge, 8 corners, 22^3 inside; 200 steps."""
    n = 24 ** 3
    spec, s0, x32, col, typ = seeded_state(W.unit_cube(n), n, W.BASE_SEED + 61, 1)
    assert np.bincount(typ, minlength=4).tolist() == [22 ** 3, 6 * 22 ** 2, 12 * 22, 8]
    steps = 200
    m, xg, tg = _gpu_long(spec, s0, x32, col, typ, steps)
    r, xo, to = _oracle_long(spec, s0, x32, col, typ, steps)
    for x, t in ((xg, tg), (xo, to)):
        assert np.array_equal(t, typ)
        w = _on_walls(x, spec)
        assert np.all(w[typ == 1] == 1) and np.all(w[typ == 2] == 2) and np.all(w[typ == 3] == 3)
        # (a normal particle mirrored from within an FP32 ulp of a wall may round onto it)
        assert np.all((x >= 0.0) & (x <= 1.0))
        # the twelve edges: 22 particles between two corners, evenly spread
        for a in range(3):
            b, c = [q for q in range(3) if q != a]
            for vb in (0.0, 1.0):
                for vc in (0.0, 1.0):
                    gaps = _chain_gaps(x, t, spec, a, {b: vb, c: vc})
                    assert gaps.size == 23
                    inner = gaps[2:-2]
                    assert inner.max() / inner.min() < 1.1, (a, vb, vc, inner.min(), inner.max())
    assert m["nonfinite"] == 0
    assert m["residual_l2"] == pytest.approx(r["residual_l2"], rel=0.05)


@pytest.mark.parametrize("kind", ["ball", "annulus"])
def test_long_run_seeded_round(torch_cuda, kind):
    """Ball and annulus: surface particles stay on their sphere / circles, normal particles
    inside, no type changes, residual close to the oracle's run."""
    spec0 = W.ball(20000) if kind == "ball" else W.annulus(20000)
    spec, s0, x32, col, typ = seeded_state(spec0, 20000, W.BASE_SEED + 62, 4)
    steps = 100
    m, xg, tg = _gpu_long(spec, s0, x32, col, typ, steps)
    r, xo, to = _oracle_long(spec, s0, x32, col, typ, steps)
    c = np.asarray(spec["centre"])
    for x, t, eps in ((xg, tg, 2e-6), (xo, to, 1e-12)):
        assert np.array_equal(t, typ)
        rr = np.linalg.norm(x - c, axis=1)
        rs = rr[typ == 1]
        on = np.abs(rs - spec["r_out"]) <= eps * spec["r_out"]
        if kind == "annulus":
            on |= np.abs(rs - spec["r_in"]) <= eps * spec["r_out"]
        assert np.all(on)
        rn = rr[typ == 0]
        assert np.all(rn <= spec["r_out"] * (1 + eps))
        if kind == "annulus":
            assert np.all(rn >= spec["r_in"] * (1 - eps))
    assert m["nonfinite"] == 0
    assert m["residual_l2"] == pytest.approx(r["residual_l2"], rel=0.05)
