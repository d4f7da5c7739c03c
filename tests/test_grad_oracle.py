"""Pins of the gradient oracle (oracle/grad.py), which restates the step in float64 PyTorch
and differentiates it with autograd:

  * its forward trajectory equals the C oracle's (an independent implementation pinned by
    test_oracle_pins) over several steps, time steps included;
  * its loss equals the loss formed from the C oracle's density summation and pair list;
  * its gradients with respect to the RBF coefficients and to initial positions equal central
    finite differences of the loss taken through the C oracle (FP64).
"""
import numpy as np
import pytest

from oracle import grad as G
from oracle import oracle as O
from paper_1906_07925_amd import workloads as W

STEPS = 4
LAM = 1.0


def _case(n_side=8, seed=3, scale_c=0.1):
    n = n_side ** 3
    spec = W.rbf_cube(n)
    cfg = dict(spec=spec, seed=W.BASE_SEED + 4, init="lattice", per_axis=n_side, n_colours=6)
    x, col, typ = W.make_state(cfg)
    x = x.astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    coeff = rng.normal(0.0, scale_c, size=spec["n_rbf"])
    return spec, spec["s0"], x, col, typ, coeff


def c_oracle_loss(spec, s0, x0, col, typ, coeff, steps, lam):
    """Loss of the module docstring of oracle/grad.py formed from the C oracle: trajectory by
    orc_step, density summation (Eq. 17) of the final state, interface term over orc_pairs."""
    op = O.OracleParams(dict(spec, rbf_coeff=np.asarray(coeff)), s0=s0)
    x, t = x0.copy(), typ.copy()
    dts = []
    for k in range(steps):
        x, t, r = O.step(op, x, col, t, k, want=())
        dts.append((r["dt1"], r["dt2"]))
    _, _, r = O.step(op, x, col, t, steps, want=("rho", "rho_t", "h"))
    e = r["rho"] / r["rho_t"] - 1.0
    pi, pj = O.pairs(op, x)
    rr = np.linalg.norm(x[pi] - x[pj], axis=1)
    hij = 0.5 * (r["h"][pi] + r["h"][pj])
    q = rr / hij
    w = np.where(q < 2.0, (1.0 - 0.5 * q) ** 4 * (1.0 + 2.0 * q), 0.0)
    ifc = 0.5 * np.sum(w[col[pi] != col[pj]])
    n = x.shape[0]
    return float((e * e).sum() / n + lam * ifc / n), x, t, dts


def test_forward_matches_c_oracle():
    spec, s0, x, col, typ, coeff = _case()
    pr = G.Problem(spec, s0, col, typ)
    L, _, _, xg, tg, info = G.run(pr, x, coeff, STEPS, LAM)
    Lc, xc, tc, dts = c_oracle_loss(spec, s0, x, col, typ, coeff, STEPS, LAM)
    assert np.max(np.abs(xg - xc)) < 1e-12
    assert np.array_equal(tg, tc)
    for r, (d1, d2) in zip(info, dts):
        assert abs(r["dt1"] - d1) <= 1e-12 * d1 and abs(r["dt2"] - d2) <= 1e-12 * d2
    assert abs(L - Lc) <= 1e-12 * abs(Lc)


def test_coefficient_gradient_matches_finite_differences():
    spec, s0, x, col, typ, coeff = _case()
    pr = G.Problem(spec, s0, col, typ)
    L, gc, _, _, _, _ = G.run(pr, x, coeff, STEPS, LAM)
    eps = 1e-5
    rng = np.random.Generator(np.random.PCG64(5))
    for k in rng.choice(len(coeff), size=6, replace=False):
        cp, cm = coeff.copy(), coeff.copy()
        cp[k] += eps
        cm[k] -= eps
        fd = (c_oracle_loss(spec, s0, x, col, typ, cp, STEPS, LAM)[0] -
              c_oracle_loss(spec, s0, x, col, typ, cm, STEPS, LAM)[0]) / (2 * eps)
        assert abs(gc[k] - fd) <= 1e-4 * np.max(np.abs(gc)) + 1e-6 * abs(fd), (k, gc[k], fd)
    # a random direction
    dirn = rng.normal(size=len(coeff))
    fd = (c_oracle_loss(spec, s0, x, col, typ, coeff + eps * dirn, STEPS, LAM)[0] -
          c_oracle_loss(spec, s0, x, col, typ, coeff - eps * dirn, STEPS, LAM)[0]) / (2 * eps)
    assert abs(gc @ dirn - fd) <= 1e-4 * abs(fd)


def test_position_gradient_matches_finite_differences():
    spec, s0, x, col, typ, coeff = _case(n_side=6)
    pr = G.Problem(spec, s0, col, typ)
    _, _, gx, _, _, _ = G.run(pr, x, coeff, STEPS, LAM, want_x0_grad=True)
    eps = 1e-7
    rng = np.random.Generator(np.random.PCG64(9))
    interior = np.nonzero(np.all((x > 0.05) & (x < 0.95), axis=1))[0]
    for i in rng.choice(interior, size=4, replace=False):
        a = int(rng.integers(0, 3))
        xp, xm = x.copy(), x.copy()
        xp[i, a] += eps
        xm[i, a] -= eps
        fd = (c_oracle_loss(spec, s0, xp, col, typ, coeff, STEPS, LAM)[0] -
              c_oracle_loss(spec, s0, xm, col, typ, coeff, STEPS, LAM)[0]) / (2 * eps)
        assert abs(gx[i, a] - fd) <= 1e-4 * np.max(np.abs(gx)) + 1e-6 * abs(fd), (i, a, gx[i, a], fd)
