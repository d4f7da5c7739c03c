"""Pins of the oracle's background mesh (level set and target field interpolated from a
Cartesian mesh, §3.1-3.2, with the projection of Eq. 32):

  * multilinear interpolation reproduces multilinear functions and their gradients exactly;
  * a planar level set moves a particle that left the region exactly onto the plane and
    re-tags it as a surface particle;
  * the normalisation integral of a constant field over a sampled ball converges to the ball's
    volume, and a sampled field reproduces the analytic one at the nodes.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_1906_07925_amd import workloads as W


def _mesh_spec(dim, n, phi_fn, s_fn):
    ax = np.linspace(0.0, 1.0, n)
    grids = np.meshgrid(*([ax] * dim), indexing="ij")
    pts = np.stack([g.transpose(*reversed(range(dim))).reshape(-1) for g in grids], axis=1)
    return dict(dim=dim, geometry="levelset", lo=(0.0,) * dim, hi=(1.0,) * dim, field="grid",
                grid_n=(n,) * dim + (1,) * (3 - dim), grid_phi=phi_fn(pts), grid_s=s_fn(pts), n=100, s0=0.05)


def test_multilinear_functions_are_exact():
    rng = np.random.Generator(np.random.PCG64(1))
    for dim in (2, 3):
        c = rng.normal(size=8)

        def f(p):
            x, y = p[:, 0], p[:, 1]
            z = p[:, 2] if dim == 3 else np.zeros_like(x)
            return c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z + c[6] * x * z + c[7] * x * y * z

        def grad(p):
            x, y = p[:, 0], p[:, 1]
            z = p[:, 2] if dim == 3 else np.zeros_like(x)
            g = [c[1] + c[4] * y + c[6] * z + c[7] * y * z, c[2] + c[4] * x + c[5] * z + c[7] * x * z,
                 c[3] + c[5] * y + c[6] * x + c[7] * x * y]
            return np.stack(g[:dim], axis=1)

        spec = _mesh_spec(dim, 7, f, lambda p: np.ones(p.shape[0]))
        op = O.OracleParams(spec)
        x = rng.uniform(0.0, 1.0, size=(50, dim))
        v, g = O.grid_interp(op, "phi", x)
        assert np.allclose(v, f(x), rtol=0, atol=1e-12)
        assert np.allclose(g, grad(x), rtol=0, atol=1e-10)


def test_planar_level_set_projection_is_exact():
    # region x < 0.6 (phi = 0.6 - x, linear, so interpolation and the normal are exact)
    spec = _mesh_spec(2, 5, lambda p: 0.6 - p[:, 0], lambda p: np.ones(p.shape[0]))
    op = O.OracleParams(spec, s0=0.01)
    # two far-apart particles: no pair forces, the time steps vanish and the drift is zero; the
    # one outside the region is projected onto the plane and re-tagged
    x = np.array([[0.7, 0.3], [0.2, 0.8]])
    x1, t1, r = O.step(op, x, np.zeros(2, np.int32), np.zeros(2, np.int32), 0)
    assert r["dt1"] == 0.0
    assert x1[0, 0] == 0.6 and x1[0, 1] == 0.3 and t1[0] == O.SURFACE
    assert np.array_equal(x1[1], x[1]) and t1[1] == O.NORMAL


def test_sampled_ball_volume_and_field():
    R = 0.4
    exact = 4.0 / 3.0 * math.pi * R ** 3
    err = {}
    for n in (17, 33, 65):
        spec = _mesh_spec(3, n, lambda p: R - np.linalg.norm(p - 0.5, axis=1), lambda p: np.ones(p.shape[0]))
        op = O.OracleParams(spec, s0=1.0)
        err[n] = abs(O.field_integral(op, 160) / exact - 1.0)
    # the interpolated boundary converges at second order in the node spacing, down to the
    # ~1e-3 resolution of the 160^3 midpoint quadrature
    assert err[17] < 0.02 and err[33] < err[17] / 3.0 and err[65] < 1.5e-3, err
    sp = W.levelset_ball(1000)
    op = O.OracleParams(sp, s0=1.0)
    nodes = np.array([[0.5, 0.5, 0.5], [0.5 + 1.0 / 47.0 * 3, 0.5 + 1.0 / 47.0, 0.5]])
    # at mesh nodes the interpolated field equals the sampled analytic one
    nodes = np.round(nodes * 47.0) / 47.0
    v, _ = O.grid_interp(op, "s", nodes)
    want = 1.0 + 2.0 * np.minimum(np.linalg.norm(nodes - 0.5, axis=1) / 0.4, 1.5)
    assert np.allclose(v, want, rtol=1e-12)
