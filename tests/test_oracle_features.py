"""Pins of the oracle's particle budget with explicitly seeded boundary features (§2.3, Eq. 4-6
with unit particle mass, Eq. 15; §3.5 particle types).

Reading under test: a feature surface carries s^-(dim-1) particles per unit area, a feature
curve s^-1 per unit length, a box corner one particle, and u = 1/s0 solves
n = I_v u^dim + sum_features I_f u^power.  The pins come from closed forms and from
independent quadrature, never from the oracle itself:

  * uniform box [0,a]x[0,b]x[0,c]: the budget factorises, n = (a u + 2)(b u + 2)(c u + 2)
    (and (a u + 2)(b u + 2) in 2D), so every count is known exactly;
  * uniform ball / disk: the sphere area 4 pi R^2 and the circle length 2 pi R;
  * radial field on the annulus: s is constant on each circle, so the integral is 2 pi r / s(r);
  * the graded cube of the benchmark: a face and an edge integral against scipy's adaptive
    quadrature of the field definition, and the six faces (twelve edges) equal by symmetry.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O
from paper_1906_07925_amd import workloads as W


def budget(spec, n, **kw):
    return O.feature_budget(O.OracleParams(spec, s0=1.0), n, **kw)


def test_box_3d_budget_factorises():
    a, b, c, u = 1.0, 2.0, 0.5, 10.0
    n = int(round((a * u + 2) * (b * u + 2) * (c * u + 2)))
    assert n == 1848
    spec = W.unit_cube(n, hi=(a, b, c))
    bd = budget(spec, n)
    assert bd["s0"] == pytest.approx(1.0 / u, rel=1e-10)
    faces = bd["count"][:6].tolist()
    assert faces == [int(u * u * b * c)] * 2 + [int(u * u * a * c)] * 2 + [int(u * u * a * b)] * 2
    edges = bd["count"][6:18].tolist()
    assert edges == [int(u * a)] * 4 + [int(u * b)] * 4 + [int(u * c)] * 4
    assert bd["count"][18:].tolist() == [1] * 8
    assert bd["type"].tolist() == [1] * 6 + [2] * 12 + [3] * 8
    assert bd["n_volume"] == int(u ** 3 * a * b * c)
    assert bd["n_volume"] + int(bd["count"].sum()) == n


def test_box_2d_budget_factorises():
    a, b, u = 2.0, 1.0, 20.0
    n = int(round((a * u + 2) * (b * u + 2)))
    spec = W.unit_square(n, hi=(a, b))
    bd = budget(spec, n)
    assert bd["s0"] == pytest.approx(1.0 / u, rel=1e-10)
    assert bd["count"].tolist() == [int(u * b)] * 2 + [int(u * a)] * 2 + [1] * 4
    assert bd["type"].tolist() == [1] * 4 + [3] * 4
    assert bd["n_volume"] == int(u * u * a * b)


@pytest.mark.parametrize("dim", [2, 3])
def test_ball_boundary_measure(dim):
    R, n = 0.5, 5000
    spec = W.ball(n, dim=dim, radius=R)
    I, typ, pw = O.features(O.OracleParams(spec, s0=1.0), 256)
    meas = 4.0 * math.pi * R * R if dim == 3 else 2.0 * math.pi * R
    assert I.tolist() == pytest.approx([meas], rel=1e-12)
    assert typ.tolist() == [1] and pw.tolist() == [dim - 1]
    # the root of the closed-form budget, to the accuracy of the volume quadrature
    vol = (4.0 / 3.0) * math.pi * R ** 3 if dim == 3 else math.pi * R * R
    u = 1.0 / budget(spec, n)["s0"]
    assert vol * u ** dim + meas * u ** (dim - 1) == pytest.approx(n, rel=1e-5)


def test_annulus_radial_field_circles():
    spec = W.annulus(20000)
    op = O.OracleParams(spec, s0=1.0)
    I, typ, pw = O.features(op, 512)

    def s(r):
        return 1.0 + spec["fa"] * (r - spec["fb"])

    exact = [2 * math.pi * spec["r_in"] / s(spec["r_in"]), 2 * math.pi * spec["r_out"] / s(spec["r_out"])]
    assert I.tolist() == pytest.approx(exact, rel=1e-12)
    assert typ.tolist() == [1, 1] and pw.tolist() == [1, 1]


def test_graded_cube_faces_and_edges():
    spec = W.cube_with_inclusion(1 << 16)
    c, fa, R = np.asarray(spec["fcentre"]), spec["fa"], spec["fb"]

    def s(x):
        return 1.0 + fa * abs(np.linalg.norm(np.asarray(x) - c) - R)

    I, typ, pw = O.features(O.OracleParams(spec, s0=1.0), 1024)
    face0, _ = integrate.dblquad(lambda z, y: s((0.0, y, z)) ** -2, 0.0, 1.0, 0.0, 1.0, epsabs=1e-12, epsrel=1e-12)
    edge0, _ = integrate.quad(lambda t: 1.0 / s((t, 0.0, 0.0)), 0.0, 1.0, epsabs=1e-13, epsrel=1e-13)
    assert I[0] == pytest.approx(face0, rel=1e-6)
    assert I[6] == pytest.approx(edge0, rel=1e-8)
    assert np.ptp(I[:6]) <= 1e-12 * I[0]
    assert np.ptp(I[6:18]) <= 1e-12 * I[6]
    assert pw.tolist() == [2] * 6 + [1] * 12 + [0] * 8


def test_budget_sums_to_n():
    spec = W.cube_with_inclusion(1 << 20)
    bd = budget(spec, 1 << 20, nq=256, nq_volume=160)
    assert bd["mass_volume"] + bd["mass"].sum() == pytest.approx(1 << 20, rel=1e-12)
    assert bd["n_volume"] + int(bd["count"].sum()) == 1 << 20
    # with part of the count on the boundary the same n spreads coarser than the volume-only
    # normalisation
    assert bd["s0"] > O.normalised_s0(O.OracleParams(spec, s0=1.0), 1 << 20, 160)


def test_periodic_has_no_features():
    spec = W.unit_cube(1000, geometry="periodic")
    bd = budget(spec, 1000)
    assert bd["count"].size == 0 and bd["n_volume"] == 1000
    assert bd["s0"] == pytest.approx(0.1, rel=1e-6)


def test_feature_seeded_generator_places_counts():
    spec = W.unit_cube(1728)
    bd = budget(spec, 1728)
    x, col, typ = W.feature_seeded(spec, bd, seed=7, n_colours=4)
    assert x.shape == (1728, 3)
    assert np.bincount(typ, minlength=4).tolist() == [1000, 600, 120, 8]
    on = ((x == 0.0) | (x == 1.0)).sum(axis=1)
    assert np.array_equal(on, typ)          # faces: 1 wall, edges: 2, corners: 3
    assert set(col.tolist()) <= set(range(4))
