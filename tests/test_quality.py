"""Mesh-quality post-processing (paper §3.7 measures) against closed forms, and the quality
the relaxation reaches on the unit square."""
import math

import numpy as np
import pytest

from paper_1906_07925_amd import quality as Q


def test_triangle_closed_forms():
    eq = np.array([[[0.0, 0.0], [1.0, 0.0], [0.5, math.sqrt(3.0) / 2.0]]])
    G, ang = Q.triangle_quality(eq)
    assert G[0] == pytest.approx(1.0, abs=1e-14) and np.allclose(ang, 60.0)
    right = np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]])
    G, ang = Q.triangle_quality(right)
    # S = 1/2, P = 1 + sqrt(2)/2, H = sqrt(2): G = sqrt(3) / (sqrt(2) + 1)
    assert G[0] == pytest.approx(math.sqrt(3.0) / (math.sqrt(2.0) + 1.0), rel=1e-14)
    assert sorted(ang[0]) == pytest.approx([45.0, 45.0, 90.0])


def test_tetra_closed_forms():
    reg = np.array([[[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]]], dtype=np.float64)
    g, dih = Q.tetra_quality(reg)
    assert g[0] == pytest.approx(1.0, rel=1e-13)
    assert np.allclose(dih, math.degrees(math.acos(1.0 / 3.0)))
    corner = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]], dtype=np.float64)
    g, dih = Q.tetra_quality(corner)
    # r_in = 1 / (3 + sqrt 3), r_circ = sqrt(3) / 2: gamma = 2 / (sqrt 3 + 1)
    assert g[0] == pytest.approx(2.0 / (math.sqrt(3.0) + 1.0), rel=1e-13)
    assert sorted(dih[0]) == pytest.approx([math.degrees(math.acos(1 / math.sqrt(3)))] * 3 + [90.0] * 3)


def test_hexagonal_patch_is_perfect():
    pts = [(i + 0.5 * (j % 2), j * math.sqrt(3.0) / 2.0) for i in range(12) for j in range(12)]
    # interior elements (the convex hull of the ragged rows adds thin triangles at the sides)
    keep = lambda c: (c[:, 0] > 1.0) & (c[:, 0] < 10.0) & (c[:, 1] > 1.0) & (c[:, 1] < 8.5)
    q = Q.mesh_quality(np.array(pts), colour=np.zeros(len(pts), np.int32), keep=keep)
    assert q["G_avg"] == pytest.approx(1.0, abs=1e-12) and q["frac_55_65"] == pytest.approx(1.0)
    assert q["comm_volume"] == 0.0 and q["n_below_30"] == 0


@pytest.mark.slow
def test_relaxation_improves_the_unit_square_mesh():
    """The oracle's relaxation of the jittered 64 x 64 lattice moves the triangulation towards
    the isotropic (hexagonal) optimum the method targets (§4.1): mean quality and the share of
    angles near 60 degrees rise."""
    from oracle import oracle as O
    from paper_1906_07925_amd import workloads as W
    cfg = W.config("square_4k")
    x, col, typ = W.make_state(cfg)
    op = O.OracleParams(cfg["spec"])
    inside = lambda c: np.all((c > 0.0) & (c < 1.0), axis=1)
    q0 = Q.mesh_quality(x, col, inside)
    xs, t = x.copy(), typ.copy()
    for k in range(400):
        xs, t, _ = O.step(op, xs, col, t, k, want=())
    q1 = Q.mesh_quality(xs, col, inside)
    print(q0, q1)
    assert q1["G_avg"] > q0["G_avg"] + 0.02
    assert q1["frac_55_65"] > q0["frac_55_65"] + 0.1
