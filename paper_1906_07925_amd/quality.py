"""Mesh quality of a relaxed particle set (post-processing on the host, §3.6-3.7).

The relaxation never builds connectivity; elements exist only to measure the result.  The
particles are triangulated (2D) or tetrahedralised (3D) with a Delaunay tessellation (Qhull via
scipy), elements outside the meshing region are dropped by an optional predicate on their
centroids, and the paper's quality measures are evaluated:

  2D: G = 2 sqrt(3) S / (P H) (S area, P half-perimeter, H longest edge; 1 for the equilateral
      triangle) and the angles: G_avg, G_min, theta_max, theta_min, the mean per-triangle minimum
      angle theta_min#, the number of triangles with an angle below 30 degrees, and the
      fraction of angles within 55-65 degrees;
  3D: the dihedral angles and the radius ratio gamma = 3 r_in / r_circ (1 for the regular
      tetrahedron): gamma_avg, gamma_min, theta_max, theta_min, theta_min#, and the slivers
      counted by smallest dihedral angle below 10, 20, 30 and 40 degrees;
  both: the communication volume N_eg / N_et of §4 (elements with vertices of different
      colours over all elements).
"""
from __future__ import annotations

import numpy as np


def _tessellate(x: np.ndarray):
    from scipy.spatial import Delaunay
    return Delaunay(x).simplices


def triangle_quality(p: np.ndarray):
    """p: (m, 3, 2) triangle vertices.  Returns (G (m,), angles in degrees (m, 3))."""
    a = np.linalg.norm(p[:, 1] - p[:, 2], axis=1)
    b = np.linalg.norm(p[:, 0] - p[:, 2], axis=1)
    c = np.linalg.norm(p[:, 0] - p[:, 1], axis=1)
    e1, e2 = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]
    S = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    P = 0.5 * (a + b + c)
    H = np.maximum(np.maximum(a, b), c)
    G = 2.0 * np.sqrt(3.0) * S / (P * H)
    # law of cosines, angle opposite each side
    def ang(x, y, z):
        return np.degrees(np.arccos(np.clip((y * y + z * z - x * x) / (2.0 * y * z), -1.0, 1.0)))
    angles = np.stack([ang(a, b, c), ang(b, a, c), ang(c, a, b)], axis=1)
    return G, angles


def tetra_quality(p: np.ndarray):
    """p: (m, 4, 3) tetrahedron vertices.  Returns (gamma (m,), dihedral angles in degrees (m, 6))."""
    v0, v1, v2, v3 = p[:, 0], p[:, 1], p[:, 2], p[:, 3]
    vol = np.abs(np.einsum("ij,ij->i", v1 - v0, np.cross(v2 - v0, v3 - v0))) / 6.0
    faces = [(v1, v2, v3), (v0, v2, v3), (v0, v1, v3), (v0, v1, v2)]
    areas = [0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1) for a, b, c in faces]
    r_in = 3.0 * vol / np.sum(areas, axis=0)
    # circumradius: |a|^2 (b x c) + |b|^2 (c x a) + |c|^2 (a x b) over 12 V, edges from v0
    a, b, c = v1 - v0, v2 - v0, v3 - v0
    num = (np.sum(a * a, 1)[:, None] * np.cross(b, c) + np.sum(b * b, 1)[:, None] * np.cross(c, a)
           + np.sum(c * c, 1)[:, None] * np.cross(a, b))
    r_circ = np.linalg.norm(num, axis=1) / (12.0 * vol)
    gamma = 3.0 * r_in / r_circ
    # dihedral angle along edge (i, j): between the two faces that contain it
    verts = [v0, v1, v2, v3]
    dih = []
    for i, j in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)):
        k, l = [m for m in range(4) if m not in (i, j)]
        e = verts[j] - verts[i]
        e = e / np.linalg.norm(e, axis=1)[:, None]
        # components of the two opposite vertices perpendicular to the edge
        u = verts[k] - verts[i]
        w = verts[l] - verts[i]
        u = u - np.sum(u * e, 1)[:, None] * e
        w = w - np.sum(w * e, 1)[:, None] * e
        cosd = np.sum(u * w, 1) / (np.linalg.norm(u, axis=1) * np.linalg.norm(w, axis=1))
        dih.append(np.degrees(np.arccos(np.clip(cosd, -1.0, 1.0))))
    return gamma, np.stack(dih, axis=1)


def mesh_quality(x: np.ndarray, colour: np.ndarray | None = None, keep=None) -> dict:
    """Quality measures of the Delaunay elements of the point set x (n, d).  keep(centroids)
    -> bool mask selects the elements inside the meshing region (all by default)."""
    x = np.asarray(x, dtype=np.float64)
    d = x.shape[1]
    simp = _tessellate(x)
    if keep is not None:
        simp = simp[keep(x[simp].mean(axis=1))]
    out = {"n_points": int(x.shape[0]), "n_elements": int(simp.shape[0])}
    if colour is not None and simp.shape[0]:
        col = np.asarray(colour)[simp]
        out["comm_volume"] = float(np.mean(np.any(col != col[:, :1], axis=1)))
    p = x[simp]
    if d == 2:
        G, ang = triangle_quality(p)
        out.update(G_avg=float(G.mean()), G_min=float(G.min()), theta_max=float(ang.max()),
                   theta_min=float(ang.min()), theta_min_avg=float(ang.min(axis=1).mean()),
                   n_below_30=int(np.sum(ang.min(axis=1) < 30.0)),
                   frac_55_65=float(np.mean((ang >= 55.0) & (ang <= 65.0))))
    else:
        gam, dih = tetra_quality(p)
        mins = dih.min(axis=1)
        out.update(gamma_avg=float(gam.mean()), gamma_min=float(gam.min()), theta_max=float(dih.max()),
                   theta_min=float(dih.min()), theta_min_avg=float(mins.mean()),
                   slivers={str(t): int(np.sum(mins < t)) for t in (10, 20, 30, 40)})
    return out
