"""Seeded synthetic workloads for the relaxation step.

This module only describes domains and draws initial particle sets: positions,
colours (sub-domain labels) and types.  It holds none of the method's arithmetic
(no kernel, field evaluation, force or integrator); both the GPU library and the
CPU oracle receive its arrays as inputs.

The shapes follow the paper's workloads (§4: graded circle, square, cube; colours
from Voronoi generators with equal mass per sub-domain, Eq. 8), scaled to the
configurations below.  No public dataset is involved: the paper's bunny and gear
geometries are not used.

Spec dictionaries carry the domain (``geometry``, ``lo``/``hi``, ``centre``,
``r_in``/``r_out``), the size field (``field`` with ``fcentre``/``fa``/``fb`` or RBF
centres/coefficients/width) and the particle count ``n``.  The field scale ``s0`` is
left to each side to normalise (integral of rho_t over the region equals ``n``)
unless a spec fixes it.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 190607925

NORMAL, SURFACE, CURVE, FIXED = 0, 1, 2, 3


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------------------
# Domains
# ---------------------------------------------------------------------------------------

def unit_square(n: int, **kw) -> dict:
    s = dict(dim=2, geometry="box", lo=(0.0, 0.0), hi=(1.0, 1.0), field="uniform", n=n)
    s.update(kw)
    return s


def unit_cube(n: int, **kw) -> dict:
    s = dict(dim=3, geometry="box", lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), field="uniform", n=n)
    s.update(kw)
    return s


def annulus(n: int, r_in: float = 0.2, r_out: float = 1.0, ratio: float = 4.0, **kw) -> dict:
    """Annulus centred at the origin; spacing grows linearly from r_in to r_out by ``ratio``."""
    s = dict(dim=2, geometry="annulus", lo=(-r_out, -r_out), hi=(r_out, r_out), centre=(0.0, 0.0),
             r_in=r_in, r_out=r_out, field="radial_linear", fcentre=(0.0, 0.0),
             fa=(ratio - 1.0) / (r_out - r_in), fb=r_in, n=n)
    s.update(kw)
    return s


def ball(n: int, dim: int = 3, radius: float = 0.5, **kw) -> dict:
    c = (0.5,) * dim
    s = dict(dim=dim, geometry="ball", lo=(0.0,) * dim, hi=(1.0,) * dim, centre=c, r_out=radius,
             field="uniform", n=n)
    s.update(kw)
    return s


def cube_with_inclusion(n: int, radius: float = 0.25, ratio: float = 4.0, **kw) -> dict:
    """Unit cube; spacing s = s0 (1 + (ratio-1) d / dmax), d = distance to the sphere."""
    dmax = math.sqrt(3.0) / 2.0 - radius
    s = dict(dim=3, geometry="box", lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), field="sphere_distance",
             fcentre=(0.5, 0.5, 0.5), fa=(ratio - 1.0) / dmax, fb=radius, n=n)
    s.update(kw)
    return s


def rbf_cube(n: int, n_rbf: int = 32, width: float = 0.15, seed: int = BASE_SEED + 4,
             coeff: np.ndarray | None = None, **kw) -> dict:
    """Unit cube with s = s0 exp(sum_k c_k G_k(x)); centres uniform in the cube (seeded).
    s0 is fixed by the particle count at c = 0 and is not renormalised as c varies."""
    rng = _rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_rbf, 3))
    if coeff is None:
        coeff = np.zeros(n_rbf)
    s = dict(dim=3, geometry="box", lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), field="rbf_exp",
             n_rbf=n_rbf, rbf_centre=centres, rbf_coeff=np.asarray(coeff, dtype=np.float64),
             rbf_width=width, s0=(1.0 / n) ** (1.0 / 3.0), n=n)
    s.update(kw)
    return s


# ---------------------------------------------------------------------------------------
# Initial particle sets
# ---------------------------------------------------------------------------------------

def levelset_ball(n: int, dim: int = 3, radius: float = 0.4, nodes: int = 48, ratio: float = 3.0, **kw) -> dict:
    """A ball given only through a background mesh: the level set R - |x - c| and the relative
    spacing 1 + (ratio - 1) |x - c| / R (graded from the centre out) sampled at nodes^dim
    nodes over the unit box; both are interpolated from the mesh.  The analytic ball is kept
    as ``shape`` to draw initial positions."""
    c = np.full(dim, 0.5)
    ax = np.linspace(0.0, 1.0, nodes)
    grids = np.meshgrid(*([ax] * dim), indexing="ij")
    # node (i, j, k) at index i + n (j + n k): x index fastest
    pts = np.stack([g.transpose(*reversed(range(dim))).reshape(-1) for g in grids], axis=1)
    r = np.linalg.norm(pts - c, axis=1)
    s = dict(dim=dim, geometry="levelset", lo=(0.0,) * dim, hi=(1.0,) * dim, field="grid",
             grid_n=(nodes,) * dim + (1,) * (3 - dim), grid_phi=radius - r,
             grid_s=1.0 + (ratio - 1.0) * np.minimum(r / radius, 1.5), shape=("ball", tuple(c), radius), n=n)
    s.update(kw)
    return s


def _inside(spec: dict, x: np.ndarray) -> np.ndarray:
    g = spec["geometry"]
    if g == "levelset":
        _, c, rad = spec["shape"]
        return np.linalg.norm(x - np.asarray(c), axis=1) < rad
    if g in ("box", "periodic"):
        lo = np.asarray(spec["lo"]); hi = np.asarray(spec["hi"])
        return np.all((x >= lo) & (x <= hi), axis=1)
    r = np.linalg.norm(x - np.asarray(spec["centre"]), axis=1)
    if g == "annulus":
        return (r >= spec["r_in"]) & (r <= spec["r_out"])
    return r <= spec["r_out"]


def _uniform_points(spec: dict, m: int, rng: np.random.Generator) -> np.ndarray:
    """m points uniform (by volume) inside the region, by rejection from the bounding box."""
    lo = np.asarray(spec["lo"], dtype=np.float64); hi = np.asarray(spec["hi"], dtype=np.float64)
    out = []
    have = 0
    while have < m:
        batch = rng.uniform(lo, hi, size=(max(2 * (m - have), 1024), spec["dim"]))
        batch = batch[_inside(spec, batch)]
        out.append(batch)
        have += batch.shape[0]
    return np.concatenate(out)[:m]


def nearest_seed(x: np.ndarray, seeds: np.ndarray, chunk: int = 1 << 16) -> np.ndarray:
    """Index of the nearest seed (FP64 distance; ties go to the lowest index)."""
    out = np.empty(x.shape[0], dtype=np.int32)
    s2 = np.sum(seeds * seeds, axis=1)
    for b in range(0, x.shape[0], chunk):
        xb = x[b:b + chunk]
        d2 = np.sum(xb * xb, axis=1)[:, None] - 2.0 * xb @ seeds.T + s2[None, :]
        out[b:b + chunk] = np.argmin(d2, axis=1)
    return out


def jittered_lattice(spec: dict, per_axis: int, rng: np.random.Generator,
                     jitter: float = 0.25) -> np.ndarray:
    """Cell-centred lattice (i + 1/2) dx over the bounding box plus U(-jitter, jitter) dx."""
    d = spec["dim"]
    lo = np.asarray(spec["lo"], dtype=np.float64); hi = np.asarray(spec["hi"], dtype=np.float64)
    dx = (hi - lo) / per_axis
    axes = [lo[a] + (np.arange(per_axis) + 0.5) * dx[a] for a in range(d)]
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, d)
    grid = grid + rng.uniform(-jitter, jitter, size=grid.shape) * dx
    return grid


def equal_mass_voronoi(spec: dict, n: int, n_colours: int, rng: np.random.Generator):
    """Random initial set: Voronoi generators uniform in the region, then particles sampled
    uniformly and accepted into the generator's cell until each colour holds its equal
    share of the particles (equal-mass partitioning, Eq. 8 with unit particle mass)."""
    seeds = _uniform_points(spec, n_colours, rng)
    quota = np.full(n_colours, n // n_colours, dtype=np.int64)
    quota[: n % n_colours] += 1
    xs, cs = [], []
    filled = np.zeros(n_colours, dtype=np.int64)
    while filled.sum() < n:
        pts = _uniform_points(spec, max(4 * int(quota.sum() - filled.sum()), 4096), rng)
        col = nearest_seed(pts, seeds)
        for c in range(n_colours):
            need = quota[c] - filled[c]
            if need <= 0:
                continue
            sel = np.nonzero(col == c)[0][:need]
            xs.append(pts[sel]); cs.append(np.full(sel.size, c, dtype=np.int32))
            filled[c] += sel.size
    x = np.concatenate(xs); c = np.concatenate(cs)
    perm = rng.permutation(n)
    return x[perm], c[perm]


def initial_state(spec: dict, seed: int, init: str, n_colours: int, per_axis: int | None = None,
                  remove_to: int | None = None, jitter: float = 0.25):
    """Returns (x float64 (n, d), colour int32 (n,), type int32 (n,))."""
    rng = _rng(seed)
    if init == "lattice":
        x = jittered_lattice(spec, per_axis, rng, jitter)
        if remove_to is not None and remove_to < x.shape[0]:
            keep = np.sort(rng.choice(x.shape[0], size=remove_to, replace=False))
            x = x[keep]
        seeds = _uniform_points(spec, n_colours, rng)
        col = nearest_seed(x, seeds)
    elif init == "random":
        x, col = equal_mass_voronoi(spec, spec["n"], n_colours, rng)
    else:
        raise ValueError(init)
    typ = np.zeros(x.shape[0], dtype=np.int32)
    return x, col.astype(np.int32), typ


def _spread(m: int, rng: np.random.Generator, jitter: float) -> np.ndarray:
    """m parameters in (0, 1), evenly spread between the ends (which other features occupy):
    (i + 1 + U(-jitter, jitter)) / (m + 1), in random order."""
    t = (np.arange(m) + 1.0 + rng.uniform(-jitter, jitter, size=m)) / (m + 1.0)
    return rng.permutation(t)


def _spread_2d(m: int, ea: float, eb: float, rng: np.random.Generator, jitter: float) -> np.ndarray:
    """m points in the open rectangle (0, ea) x (0, eb): a jittered p x q lattice of spacing
    about sqrt(ea eb / m) between the sides, with p q - m sites dropped at random."""
    p = max(1, int(round(math.sqrt(m * ea / eb))))
    q = max(1, int(math.ceil(m / p)))
    while p * q < m:
        p += 1
    i, j = np.meshgrid(np.arange(p), np.arange(q), indexing="ij")
    u = (i.reshape(-1) + 1.0 + rng.uniform(-jitter, jitter, size=p * q)) / (p + 1.0)
    v = (j.reshape(-1) + 1.0 + rng.uniform(-jitter, jitter, size=p * q)) / (q + 1.0)
    keep = rng.choice(p * q, size=m, replace=False)
    return np.stack([u[keep] * ea, v[keep] * eb], axis=1)


def _round_points(m: int, dim: int, rng: np.random.Generator, jitter: float) -> np.ndarray:
    """m near-evenly spread unit vectors: equal angles on the circle, the Fibonacci (golden
    angle) spiral on the sphere; jittered and randomly rotated."""
    if dim == 2:
        th = (np.arange(m) + 0.5 + rng.uniform(-jitter, jitter, size=m)) * (2.0 * math.pi / m)
        th = th + rng.uniform(0.0, 2.0 * math.pi)
        return rng.permutation(np.stack([np.cos(th), np.sin(th)], axis=1))
    k = np.arange(m) + 0.5
    z = 1.0 - 2.0 * k / m
    ph = k * math.pi * (3.0 - math.sqrt(5.0)) + rng.uniform(-jitter, jitter, size=m) * (2.0 * math.pi / math.sqrt(m))
    r = np.sqrt(np.maximum(1.0 - z * z, 0.0))
    v = np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)
    # random rotation (QR of a Gaussian matrix, sign-fixed)
    qm, rm = np.linalg.qr(rng.normal(size=(3, 3)))
    qm = qm * np.sign(np.diag(rm))
    return rng.permutation(v @ qm.T)


def feature_points(spec: dict, k: int, m: int, rng: np.random.Generator, jitter: float = 0.1) -> np.ndarray:
    """m points spread evenly over boundary feature k of the region (jittered 1D / 2D lattices,
    equal angles, the Fibonacci sphere), features numbered as the library's particle budget
    numbers them (box: faces or sides 2a + h, then in 3D edges 4a + hb + 2hc, then corners;
    ball: its sphere; annulus: inner, then outer circle).  Even spreading keeps the initial
    gaps near the target spacing: on a 1D or 2D feature the kernel's repulsion weakens for
    pairs closer than half a smoothing length, so uniformly random points would stay bunched."""
    d = spec["dim"]
    g = spec["geometry"]
    if g in ("ball", "annulus"):
        c = np.asarray(spec["centre"], dtype=np.float64)
        r = spec["r_in"] if (g == "annulus" and k == 0) else spec["r_out"]
        return c + r * _round_points(m, d, rng, jitter)
    lo = np.asarray(spec["lo"], dtype=np.float64)
    hi = np.asarray(spec["hi"], dtype=np.float64)
    n_faces = 2 * d
    n_edges = 12 if d == 3 else 0
    x = np.tile(lo, (m, 1))
    if k < n_faces:
        a, h = divmod(k, 2)
        x[:, a] = hi[a] if h else lo[a]
        others = [b for b in range(d) if b != a]
        if d == 2:
            b = others[0]
            x[:, b] = lo[b] + _spread(m, rng, jitter) * (hi[b] - lo[b])
        else:
            b, c = others
            uv = _spread_2d(m, hi[b] - lo[b], hi[c] - lo[c], rng, jitter)
            x[:, b] = lo[b] + uv[:, 0]
            x[:, c] = lo[c] + uv[:, 1]
        return x
    if k < n_faces + n_edges:
        a, bits = divmod(k - n_faces, 4)
        b, c = (1, 2) if a == 0 else ((0, 2) if a == 1 else (0, 1))
        x[:, a] = lo[a] + _spread(m, rng, jitter) * (hi[a] - lo[a])
        x[:, b] = hi[b] if bits & 1 else lo[b]
        x[:, c] = hi[c] if bits & 2 else lo[c]
        return x
    bits = k - n_faces - n_edges
    return np.tile(np.where([(bits >> a) & 1 for a in range(d)], hi, lo), (m, 1))


def feature_seeded(spec: dict, budget: dict, seed: int, n_colours: int):
    """Initial set with the boundary features seeded explicitly (§3.5): budget['count'][k]
    particles of type budget['type'][k] uniform on feature k, and budget['n_volume'] normal
    particles uniform in the interior; colours from the nearest of n_colours seeds.  The
    budget comes from either side's particle-budget routine.  Returns (x, colour, type)."""
    rng = _rng(seed)
    xs, ts = [], []
    for k, (cnt, typ) in enumerate(zip(budget["count"], budget["type"])):
        if cnt > 0:
            xs.append(feature_points(spec, k, int(cnt), rng))
            ts.append(np.full(int(cnt), int(typ), dtype=np.int32))
    nv = int(budget["n_volume"])
    xs.append(_uniform_points(spec, nv, rng))
    ts.append(np.zeros(nv, dtype=np.int32))
    x = np.concatenate(xs)
    typ = np.concatenate(ts)
    perm = rng.permutation(x.shape[0])
    x, typ = x[perm], typ[perm]
    seeds = _uniform_points(spec, n_colours, rng)
    return x, nearest_seed(x, seeds).astype(np.int32), typ


# ---------------------------------------------------------------------------------------
# The five configurations
# ---------------------------------------------------------------------------------------

def config(name: str, scale: float = 1.0) -> dict:
    """Workload description.  ``scale`` < 1 shrinks the particle count for tests while
    keeping the domain, field and colour structure."""
    if name == "square_4k":      # 2D unit square, 64x64 jittered lattice, 4 colours, 200 steps
        per = max(4, int(round(64 * math.sqrt(scale))))
        n = per * per
        return dict(spec=unit_square(n), seed=BASE_SEED + 0, init="lattice", per_axis=per,
                    n_colours=4, steps=200)
    if name == "annulus_262k":   # 2D annulus 0.2..1, 1:4 linear grading, 16 colours, random
        n = max(64, int(round(262144 * scale)))
        return dict(spec=annulus(n), seed=BASE_SEED + 1, init="random", n_colours=16, steps=2000)
    if name == "cube_inclusion_2m":  # 3D cube, sphere-distance grading 1:4, 128^3 lattice, 64 colours
        per = max(4, int(round(128 * scale ** (1.0 / 3.0))))
        n = per ** 3
        return dict(spec=cube_with_inclusion(n), seed=BASE_SEED + 2, init="lattice", per_axis=per,
                    n_colours=64, steps=1000)
    if name == "rbf_cube_1m":    # 3D cube, 2^20 particles from a 102^3 lattice, 32-RBF field
        per = max(4, int(round(102 * scale ** (1.0 / 3.0))))
        n = min(per ** 3, max(8, int(round((1 << 20) * scale))))
        return dict(spec=rbf_cube(n), seed=BASE_SEED + 4, init="lattice", per_axis=per,
                    remove_to=n, n_colours=16, steps=50)
    raise KeyError(name)


def batched_domains(scale: float = 1.0, seed: int = BASE_SEED + 3, n_dom: int = 64):
    """64 independent domains: squares, annuli, cubes, balls (16 each at full size), particle
    counts log-uniform in [1e4, 5e5] times ``scale``, 4..32 colours, random equal-mass init."""
    rng = _rng(seed)
    kinds = ["square", "annulus", "cube", "ball"]
    out = []
    for k in range(n_dom):
        kind = kinds[(k * len(kinds)) // n_dom]
        n = int(round(math.exp(rng.uniform(math.log(1e4), math.log(5e5))) * scale))
        n = max(n, 64)
        nc = int(rng.integers(4, 33))
        if kind == "square":
            spec = unit_square(n)
        elif kind == "annulus":
            spec = annulus(n)
        elif kind == "cube":
            spec = unit_cube(n)
        else:
            spec = ball(n)
        out.append(dict(spec=spec, seed=int(rng.integers(0, 2**31)), init="random", n_colours=nc,
                        kind=kind))
    return out


def make_state(cfg: dict):
    return initial_state(cfg["spec"], cfg["seed"], cfg["init"], cfg["n_colours"],
                         per_axis=cfg.get("per_axis"), remove_to=cfg.get("remove_to"))
