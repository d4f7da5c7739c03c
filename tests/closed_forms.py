"""Closed forms of one relaxation step for configurations small enough to work out by hand.

Each case below places two or three particles so that the step's sums have one term per
particle, derives every quantity of the step from the paper's equations for that arrangement,
and compares with the oracle's step.  The expected values are written out from the derivation
in each docstring, not taken from the oracle:

  * the pressure and surface-tension acceleration of Eq. 18 and 23-24 with P = p0 / rho_t^2
    (Eq. 19, gamma = 2);
  * the absolute first time step of Eq. 29 with the cut-off radius r_c = kappa h;
  * the mid-point velocity of Eq. 26 after the velocity reset;
  * the viscosity of Eq. 21-22 and the viscous acceleration of Eq. 20 with its harmonic mean of
    the two dynamic viscosities;
  * the second time step (all three criteria of Eq. 29), the velocity of Eq. 27 and the drift of
    Eq. 28;
  * the treatment of a particle that crossed the boundary: the projection and re-tagging of
    Eq. 32 or, for seeded features, its mirror image;
  * the force projection of a feature particle on a level set (Eq. 30-31).

With equal smoothing lengths the pair sits at r = h (q = 1), where the Wendland C2 kernel takes
the rational values W(0, h) = alpha / h^d, W(h, h) = 3 alpha / (16 h^d) and
dW/dr(h, h) = -5 alpha / (8 h^(d+1)), alpha_2 = 7 / (4 pi), alpha_3 = 21 / (16 pi).  With unequal
lengths the kernel enters through the oracle's kernel routine, which the kernel tests pin on
their own (unit integral, derivative equal to a finite difference, support).

Every check function returns a list of (label, got, expected, tolerance) -- the tolerance is
relative to the expected value, or absolute where that value is zero -- so that the pin tests can
assert them and the mutation test can show that a planted slip in the oracle fails at least one
of them.
"""
from __future__ import annotations

import math

import numpy as np

TAU, KAPPA, P0, SIGMA0 = 1.3, 2.0, 1.0, 3.0
NU_C, C_ACC, C_VEL, C_VISC = 0.1, 0.25, 1.0 / 40.0, 0.125
ALPHA = {2: 7.0 / (4.0 * math.pi), 3: 21.0 / (16.0 * math.pi)}
TOL = 1e-12


def _axis(dim, k=0):
    e = np.zeros(dim)
    e[k] = 1.0
    return e


def _step(O, spec, x, col, typ, s0):
    op = O.OracleParams(dict(spec, n=x.shape[0]), s0=s0)
    return O.step(op, np.asarray(x, np.float64), np.asarray(col, np.int32), np.asarray(typ, np.int32), 0)


def equal_pair(dim: int, beta: float, s0: float = 0.05):
    """Hand derivation for two normal particles at distance r = h in a uniform field.

    rho_t = s0^-d, h = tau s0, P = p0 s0^(2d) for both particles.
      rho        = W(0) + W(h)                    = 19 alpha / (16 h^d)
      |a|        = (1 + beta) (P + P) |dW/dr|      = (1 + beta) (5/4) alpha p0 s0^(2d) / h^(d+1)
                   directed away from the other particle (repulsive)
      dt1        = c_acc sqrt(kappa h / |a|)
      |v~|       = |a| dt1 / 2
      nu, eta    = nu_c kappa h |v~|,  rho_t nu   (equal for both)
      harmonic mean 2 eta eta / (eta + eta) = eta
      v~_1 - v~_2 = 2 |v~| e_12, so
      |a~|       = eta (2 s0^(2d)) (5 alpha / (8 h^(d+1))) (2 |v~|) / h,  opposing v~
      dt2        = min(c_acc sqrt(kappa h/|a|), c_vel kappa h/|v~|, c_visc (kappa h)^2/nu)
      |v|        = |v~| - |a~| dt2 / 2,  |dr| = |v| dt2 along v~.
    Returns a dict of these magnitudes."""
    al = ALPHA[dim]
    h = TAU * s0
    P = P0 * s0 ** (2 * dim)
    rho_t = s0 ** -dim
    rho = 19.0 * al / (16.0 * h ** dim)
    dw = 5.0 * al / (8.0 * h ** (dim + 1))            # |dW/dr| at q = 1
    amag = (1.0 + beta) * 2.0 * P * dw
    rc = KAPPA * h
    dt1 = C_ACC * math.sqrt(rc / amag)
    vt = 0.5 * amag * dt1
    nu = NU_C * rc * vt
    eta = rho_t * nu
    atmag = eta * (2.0 * s0 ** (2 * dim)) * dw * (2.0 * vt) / h
    dt2 = min(C_ACC * math.sqrt(rc / amag), C_VEL * rc / vt, C_VISC * rc * rc / nu)
    v = vt - 0.5 * atmag * dt2
    return dict(h=h, rho=rho, rho_t=rho_t, a=amag, dt1=dt1, vt=vt, at=atmag, dt2=dt2, v=v, dr=v * dt2,
                kinetic=v * v)


def check_equal_pair(O, dim: int, different_colours: bool):
    """Two particles at r = h on the x axis in the middle of the unit box."""
    beta = SIGMA0 if different_colours else 0.0
    s0 = 0.05
    cf = equal_pair(dim, beta, s0)
    h = cf["h"]
    centre = np.full(dim, 0.5)
    e = _axis(dim)
    x = np.stack([centre - 0.5 * h * e, centre + 0.5 * h * e])
    spec = dict(dim=dim, geometry="box", lo=(0.0,) * dim, hi=(1.0,) * dim, field="uniform", sigma0=SIGMA0)
    col = [0, 1] if different_colours else [0, 0]
    x1, t1, r = _step(O, spec, x, col, [0, 0], s0)
    e12 = -e                                           # (x_1 - x_2) / r
    out = [("rho_1", r["rho"][0], cf["rho"], TOL), ("rho_2", r["rho"][1], cf["rho"], TOL),
           ("rho_t", r["rho_t"][0], cf["rho_t"], TOL), ("dt1", r["dt1"], cf["dt1"], TOL),
           ("dt2", r["dt2"], cf["dt2"], TOL), ("kinetic", r["kinetic"], cf["kinetic"], 1e-11)]
    for c in range(dim):
        out += [(f"a_1[{c}]", r["a"][0, c], cf["a"] * e12[c], TOL), (f"a_2[{c}]", r["a"][1, c], -cf["a"] * e12[c], TOL),
                (f"vt_1[{c}]", r["vt"][0, c], cf["vt"] * e12[c], TOL),
                (f"at_1[{c}]", r["at"][0, c], -cf["at"] * e12[c], 1e-11),
                (f"at_2[{c}]", r["at"][1, c], cf["at"] * e12[c], 1e-11),
                (f"v_1[{c}]", r["v"][0, c], cf["v"] * e12[c], 1e-11),
                (f"x_1[{c}]", x1[0, c], x[0, c] + cf["dr"] * e12[c], TOL),
                (f"x_2[{c}]", x1[1, c], x[1, c] - cf["dr"] * e12[c], TOL)]
    out += [("pairs", r["pairs"], 2, 0), ("interface_pairs", r["interface_pairs"], 1 if different_colours else 0, 0),
            ("nearest", r["nn"][0], h, TOL)]
    return out


def check_unequal_pair(O, dim: int):
    """Two particles of different smoothing lengths in a radially graded field.

    s = s0 (1 + fa |x - c|) with s0 = 0.02, fa = 4, c on the x axis; particle 1 at distance
    0.25 from c (s_1 = 0.04), particle 2 a further r = 0.07 out (s_2 = 0.0456).  Then
    h_i = tau s_i, rho_t,i = s_i^-d, P_i = s_i^(2d), h_12 = (h_1 + h_2) / 2 and, with
    W' = dW/dr(r, h_12), e_12 = (x_1 - x_2) / r:
      rho_i  = W(0, h_i) + W(r, h_i)                        (own smoothing length, Eq. 17)
      a_1    = -(1 + beta) (P_1 + P_2) W' e_12 = -a_2
      dt1    = c_acc min_i sqrt(kappa h_i / |a|)            (the finer particle binds)
      v~_i   = a_i dt1 / 2,  eta_i = s_i^-d nu_c kappa h_i |v~|
      a~_1   = [2 eta_1 eta_2 / (eta_1 + eta_2)] (s_1^(2d) + s_2^(2d)) W' (v~_1 - v~_2) / r = -a~_2
      dt2    = min over i of the three criteria of Eq. 29
      v_i    = v~_i + a~_i dt2 / 2,  x_i += v_i dt2."""
    s0, fa, R1, r = 0.02, 4.0, 0.25, 0.07
    c = np.full(dim, 0.5)
    c[0] = 0.1
    e = _axis(dim)
    x = np.stack([c + R1 * e, c + (R1 + r) * e])
    s = np.array([s0 * (1.0 + fa * R1), s0 * (1.0 + fa * (R1 + r))])
    h = TAU * s
    h12 = 0.5 * (h[0] + h[1])
    beta = SIGMA0
    wp = O.kernel_dw(r, h12, dim)
    P = s ** (2 * dim)
    e12 = -e
    a1 = -(1.0 + beta) * (P[0] + P[1]) * wp * e12
    amag = np.linalg.norm(a1)
    rc = KAPPA * h
    dt1 = C_ACC * min(math.sqrt(rc[0] / amag), math.sqrt(rc[1] / amag))
    vt1 = 0.5 * a1 * dt1
    vtm = np.linalg.norm(vt1)
    nu = NU_C * rc * vtm
    eta = s ** -dim * nu
    H = 2.0 * eta[0] * eta[1] / (eta[0] + eta[1])
    at1 = H * (s[0] ** (2 * dim) + s[1] ** (2 * dim)) * wp * (2.0 * vt1) / r
    dt2 = min(min(C_ACC * math.sqrt(rc[i] / amag), C_VEL * rc[i] / vtm, C_VISC * rc[i] ** 2 / nu[i]) for i in (0, 1))
    v1 = vt1 + 0.5 * at1 * dt2
    rho = [O.kernel_w(0.0, h[i], dim) + O.kernel_w(r, h[i], dim) for i in (0, 1)]
    spec = dict(dim=dim, geometry="box", lo=(0.0,) * dim, hi=(1.0,) * dim, field="radial_linear",
                fcentre=tuple(c), fa=fa, fb=0.0, sigma0=SIGMA0)
    x1, _, res = _step(O, spec, x, [0, 1], [0, 0], s0)
    out = [("h_1", res["h"][0], h[0], TOL), ("h_2", res["h"][1], h[1], TOL),
           ("rho_1", res["rho"][0], rho[0], TOL), ("rho_2", res["rho"][1], rho[1], TOL),
           ("dt1", res["dt1"], dt1, TOL), ("dt2", res["dt2"], dt2, TOL)]
    for k in range(dim):
        out += [(f"a_1[{k}]", res["a"][0, k], a1[k], TOL), (f"a_2[{k}]", res["a"][1, k], -a1[k], TOL),
                (f"at_1[{k}]", res["at"][0, k], at1[k], 1e-11), (f"at_2[{k}]", res["at"][1, k], -at1[k], 1e-11),
                (f"x_1[{k}]", x1[0, k], x[0, k] + v1[k] * dt2, TOL),
                (f"x_2[{k}]", x1[1, k], x[1, k] - v1[k] * dt2, TOL)]
    return out


def check_wall_crossing(O, dim: int, seeded: bool):
    """A particle pushed a distance 3D/4 past the wall x = 0 of the unit box.

    Particle A sits D/4 inside the wall with particle B at r = h further in; the pair is the
    equal pair above (same colour), so A moves by D = |dr| towards the wall and lands at
    x = -3D/4.  Seeded features (no particle changes type): A is mirrored to x = +3D/4 and
    stays normal.  Otherwise (Eq. 32, re-tagging): A is moved to the closest wall point x = 0
    and becomes a surface particle (one face)."""
    cf = equal_pair(dim, 0.0)
    h, D = cf["h"], cf["dr"]
    e = _axis(dim)
    base = np.full(dim, 0.5)
    base[0] = 0.25 * D
    x = np.stack([base, base + h * e])
    spec = dict(dim=dim, geometry="box", lo=(0.0,) * dim, hi=(1.0,) * dim, field="uniform", seeded=seeded)
    x1, t1, _ = _step(O, spec, x, [0, 0], [0, 0], 0.05)
    if seeded:
        return [("x_A", x1[0, 0], 0.75 * D, 1e-10), ("type_A", t1[0], 0, 0), ("x_B", x1[1, 0], base[0] + h + D, TOL)]
    return [("x_A", x1[0, 0], 0.0, 0), ("type_A", t1[0], 1, 0), ("x_B", x1[1, 0], base[0] + h + D, TOL)]


def check_circle_crossing(O, dim: int, seeded: bool, inner: bool = False):
    """A particle pushed a distance 3D/4 across a circle / sphere of radius R.

    Outer boundary (ball of radius R = 0.4): A at radius R - D/4 with B at r = h further in
    along the same ray; A moves out by D to radius R + 3D/4.  Inner boundary (annulus,
    r_in = 0.2, 2D): A at r_in + D/4 with B further out; A moves in to r_in - 3D/4.  Seeded: A
    is mirrored through the circle, radius 2R - |x - c| (R - 3D/4, resp. r_in + 3D/4), and
    stays normal.  Otherwise (Eq. 32): A is projected radially onto the circle and becomes a
    surface particle."""
    cf = equal_pair(dim, 0.0)
    h, D = cf["h"], cf["dr"]
    e = _axis(dim)
    if inner:
        c = np.zeros(dim)
        Rb = 0.2
        ra, rb = Rb + 0.25 * D, Rb + 0.25 * D + h
        spec = dict(dim=2, geometry="annulus", lo=(-1.0, -1.0), hi=(1.0, 1.0), centre=(0.0, 0.0), r_in=0.2,
                    r_out=1.0, field="uniform", seeded=seeded)
        want = Rb + 0.75 * D if seeded else Rb
    else:
        c = np.full(dim, 0.5)
        Rb = 0.4
        ra, rb = Rb - 0.25 * D, Rb - 0.25 * D - h
        spec = dict(dim=dim, geometry="ball", lo=(0.0,) * dim, hi=(1.0,) * dim, centre=tuple(c), r_out=Rb,
                    field="uniform", seeded=seeded)
        want = Rb - 0.75 * D if seeded else Rb
    x = np.stack([c + ra * e, c + rb * e])
    x1, t1, _ = _step(O, spec, x, [0, 0], [0, 0], 0.05)
    rad = np.linalg.norm(x1[0] - c)
    off_axis = float(np.linalg.norm(x1[0, 1:] - c[1:]))
    return [("radius_A", rad, want, 1e-10), ("type_A", t1[0], 0 if seeded else 1, 0), ("off_axis_A", off_axis, 0.0, 0)]


def _plane_spec(dim, nrm, p, seeded=False):
    """Level-set region phi(x) = n . (x - p) > 0 on a 5^d background mesh over the unit box; a
    linear function is reproduced exactly by the multilinear interpolation, and its gradient is
    n everywhere."""
    ax = np.linspace(0.0, 1.0, 5)
    grids = np.meshgrid(*([ax] * dim), indexing="ij")
    pts = np.stack([g.transpose(*reversed(range(dim))).reshape(-1) for g in grids], axis=1)
    phi = (pts - p) @ nrm
    return dict(dim=dim, geometry="levelset", lo=(0.0,) * dim, hi=(1.0,) * dim, field="uniform",
                grid_n=(5,) * dim + (1,) * (3 - dim), grid_phi=phi, grid_s=np.ones(pts.shape[0]), seeded=seeded)


def _plane_frame(dim):
    if dim == 2:
        n = np.array([0.6, 0.8])
        t = np.array([0.8, -0.6])
    else:
        n = np.array([0.48, 0.6, 0.64])
        t = np.array([0.6, -0.48, 0.0]) / math.sqrt(0.6 ** 2 + 0.48 ** 2)
    return n, t


def check_levelset_force_projection(O, dim: int):
    """A surface particle S on a planar level set with a fixed particle F at r = h inside the
    region, in the direction u = (n + t)/sqrt(2) (n the unit normal, t a unit tangent).

    The force on S (Eq. 18, same colour, equal P) is -(P + P) dW/dr e_SF with e_SF = -u, i.e.
    |a| = 2 P |W'| along -u; the force mapping of Eq. 31 removes its normal component and leaves
    a = -(2 P |W'| / sqrt(2)) t.  F is fixed (no force, no velocity), so S alone sets
    dt1 = c_acc sqrt(kappa h / |a|); F's viscosity is zero, the harmonic mean vanishes and
    a~ = 0.  Hence v = v~ = a dt1 / 2, the drift v dt2 is tangential, dt2 = min of the three
    criteria of Eq. 29, and S stays on the plane."""
    cf = equal_pair(dim, 0.0)
    h = cf["h"]
    n, t = _plane_frame(dim)
    u = (n + t) / math.sqrt(2.0)
    p = np.full(dim, 0.5)
    x = np.stack([p, p + h * u])
    x1, t1, r = _step(O, _plane_spec(dim, n, p), x, [0, 0], [1, 3], 0.05)
    amag = cf["a"] / math.sqrt(2.0)                     # cf["a"] = 2 P |W'| (beta = 0)
    rc = KAPPA * h
    dt1 = C_ACC * math.sqrt(rc / amag)
    vt = 0.5 * amag * dt1
    dt2 = min(C_ACC * math.sqrt(rc / amag), C_VEL * rc / vt, C_VISC * rc * rc / (NU_C * rc * vt))
    out = [("dt1", r["dt1"], dt1, TOL), ("dt2", r["dt2"], dt2, TOL), ("type_S", t1[0], 1, 0),
           ("a.n/|a|", float(r["a"][0] @ n) / amag, 0.0, 1e-14), ("at_S", float(np.linalg.norm(r["at"][0])), 0.0, 0),
           ("phi_S/h", float((x1[0] - p) @ n) / h, 0.0, 1e-12)]
    for k in range(dim):
        out += [(f"a_S[{k}]", r["a"][0, k], -amag * t[k], TOL), (f"x_S[{k}]", x1[0, k], p[k] - vt * dt2 * t[k], TOL),
                (f"x_F[{k}]", x1[1, k], x[1, k], 0)]
    return out


def check_levelset_crossing(O, dim: int, seeded: bool):
    """A normal particle pushed a distance 3D/4 through a planar level set (phi = 0 plane with
    unit normal n): A at phi = D/4 with B at r = h further in along n, so A ends at
    phi = -3D/4.  Seeded: mirror image x - 2 phi n (phi = +3D/4), type kept.  Otherwise (Eq. 32):
    x - phi n onto the plane, re-tagged as a surface particle."""
    cf = equal_pair(dim, 0.0)
    h, D = cf["h"], cf["dr"]
    n, _ = _plane_frame(dim)
    p = np.full(dim, 0.5)
    x = np.stack([p + 0.25 * D * n, p + (0.25 * D + h) * n])
    x1, t1, _ = _step(O, _plane_spec(dim, n, p, seeded=seeded), x, [0, 0], [0, 0], 0.05)
    phi = float((x1[0] - p) @ n)
    tang = float(np.linalg.norm((x1[0] - p) - phi * n))
    phi_check = ("phi_A", phi, 0.75 * D, 1e-9) if seeded else ("phi_A/h", phi / h, 0.0, 1e-12)
    return [phi_check, ("type_A", t1[0], 0 if seeded else 1, 0), ("tangential_A/h", tang / h, 0.0, 1e-12)]


def failures(checks):
    """The checks that fail: |got - want| > tol |want|, or |got| > tol where want = 0."""
    bad = []
    for label, got, want, tol in checks:
        err = abs(float(got) - float(want))
        lim = tol * abs(float(want)) if want != 0 else tol
        if not err <= lim:
            bad.append((label, float(got), float(want)))
    return bad


def all_checks(O):
    """Every closed-form case, as (case name, checks)."""
    cases = []
    for dim in (2, 3):
        for diff in (False, True):
            cases.append((f"equal_pair_{dim}d_{'two' if diff else 'one'}_colour", check_equal_pair(O, dim, diff)))
        cases.append((f"unequal_pair_{dim}d", check_unequal_pair(O, dim)))
        for seeded in (False, True):
            tag = "seeded" if seeded else "retag"
            cases.append((f"wall_{dim}d_{tag}", check_wall_crossing(O, dim, seeded)))
            cases.append((f"ball_{dim}d_{tag}", check_circle_crossing(O, dim, seeded)))
            cases.append((f"levelset_crossing_{dim}d_{tag}", check_levelset_crossing(O, dim, seeded)))
        cases.append((f"levelset_force_{dim}d", check_levelset_force_projection(O, dim)))
    for seeded in (False, True):
        cases.append((f"annulus_inner_{'seeded' if seeded else 'retag'}", check_circle_crossing(O, 2, seeded, inner=True)))
    return cases
