"""Gradient oracle for the relaxation step -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke entry point and the benchmark's CPU baseline may import this module.
It shares no code with the HIP library.

A plain float64 PyTorch (CPU) restatement of one relaxation step of Ji, Fu, Hu & Adams
(arXiv 1906.07925, Algorithm 1), differentiated by torch.autograd, for small particle counts
(candidate pairs by brute force).  It follows the same readings as the C oracle in
mpsph_oracle.c, step for step:

  target field and scale          s(x), rho_t = s^-d, h = tau s, P = p0 / rho_t^2   (Eq. 1-2, 16, 19)
  pressure + surface tension      a_i = -sum_j (1 + beta_ij)(P_i + P_j) W'(r_ij, h_ij) e_ij  (Eq. 18, 23-24)
  force mapping of features       zero the normal components on box faces          (Eq. 30-31)
  first time step                 dt1 = min_i c_acc sqrt(kappa h_i / |a_i|)          (Eq. 29, v = 0)
  mid-point velocity, viscosity   v~ = a dt1 / 2; eta = rho_t nu_coeff kappa h |v~|   (Eq. 21-22, 26)
  viscous acceleration            a~_i = sum_j [2 eta_i eta_j/(eta_i + eta_j)]
                                         (1/rho_t,i^2 + 1/rho_t,j^2) W'(r_ij,h_ij)/r_ij (v~_i - v~_j)  (Eq. 20)
  second time step                three-term minimum of Eq. 29
  velocity, drift, box walls      v = v~ + a~ dt2 / 2, x += v dt2, clamp and re-tag  (Eq. 27-28, 32)

The loss after the last step (a density error plus a smooth interface measure):

  L = (1/N) sum_i (rho_i / rho_t,i - 1)^2 + (lambda / N) sum_{i<j, C_i != C_j} W(r_ij, h_ij) / W(0, h_ij)

with the density summation of Eq. 17 (self term included).  Piecewise-constant parts (pair
sets, type masks, re-tagging, which particle attains a minimum) are fixed from the values of
the forward pass; the gradient flows through everything else, through the minimum of a time
step to the particle that attains it, and through the clamp where a coordinate stays inside.
Box geometry only.
"""
from __future__ import annotations

import math

import numpy as np
import torch

T = torch.float64


def alpha(d: int) -> float:
    """Wendland C2 normalisation with support 2h."""
    return 7.0 / (4.0 * math.pi) if d == 2 else 21.0 / (16.0 * math.pi)


class Problem:
    """Constants of a box-domain relaxation run.  ``spec`` is a workload description; ``s0``
    the fixed field scale."""

    def __init__(self, spec: dict, s0: float, colour, ptype):
        if spec["geometry"] != "box":
            raise ValueError("the gradient oracle handles box domains")
        self.d = int(spec["dim"])
        self.lo = torch.tensor(spec["lo"][:self.d], dtype=T)
        self.hi = torch.tensor(spec["hi"][:self.d], dtype=T)
        self.field = spec["field"]
        self.spec = spec
        self.s0 = float(s0)
        self.tau = spec.get("tau", 1.3)
        self.kappa = spec.get("kappa", 2.0)
        self.p0 = spec.get("p0", 1.0)
        self.sigma0 = spec.get("sigma0", 3.0)
        self.t0 = int(spec.get("t0", -1))
        self.t1 = int(spec.get("t1", -1))
        self.nu = spec.get("nu_coeff", 0.1)
        self.c_acc = spec.get("c_acc", 0.25)
        self.c_vel = spec.get("c_vel", 1.0 / 40.0)
        self.c_visc = spec.get("c_visc", 0.125)
        self.colour = torch.as_tensor(np.asarray(colour, dtype=np.int64))
        self.type0 = np.asarray(ptype, dtype=np.int64).copy()
        if self.field == "rbf_exp":
            self.mu = torch.tensor(np.asarray(spec["rbf_centre"], dtype=np.float64)[:, :self.d], dtype=T)
            self.width = float(spec["rbf_width"])

    def sigma(self, t: int) -> float:
        """Surface-tension ramp of Eq. 25 over steps (t0, t1]."""
        if self.t0 < 0 or t <= self.t0:
            return self.sigma0
        if t <= self.t1:
            return self.sigma0 * (1.0 - (t - self.t0) / (self.t1 - self.t0))
        return 0.0

    def spacing(self, x, coeff):
        """s(x) for the fields the gradient is taken for: uniform, or s0 exp(sum_k c_k G_k(x))."""
        if self.field == "uniform":
            return torch.full((x.shape[0],), self.s0, dtype=T)
        if self.field != "rbf_exp":
            raise ValueError("the gradient oracle handles the uniform and RBF fields")
        d2 = ((x[:, None, :] - self.mu[None, :, :]) ** 2).sum(-1)
        g = torch.exp(-d2 / (2.0 * self.width ** 2))
        return self.s0 * torch.exp(g @ coeff)


def _candidates(x: np.ndarray, reach: np.ndarray):
    """All ordered pairs i != j with |x_i - x_j| < max(reach_i, reach_j) (brute force)."""
    diff = x[:, None, :] - x[None, :, :]
    r = np.sqrt((diff ** 2).sum(-1))
    m = r < np.maximum(reach[:, None], reach[None, :]) * (1.0 + 1e-9)
    np.fill_diagonal(m, False)
    i, j = np.nonzero(m)
    return torch.as_tensor(i), torch.as_tensor(j)


def _norm(v):
    """|v| per row with a gradient that is zero (not NaN) at v = 0."""
    n2 = (v * v).sum(-1)
    pos = n2 > 0
    return torch.where(pos, torch.sqrt(torch.where(pos, n2, torch.ones_like(n2))), torch.zeros_like(n2))


def _project(pr: Problem, x, typ: np.ndarray, f):
    """Force mapping of feature particles in a box: drop the components along the normals of
    the faces the particle lies on; fixed particles carry no force."""
    xd = x.detach()
    on = (xd == pr.lo) | (xd == pr.hi)
    t = torch.as_tensor(typ)
    keep = ~((t[:, None] > 0) & on)
    keep &= (t[:, None] != 3)
    return f * keep.to(T)


def step(pr: Problem, x, typ: np.ndarray, t: int, coeff):
    """One relaxation step.  x: (n, d) float64 tensor (differentiable), typ: int array.
    Returns (new x, new types, dict of dt1, dt2)."""
    d, kap = pr.d, pr.kappa
    s = pr.spacing(x, coeff)
    h = pr.tau * s
    rho_t = s ** (-d)
    P = pr.p0 / rho_t ** 2
    i, j = _candidates(x.detach().numpy(), kap * h.detach().numpy())
    u = x[i] - x[j]
    r = _norm(u)
    hij = 0.5 * (h[i] + h[j])
    ti, tj = torch.as_tensor(typ)[i], torch.as_tensor(typ)[j]
    act = ((r.detach() < kap * hij.detach()) & (tj >= ti) & (r.detach() > 0)).to(T)
    rs = torch.where(r > 0, r, torch.ones_like(r))
    q = r / hij
    w = torch.clamp(1.0 - 0.5 * q, min=0.0)
    dW = alpha(d) * hij ** (-d - 1) * (-5.0 * q) * w ** 3            # dW/dr at h_ij
    beta = torch.where(pr.colour[i] != pr.colour[j], pr.sigma(t), 0.0).to(T)
    coef = -(1.0 + beta) * (P[i] + P[j]) * dW / rs * act
    a = torch.zeros_like(x).index_add(0, i, coef[:, None] * u)
    a = _project(pr, x, typ, a)
    movable = torch.as_tensor(typ != 3)
    am = _norm(a)
    big = torch.full_like(am, math.inf)
    c1 = torch.where(movable & (am > 0), pr.c_acc * torch.sqrt(kap * h / torch.where(am > 0, am, torch.ones_like(am))),
                     big)
    dt1 = c1.min() if bool(torch.isfinite(c1).any()) else torch.zeros((), dtype=T)
    vt = 0.5 * a * dt1 * movable.to(T)[:, None]
    vm = _norm(vt)
    eta = rho_t * pr.nu * kap * h * vm
    esum = eta[i] + eta[j]
    hm = torch.where(esum > 0, 2.0 * eta[i] * eta[j] / torch.where(esum > 0, esum, torch.ones_like(esum)),
                     torch.zeros_like(esum))
    inv2 = 1.0 / rho_t[i] ** 2 + 1.0 / rho_t[j] ** 2
    cv = hm * inv2 * dW / rs * act
    at = torch.zeros_like(x).index_add(0, i, cv[:, None] * (vt[i] - vt[j]))
    at = _project(pr, x, typ, at)
    rc = kap * h
    nu = pr.nu * rc * vm
    one = torch.ones_like(am)
    c2 = torch.stack([
        torch.where(movable & (am > 0), pr.c_acc * torch.sqrt(rc / torch.where(am > 0, am, one)), big),
        torch.where(movable & (vm > 0), pr.c_vel * rc / torch.where(vm > 0, vm, one), big),
        torch.where(movable & (nu > 0), pr.c_visc * rc * rc / torch.where(nu > 0, nu, one), big)])
    dt2 = c2.min() if bool(torch.isfinite(c2).any()) else torch.zeros((), dtype=T)
    v = (vt + 0.5 * at * dt2) * movable.to(T)[:, None]
    xn = x + v * dt2
    # box walls: clamp (the gradient passes where the coordinate stays inside, walls included)
    xn = torch.maximum(torch.minimum(xn, pr.hi), pr.lo)
    xd = xn.detach()
    nf = ((xd == pr.lo) | (xd == pr.hi)).sum(-1).numpy()
    ft = np.where(nf <= 0, 0, np.where(nf == 1, 1, np.where(nf == 2, 2 if d == 3 else 3, 3)))
    typ_new = np.where(typ == 3, 3, np.maximum(typ, ft))
    return xn, typ_new, {"dt1": float(dt1.detach()), "dt2": float(dt2.detach())}


def loss(pr: Problem, x, coeff, lam: float):
    """Density error plus smooth interface measure at positions x (see the module docstring)."""
    d, kap = pr.d, pr.kappa
    n = x.shape[0]
    s = pr.spacing(x, coeff)
    h = pr.tau * s
    i, j = _candidates(x.detach().numpy(), kap * h.detach().numpy())
    u = x[i] - x[j]
    r = _norm(u)
    qi = r / h[i]
    wi = torch.clamp(1.0 - 0.5 * qi, min=0.0)
    dens = wi ** 4 * (1.0 + 2.0 * qi)
    ssum = 1.0 + torch.zeros(n, dtype=T).index_add(0, i, dens)        # self term w(0) = 1
    e = alpha(d) * pr.tau ** (-d) * ssum - 1.0                          # rho / rho_t - 1
    hij = 0.5 * (h[i] + h[j])
    q = r / hij
    wq = torch.clamp(1.0 - 0.5 * q, min=0.0)
    diff = (pr.colour[i] != pr.colour[j]).to(T)
    ifc = (diff * wq ** 4 * (1.0 + 2.0 * q)).sum() * 0.5
    return (e * e).sum() / n + lam * ifc / n


def run(pr: Problem, x0: np.ndarray, coeff: np.ndarray, steps: int, lam: float, t_start: int = 0,
        want_x0_grad: bool = False):
    """Forward over ``steps`` steps and the loss; returns (loss, dL/dcoeff, dL/dx0 or None,
    final x, final types, list of per-step dicts)."""
    c = torch.tensor(np.asarray(coeff, dtype=np.float64), dtype=T, requires_grad=True)
    x = torch.tensor(np.asarray(x0, dtype=np.float64), dtype=T, requires_grad=want_x0_grad)
    xs = x
    typ = pr.type0.copy()
    info = []
    for k in range(steps):
        xs, typ, r = step(pr, xs, typ, t_start + k, c)
        info.append(r)
    L = loss(pr, xs, c, lam)
    L.backward()
    gx = x.grad.numpy().copy() if want_x0_grad else None
    gc = c.grad.numpy().copy() if c.grad is not None else np.zeros_like(np.asarray(coeff, dtype=np.float64))
    return float(L.detach()), gc, gx, xs.detach().numpy(), typ, info
