"""O(N^2) numpy micro-oracle for tiny inputs (N <= ~2000).

TEST INFRASTRUCTURE ONLY.  An independent, fully vectorised restatement of the
pair sums of one relaxation step (paper §3.3-3.4: Eq. 17, 18, 20-24, 26, 29) over
*all* particle pairs, with no neighbour search at all.  It pins the C oracle's cell
grid, candidate culling and per-particle assembly.  Feature particles and the drift
are not modelled here (all particles are treated as normal), so it is used on
all-normal inputs.
"""
from __future__ import annotations

import math

import numpy as np


def wendland(q: np.ndarray, dim: int):
    """Wendland C2 on support q < 2: returns (w(q), dw/dq(q)) without the h^-d factors."""
    alpha = 7.0 / (4.0 * math.pi) if dim == 2 else 21.0 / (16.0 * math.pi)
    u = np.clip(1.0 - 0.5 * q, 0.0, None)
    w = alpha * u**4 * (1.0 + 2.0 * q)
    dw = alpha * (-5.0 * q) * u**3
    inside = q < 2.0
    return np.where(inside, w, 0.0), np.where(inside, dw, 0.0)


def step_sums(x: np.ndarray, colour: np.ndarray, rho_t: np.ndarray, h: np.ndarray, sigma: float,
              p0: float = 1.0, kappa: float = 2.0, nu_coeff: float = 0.1, c_acc: float = 0.25,
              c_vel: float = 1.0 / 40.0, c_visc: float = 0.125, box: np.ndarray | None = None):
    """All-pairs evaluation.  ``box`` (per-axis lengths) enables the minimum image."""
    n, d = x.shape
    diff = x[:, None, :] - x[None, :, :]
    if box is not None:
        diff -= box * np.round(diff / box)
    r = np.sqrt(np.sum(diff * diff, axis=-1))
    off = ~np.eye(n, dtype=bool)
    hij = 0.5 * (h[:, None] + h[None, :])
    # density with h_i, self included (kernel value at r = 0 on the diagonal)
    wi, _ = wendland(r / h[:, None], d)
    rho = np.sum(wi * (r < kappa * h[:, None]), axis=1) / h**d
    inter = (r < kappa * hij) & off
    _, dwq = wendland(r / hij, d)
    dW = dwq / hij ** (d + 1)
    P = p0 / rho_t**2
    beta = np.where(colour[:, None] != colour[None, :], sigma, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(inter & (r > 0), -(1.0 + beta) * (P[:, None] + P[None, :]) * dW / r, 0.0)
    a = np.einsum("ij,ijk->ik", s, diff)
    A = np.sum(np.abs(s) * r, axis=1)
    am = np.linalg.norm(a, axis=1)
    rc = kappa * h
    with np.errstate(divide="ignore"):
        dt1 = np.min(np.where(am > 0, c_acc * np.sqrt(rc / np.where(am > 0, am, 1.0)), np.inf))
    dt1 = 0.0 if not np.isfinite(dt1) else dt1
    vt = 0.5 * a * dt1
    vm = np.linalg.norm(vt, axis=1)
    nu = nu_coeff * rc * vm
    eta = rho_t * nu
    den = eta[:, None] + eta[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        etaij = np.where(den > 0, 2.0 * eta[:, None] * eta[None, :] / np.where(den > 0, den, 1.0), 0.0)
        inv2 = 1.0 / rho_t[:, None] ** 2 + 1.0 / rho_t[None, :] ** 2
        sv = np.where(inter & (r > 0), etaij * inv2 * dW / r, 0.0)
    vij = vt[:, None, :] - vt[None, :, :]
    at = np.einsum("ij,ijk->ik", sv, vij)
    cand = [np.where(am > 0, c_acc * np.sqrt(rc / np.where(am > 0, am, 1.0)), np.inf),
            np.where(vm > 0, c_vel * rc / np.where(vm > 0, vm, 1.0), np.inf),
            np.where(nu > 0, c_visc * rc**2 / np.where(nu > 0, nu, 1.0), np.inf)]
    dt2 = float(np.min(np.minimum(np.minimum(cand[0], cand[1]), cand[2])))
    dt2 = 0.0 if not np.isfinite(dt2) else dt2
    v = vt + 0.5 * at * dt2
    pairs = int(np.sum(inter))
    ifc = int(np.sum(inter & (colour[:, None] != colour[None, :]))) // 2
    nn = np.min(np.where(inter, r, np.inf), axis=1)
    return dict(rho=rho, a=a, a_abs=A, dt1=float(dt1), vt=vt, at=at, dt2=dt2, v=v, dr=v * dt2,
                pairs=pairs, interface_pairs=ifc, nn=nn)
