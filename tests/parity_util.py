"""Helpers that run the same seeded input through the HIP library and the CPU oracle."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_1906_07925_amd import workloads as W

FIELDS = ("rho", "rho_t", "h", "a", "a_abs", "vt", "at", "v", "dr", "nn", "x0")


def state_f32(cfg):
    """Seeded initial state with positions rounded to float32 (the GPU's input type); the oracle
    receives the same float32 values widened to float64."""
    x, col, typ = W.make_state(cfg)
    x32 = x.astype(np.float32)
    return x32, col, typ


def oracle_step(spec, s0, x32, col, typ, step_index=0, search="grid"):
    op = O.OracleParams(spec, s0=s0, search=search)
    x1, t1, r = O.step(op, x32.astype(np.float64), col, typ, step_index)
    return op, x1, t1, r


def gpu_run(spec, s0, x32, col, typ, steps=1, cell_log2=-1, debug=True, fields=FIELDS):
    import torch
    from paper_1906_07925_amd import mpsph as M
    n = x32.shape[0]
    R = M.Relaxer(spec, n=n, s0=s0, cell_log2=cell_log2, debug=debug)
    R.load(torch.from_numpy(x32).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    R.step(steps)
    m = R.metrics(allow_nonfinite=True)
    out = {k: R.field(k).cpu().numpy().astype(np.float64) for k in fields} if steps > 0 else {}
    xg, tg = R.store()
    out["x1"] = xg.cpu().numpy().astype(np.float64)
    out["t1"] = tg.cpu().numpy()
    out["k"] = R.cell_log2()
    R.close()
    return m, out


def rel(a, b):
    d = np.linalg.norm(np.asarray(a) - np.asarray(b))
    s = np.linalg.norm(np.asarray(b))
    return d / s if s > 0 else d


def check_single_step(spec, s0, x32, col, typ, tol=1e-5, cell_log2=-1, report=None):
    """Single step from identical FP32 inputs: GPU FP32 vs oracle FP64, per quantity."""
    op, x1, t1, r = oracle_step(spec, s0, x32, col, typ)
    m, g = gpu_run(spec, s0, x32, col, typ, cell_log2=cell_log2)
    d = spec["dim"]
    errs = {}
    # start-of-step positions round-trip through (cell, offset) to within float32 rounding
    errs["x0"] = np.max(np.abs(g["x0"] - x32)) / max(np.max(np.abs(x32)), 1e-30)
    # density: sum of positive terms, relative per particle
    errs["rho"] = np.max(np.abs(g["rho"] - r["rho"]) / r["rho"])
    errs["rho_t"] = np.max(np.abs(g["rho_t"] - r["rho_t"]) / r["rho_t"])
    # accelerations: condition-aware per particle and normwise.  Per particle the bound is
    #   tol * A_i + delta_i * K_i,
    # A_i = sum of |pair terms| (FP32 accumulation), K_i = sum of |pair term| (1 + 3q/(2 - q)):
    # a relative change delta of r_ij changes a kernel-derivative term by (1 + 3q/(2-q)) delta
    # (the factor (1 - q/2)^3 near the support edge).  delta_i is 4 ulp of FP32 plus the
    # rounding of the GPU's float32 cell offsets, ~1.5e-7 cell side cs over the separation
    # (bounded through the nearest-neighbour distance nn_i of the oracle).
    L = max(spec["hi"][a] - spec["lo"][a] for a in range(d))
    cs = L / (2 ** g["k"] - 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        dlt = 4.0 * 2.0 ** -24 + 1.5e-7 * cs / r["nn"]
    dlt = np.where(np.isfinite(dlt), dlt, 0.0)[:, None]
    A = r["a_abs"][:, None]
    bound_a = tol * A + dlt * r["a_kabs"][:, None]
    da = np.abs(g["a"] - r["a"])
    errs["a_cond"] = np.max(np.where(bound_a > 0, da / np.maximum(bound_a, 1e-300) * tol, da))
    errs["a_norm"] = rel(g["a"], r["a"])
    errs["dt1"] = abs(m["dt1"] - r["dt1"]) / r["dt1"] if r["dt1"] > 0 else abs(m["dt1"])
    errs["dt2"] = abs(m["dt2"] - r["dt2"]) / r["dt2"] if r["dt2"] > 0 else abs(m["dt2"])
    errs["vt_norm"] = rel(g["vt"], r["vt"])
    # the viscous acceleration also inherits the error of a: v~ = a dt1 / 2 enters the velocity
    # differences and, through |v~|, the viscosities; a near-balanced particle (|a_j| << A_j)
    # has a v~ of large relative error.  The oracle's at_prop is that propagated error per unit
    # relative error of the |pair term| sums of a.
    AT = r["at_abs"][:, None]
    dat = np.abs(g["at"] - r["at"])
    bound_at = tol * AT + dlt * r["at_kabs"][:, None] + tol * r["at_prop"][:, None]
    errs["at_cond"] = np.max(np.where(bound_at > 0, dat / np.maximum(bound_at, 1e-300) * tol, dat))
    errs["at_norm"] = rel(g["at"], r["at"])
    errs["v_norm"] = rel(g["v"], r["v"])
    errs["dr_norm"] = rel(g["dr"], r["dr"])
    errs["residual_l2"] = abs(m["residual_l2"] - r["residual_l2"]) / max(r["residual_l2"], 1.0)
    errs["kinetic"] = abs(m["kinetic"] - r["kinetic"]) / r["kinetic"] if r["kinetic"] > 0 else abs(m["kinetic"])
    errs["elr_mean"] = abs(m["elr_mean"] - r["elr_mean"]) / max(r["elr_mean"], 1e-30)
    counts = dict(pairs=(m["pairs"], r["pairs"]), interface_pairs=(m["interface_pairs"], r["interface_pairs"]),
                  n_normal=(m["n_normal"], r["n_normal"]), band=r["band_pairs"])
    if report is not None:
        report.update(errs=errs, counts=counts, k=g["k"], oracle=r, gpu_metrics=m)
    # bounds
    assert errs["x0"] < 4e-7, errs
    for k in ("rho", "rho_t", "a_cond", "a_norm", "dt1", "dt2", "vt_norm", "v_norm", "dr_norm", "residual_l2",
              "kinetic", "elr_mean"):
        assert errs[k] <= tol, (k, errs)
    assert errs["at_cond"] <= 10 * tol and errs["at_norm"] <= tol, errs
    band = r["band_pairs"]
    assert abs(m["pairs"] - r["pairs"]) <= band, counts
    assert abs(m["interface_pairs"] - r["interface_pairs"]) <= band, counts
    assert m["n_normal"] == r["n_normal"] and m["nonfinite"] == 0
    # positions after the step: displacement error plus float32 rounding of the position; a
    # projection onto a circle or sphere is computed relative to the centre in FP32 cell units,
    # so it rounds at a few ulp of the radius whatever the size of the coordinate
    dx = np.abs(g["x1"] - x1)
    ulp = np.spacing(np.abs(x1).astype(np.float32)).astype(np.float64)
    if spec["geometry"] in ("ball", "annulus"):
        ulp = ulp + 2.0 ** -24 * spec["r_out"]
    drn = np.linalg.norm(r["dr"], axis=1)[:, None]
    assert np.all(dx <= 4 * ulp + 10 * tol * drn + 1e-12), np.max(dx / (4 * ulp + 10 * tol * drn))
    assert np.array_equal(g["t1"], t1)
    return errs
