"""The closed-form pins catch plausible slips in the oracle.

Each case plants one mistake in a copy of the oracle's C source (a dropped factor, a wrong
radius, a clamp in place of a mirror, a missing projection, a flipped sign), compiles the copy
with the oracle's own flags and requires at least one closed-form check of
tests/closed_forms.py to fail against it.  The planted mistakes live only in the temporary copy.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle import oracle as O
from tests import closed_forms as CF

SRC = os.path.join(os.path.dirname(O.__file__), "mpsph_oracle.c")

# (name, text in the oracle, replacement, expected number of occurrences)
MUTANTS = [
    ("halved_harmonic_mean", "double etaij = 2.0 * eta[i] * eta[j] / (eta[i] + eta[j]);",
     "double etaij = eta[i] * eta[j] / (eta[i] + eta[j]);", 1),
    ("arithmetic_mean_viscosity", "double etaij = 2.0 * eta[i] * eta[j] / (eta[i] + eta[j]);",
     "double etaij = 0.5 * (eta[i] + eta[j]);", 1),
    ("viscosity_with_h_not_rc", "eta[i] = rho_t[i] * p->nu_coeff * kap * h[i] * sqrt(sp);",
     "eta[i] = rho_t[i] * p->nu_coeff * h[i] * sqrt(sp);", 1),
    ("viscous_density_of_i_only", "double inv2 = 1.0 / (rho_t[i] * rho_t[i]) + 1.0 / (rho_t[j] * rho_t[j]);",
     "double inv2 = 2.0 / (rho_t[i] * rho_t[i]);", 1),
    ("dt1_radius_h_not_kappa_h", "if (am > 0.0) dt1 = fmin(dt1, p->c_acc * sqrt(kap * h[i] / am));",
     "if (am > 0.0) dt1 = fmin(dt1, p->c_acc * sqrt(h[i] / am));", 1),
    ("dt2_without_cfl_term", "if (vm > 0.0) dt2 = fmin(dt2, p->c_vel * rci / vm);", "", 1),
    ("midpoint_velocity_without_half", "0.0 : 0.5 * a[i * d + c] * dt1;", "0.0 : a[i * d + c] * dt1;", 1),
    ("velocity_with_full_viscous_kick", "vt[i * d + c] + 0.5 * at[i * d + c] * dt2;",
     "vt[i * d + c] + at[i * d + c] * dt2;", 1),
    ("pressure_over_rho_t_not_squared", "P[i] = p->p0 / (rho_t[i] * rho_t[i]);", "P[i] = p->p0 / rho_t[i];", 1),
    ("attractive_pair_force", "double s = -(1.0 + beta) * (P[i] + P[j])", "double s = (1.0 + beta) * (P[i] + P[j])", 1),
    ("surface_tension_without_one", "double s = -(1.0 + beta) * (P[i] + P[j])", "double s = -(2.0 * beta) * (P[i] + P[j])", 1),
    ("pair_length_max_not_mean", "double hij = 0.5 * (h[i] + h[j]);", "double hij = fmax(h[i], h[j]);", 2),
    ("density_with_pair_length", "if (r < kap * h[i]) rs += orc_kernel_w(r, h[i], d);",
     "if (r < kap * h[i]) rs += orc_kernel_w(r, 0.5 * (h[i] + h[j]), d);", 1),
    ("seeded_wall_clamps", "if (xi[a] < p->lo[a]) xi[a] = fmin(2.0 * p->lo[a] - xi[a], p->hi[a]);",
     "if (xi[a] < p->lo[a]) xi[a] = p->lo[a];", 1),
    ("seeded_sphere_projects", "rt = 2.0 * p->r_out - r;", "rt = p->r_out;", 1),
    ("seeded_inner_circle_projects", "rt = 2.0 * p->r_in - r;", "rt = p->r_in;", 1),
    ("seeded_levelset_projects", "double f = *type == ORC_NORMAL ? 2.0 : 1.0;", "double f = 1.0;", 1),
    ("levelset_force_not_mapped", "for (int a = 0; a < d; ++a) f[a] -= dot * g[a] / gn;", ";", 1),
    ("levelset_crossing_not_retagged", "if (*type < ORC_SURFACE) *type = ORC_SURFACE;", ";", 1),
]


def _build(tmp, name, old, new, count):
    src = open(SRC, encoding="utf-8").read()
    assert src.count(old) == count, (name, src.count(old))
    path = os.path.join(tmp, f"{name}.c")
    with open(path, "w", encoding="utf-8") as f:
        f.write(src.replace(old, new))
    so = os.path.join(tmp, f"lib_{name}.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                           "-I", os.path.dirname(SRC), path,
                           "-o", so, "-lm"])
    return so


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("mutants"))
    with ThreadPoolExecutor(max_workers=8) as ex:
        futs = {m[0]: ex.submit(_build, tmp, *m) for m in MUTANTS}
        return {k: f.result() for k, f in futs.items()}


def _run_against(monkeypatch, so):
    monkeypatch.setattr(O, "_SO", so)
    monkeypatch.setattr(O, "_lib", None)
    try:
        cases = CF.all_checks(O)
    except (ArithmeticError, ValueError, RuntimeError) as e:      # a domain error is a failure too
        return [("exception", repr(e))]
    return [(name, bad) for name, checks in cases for bad in [CF.failures(checks)] if bad]


def test_unmodified_copy_passes(monkeypatch, tmp_path):
    so = _build(str(tmp_path), "unmodified", "#include <math.h>", "#include <math.h>", 1)
    assert _run_against(monkeypatch, so) == []


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(monkeypatch, mutant_libs, name):
    failed = _run_against(monkeypatch, mutant_libs[name])
    assert failed, f"no closed-form pin fails with the mistake '{name}'"
