"""Closed-form pins of the oracle's step (two- and three-particle arrangements worked out by
hand from Eq. 17-32; the derivations are in tests/closed_forms.py).

They fix what the invariance and brute-force pins cannot: the size of the viscous term (its
harmonic mean of the viscosities, Eq. 20-22), the absolute first time step with r_c = kappa h
(Eq. 29), the velocity and drift (Eq. 26-28), the mirror rule of seeded features at box walls,
circles, spheres and level sets, the projection and re-tagging of Eq. 32, and the force mapping
of a surface particle on a level set (Eq. 31).
"""
import pytest

from oracle import oracle as O
from tests import closed_forms as CF


@pytest.fixture(scope="module")
def checks(oracle_lib):
    return dict(CF.all_checks(O))


NAMES = [f"equal_pair_{d}d_{c}_colour" for d in (2, 3) for c in ("one", "two")] + \
    [f"unequal_pair_{d}d" for d in (2, 3)] + \
    [f"{kind}_{d}d_{tag}" for kind in ("wall", "ball", "levelset_crossing") for d in (2, 3) for tag in ("retag", "seeded")] + \
    [f"levelset_force_{d}d" for d in (2, 3)] + ["annulus_inner_retag", "annulus_inner_seeded"]


@pytest.mark.parametrize("name", NAMES)
def test_closed_form(checks, name):
    bad = CF.failures(checks[name])
    assert not bad, bad


def test_every_case_is_listed(checks):
    assert sorted(checks) == sorted(NAMES)
