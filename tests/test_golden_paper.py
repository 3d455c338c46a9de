"""The dimensionless groups the paper prints (Sections 4.2-4.4) against the readings of its units.

The paper gives only density ratios.  Its printed capillary and Weber numbers contain the
water density, and they come out as printed only with the light phase at density 1 and
the water at rho_ratio (with water at density 1 they would be 1000x smaller); the fine
droplet-collision case prints U = 0.75, but its printed Re and We both need U = 0.075.
The Rayleigh-Taylor input of the tests and the bench is built from the printed groups of
the rho_ratio = 3 case; it must reproduce them.
"""
import json
import math
import os

import pytest

import pfinputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_dimensionless_groups.json")
CASES = json.load(open(GOLDEN))["cases"]


def _groups(p, rho_water):
    """Re, We, Ca, Pe with the paper's definitions: Re = U l / nu_water, We = rho_water U^2
    l / sigma, Ca = rho_water U nu_water / sigma, Pe = U l / M, where l is the diameter
    (collision), the horizontal length (Rayleigh-Taylor, U = sqrt(g L)) or the column
    height (dam break, U = sqrt(g H))."""
    if "D" in p:
        U, l = p["U"], p["D"]
    elif "L" in p:
        l = p["L"]
        U = math.sqrt(p["g"] * l)
    else:
        l = p["H"]
        U = math.sqrt(p["g"] * l)
    out = {"Re": U * l / p["nu_water"], "We": rho_water * U * U * l / p["sigma"],
           "Ca": rho_water * U * p["nu_water"] / p["sigma"]}
    if "M" in p:
        out["Pe"] = U * l / p["M"]
    return out


def _close(value, printed):
    # two printed significant digits: within half a unit of the second digit, plus the
    # "approximately" of the Rayleigh-Taylor Re (3159 for the 256-wide case)
    return abs(value - printed) <= 0.06 * abs(printed)


@pytest.mark.parametrize("case", CASES, ids=[c["source"][:40] for c in CASES])
def test_printed_groups_with_heavy_phase_at_rho_ratio(case):
    p = case["params"]
    got = _groups(p, rho_water=p["rho_ratio"])
    for name, printed in case["printed"].items():
        assert _close(got[name], printed), (name, got[name], printed)


@pytest.mark.parametrize("case", [c for c in CASES if {"We", "Ca"} & set(c["printed"])
                                  and c["params"]["rho_ratio"] >= 1000],
                         ids=lambda c: c["source"][:40])
def test_water_at_density_one_contradicts_the_paper(case):
    p = case["params"]
    got = _groups(p, rho_water=1.0)
    for name in {"We", "Ca"} & set(case["printed"]):
        assert not _close(got[name], case["printed"][name]), name


def test_fine_collision_speed_reading():
    case = next(c for c in CASES if "U_as_printed" in c["params"])
    p = dict(case["params"])
    assert _close(_groups(p, p["rho_ratio"])["Re"], case["printed"]["Re"])
    p["U"] = p["U_as_printed"]
    got = _groups(p, p["rho_ratio"])
    assert not _close(got["Re"], case["printed"]["Re"])
    assert not _close(got["We"], case["printed"]["We"])


def test_rayleigh_taylor_input_reproduces_printed_groups():
    cfg = pfinputs.rayleigh_taylor()
    case = next(c for c in CASES if c["params"].get("rho_ratio") == 3)
    L = cfg["shape"][0]
    U = math.sqrt(abs(cfg["g"][1]) * L)
    assert cfg["rho_L"] == 1.0 and cfg["rho_H"] == case["params"]["rho_ratio"]
    assert _close(U * L / cfg["nu_H"], case["printed"]["Re"])
    assert _close(U * L / cfg["M"], case["printed"]["Pe"])
    assert _close(cfg["rho_H"] * U * cfg["nu_H"] / cfg["sigma"], case["printed"]["Ca"])
    # equal dynamic viscosities (mu_ratio 1 of that case)
    assert abs(cfg["rho_H"] * cfg["nu_H"] - cfg["rho_L"] * cfg["nu_L"]) < 1e-12
