"""The resonant wavelength of the electron cyclotron drift instability
(Section 3.6, Figure 10): the cyclotron resonance selects
lambda_1 = 2 pi v_E / omega_ce, v_E = E / B, which the paper gives as
1.786 mm at B = 200 G and E = 20 kV/m and measures as 1.787 mm
(tests/golden/exb_wavelength.json).  The ECDI box of the workloads holds a
whole number of these wavelengths."""
import json
import math
import os

import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exb_wavelength.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_lambda1_matches_the_paper():
    g = _golden()
    lam_mm = W.lambda1(e_field=g["e_v_per_m"], b_field=g["b_tesla"]) * 1e3
    # to the printed digits of the prediction, and within the run's 1.787
    assert abs(lam_mm - g["lambda1_mm_predicted"]) <= 0.0005, lam_mm
    assert abs(lam_mm - g["lambda1_mm_measured"]) <= 0.0015, lam_mm


def test_lambda1_from_its_physical_constants():
    # independent of the workload module's own constants: CODATA electron
    # mass and elementary charge, omega_ce = e B / m_e
    g = _golden()
    me, e = 9.1093837015e-31, 1.602176634e-19
    v_e = g["e_v_per_m"] / g["b_tesla"]
    lam = 2.0 * math.pi * v_e / (e * g["b_tesla"] / me)
    assert W.lambda1(e_field=g["e_v_per_m"], b_field=g["b_tesla"]) == pytest.approx(lam, rel=1e-9)


def test_ecdi_box_holds_whole_wavelengths():
    g = _golden()
    lam = W.lambda1(e_field=g["e_v_per_m"], b_field=g["b_tesla"])
    cfg = W.ecdi(n_lambda=15, n_per_species=64, n_cells=1024)
    assert cfg["length"] == pytest.approx(15 * lam, rel=1e-14)
    assert cfg["renew_lz"] > 0.0
    assert cfg["b_ext"][1] == g["b_tesla"] and cfg["e_ext"][2] == g["e_v_per_m"]
