"""The electron cyclotron drift instability on the GPU (Section 3.6, Figure
10): in a periodic azimuthal box of 15 resonant wavelengths at the paper's
fields (B = 200 G, E = 20 kV/m) and density (1e17 m^-3), with axial renewal,
the cyclotron resonance makes mode 15 -- the wavelength
lambda_1 = 2 pi v_E / omega_ce, 1.786 mm -- the dominant mode of the ion
density while the instability grows (tests/golden/exb_wavelength.json).

At 1e6 macro-particles per species the thermal noise seeds the growth early:
the fluctuation passes a few per cent of the mean after about 0.5 us and
mode 15 leads the space-time spectrum from there to about 1.2 us, after
which the inverse cascade moves power to longer modes."""
import json
import os

import numpy as np
import pytest

import workloads as W
from paper_2609_17151_amd import spectrum

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exb_wavelength.json")


def test_resonant_mode_dominates_during_growth():
    import paper_2609_17151_amd as P
    with open(GOLDEN) as f:
        g = json.load(f)
    cfg = W.ecdi(n_lambda=15, n_cells=1024, n_per_species=1_000_000, b_field=g["b_tesla"], e_field=g["e_v_per_m"])
    sim = P.Sim(cfg)
    every = 128
    dts = every * cfg["dt"]
    count = int(round(1.2e-6 / dts))
    hist = spectrum.record(sim, 1, every, count)
    assert sim.renewed().sum() > 0
    t = (np.arange(count) + 1) * dts
    early = hist[t < 0.2e-6]
    grow = hist[(t >= 0.6e-6) & (t < 1.2e-6)]
    m, lam = spectrum.dominant_mode(grow, cfg["length"], dts)
    amp0 = float(np.std(early) / np.mean(hist))
    amp1 = float(np.std(grow) / np.mean(hist))
    print("ECDI: dominant mode %d (%.4f mm) over 0.6-1.2 us; fluctuation %.3f -> %.3f of the mean"
          % (m, lam * 1e3, amp0, amp1))
    assert amp1 > 2.0 * amp0                          # the instability grows
    assert m == 15
    assert abs(lam * 1e3 - g["lambda1_mm_predicted"]) <= 0.0005
    sim.close()
