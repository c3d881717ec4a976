"""Pins of the electrode drives in the oracle (Section 3.2: a current-source
drive; Section 3.3: the two-harmonic voltage waveform and its DC self-bias,
which a series blocking capacitor lets develop).

Closed forms: a vacuum gap driven by a voltage has phi(0, t) = V(t); behind
a series capacitor C the source divides with the gap's capacitance eps0/L,
phi0(t) = (C V(t) + eps0 V(0) / L) / (C + eps0 / L); a current source
charges the electrode, phi0(t) = (L / eps0) int_0^t J; a floating electrode
(C = 0) that collects a sheet of unit negative charges ends at
phi0 = -(w / eps0) sum_p x_p(0) (the charge each particle induces on it,
-q w (1 - x/L), becomes its whole charge on arrival)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _vacuum(drive, waveform=W.WAVE_SINE, cap=0.0, j_amp=0.0, V=3.0, f=1.3, phase=0.4, nc=20, L=2.0, eps0=1.7,
            dt=0.01):
    sp = W.species(-1.0, 1.0, 1.0, 0, 1.0, capacity=16, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=nc, bc=1, field_solve=1, length=L, dt=dt, eps0=eps0, v_amp=V, v_freq=f,
                        v_phase=phase, species=[sp], drive=drive, waveform=waveform, cap=cap, j_amp=j_amp)
    o = oracle.Oracle(cfg, load=False)
    o.refresh_field()
    return o, cfg


def _linear(o, cfg, p0):
    rho, phi, ef = o.field()
    nn = cfg["n_cells"] + 1
    np.testing.assert_allclose(phi, p0 * (1.0 - np.arange(nn) / (nn - 1)), atol=1e-12 * max(1.0, abs(p0)))
    np.testing.assert_allclose(ef, p0 / cfg["length"], atol=1e-12 * max(1.0, abs(p0)))


def test_two_harmonic_voltage_waveform():
    o, cfg = _vacuum(W.DRIVE_VOLTAGE, waveform=W.WAVE_TWO_HARMONIC)
    V, w, th, dt = 3.0, 2 * math.pi * 1.3, 0.4, 0.01
    for n in (1, 7, 30):
        o.step(n if n == 1 else n - o.step_index)
        t = o.step_index * dt
        _linear(o, cfg, V * (math.cos(w * t + th) + math.cos(2 * w * t)))


def test_series_capacitor_divides_with_the_gap():
    C = 0.6
    o, cfg = _vacuum(W.DRIVE_CAPACITOR, cap=C)
    V, w, th, dt, L, e0 = 3.0, 2 * math.pi * 1.3, 0.4, 0.01, 2.0, 1.7
    v0 = V * math.sin(th)
    assert o.circuit()[0] == pytest.approx(v0, abs=1e-13)        # starts uncharged
    for n in (5, 23, 61):
        o.step(n - o.step_index)
        t = o.step_index * dt
        p0 = (C * V * math.sin(w * t + th) + e0 * v0 / L) / (C + e0 / L)
        _linear(o, cfg, p0)
        assert o.circuit()[0] == pytest.approx(p0, abs=1e-12)


def test_current_source_charges_the_electrode():
    J = 0.25
    o, cfg = _vacuum(W.DRIVE_CURRENT, j_amp=J)
    w, th, dt, L, e0 = 2 * math.pi * 1.3, 0.4, 0.01, 2.0, 1.7
    assert o.circuit()[0] == 0.0
    for n in (3, 40, 77):
        o.step(n - o.step_index)
        t = o.step_index * dt
        q = J / w * (math.cos(th) - math.cos(w * t + th))
        _linear(o, cfg, L / e0 * q)
        assert o.circuit()[1] == pytest.approx(q, abs=1e-14)


def test_floating_electrode_collects_a_sheet():
    n, L, e0, w = 500, 1.0, 1.0, 1e-7
    sp = W.species(-1.0, 1.0, w, 0, 1.0, capacity=n, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=50, bc=1, field_solve=1, length=L, dt=0.01, eps0=e0, species=[sp],
                        drive=W.DRIVE_CAPACITOR, cap=0.0)
    o = oracle.Oracle(cfg, load=False)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.0, L, n)
    o.set_particles(0, x, -np.ones(n), np.zeros(n), np.zeros(n), np.arange(n))
    o.refresh_field()
    assert o.circuit()[0] == pytest.approx(0.0, abs=1e-12)
    o.step(int(L / 0.01) + 2)
    assert len(o.get_particles(0)["x"]) == 0 and o.counters()["absorbed"][0][0] == n
    assert o.circuit()[0] == pytest.approx(-w / e0 * x.sum(), rel=1e-9)


def test_gauss_law_and_charge_bookkeeping_with_plasma():
    # argon with walls, secondaries and a series capacitor: at every step the
    # conductor's charge equals eps0 E(0) + C (phi0 - V), and it changes by
    # exactly the charge the particles brought
    cfg = W.argon_rf(n_init=3000, n_cells=100, weight=2e10, capacity=30000)
    cfg.update(drive=W.DRIVE_CAPACITOR, cap=5e-3)
    tabs = W.argon_tables(n=200)
    o = oracle.Oracle(cfg, tabs)
    C, e0 = cfg["cap"], cfg["eps0"]
    prev_q, prev_c = None, None
    for _ in range(12):
        o.step(5)
        p0, q = o.circuit()
        t = o.step_index * cfg["dt"]
        V = cfg["v_amp"] * math.sin(2 * math.pi * cfg["v_freq"] * t + cfg["v_phase"])
        ef = o.field()[2]
        assert q == pytest.approx(e0 * ef[0] + C * (p0 - V), rel=1e-9, abs=1e-9 * abs(C * V))
        c = o.counters()
        coll = sum(cfg["species"][k]["charge"] * cfg["species"][k]["weight"] * c["absorbed"][k][0]
                   for k in range(2)) - cfg["species"][0]["charge"] * cfg["species"][0]["weight"] * c["see_emitted"][0]
        if prev_q is not None:
            assert q - prev_q == pytest.approx(coll - prev_c, rel=1e-9, abs=1e-20)
        prev_q, prev_c = q, coll


def test_circuit_state_can_be_restored_and_is_rejected_without_a_circuit():
    o, cfg = _vacuum(W.DRIVE_CURRENT, j_amp=0.1)
    o.step(9)
    q = o.circuit()[1]
    o.set_circuit(q + 0.5)
    assert o.circuit()[1] == pytest.approx(q + 0.5)
    v, _ = _vacuum(W.DRIVE_VOLTAGE)
    with pytest.raises(oracle.OracleError):
        v.set_circuit(0.0)
    sp = W.species(-1.0, 1.0, 1.0, 0, 1.0, capacity=16, load=W.LOAD_NONE)
    with pytest.raises(oracle.OracleError):      # a periodic box has no electrode
        oracle.Oracle(W.base_config(bc=0, species=[sp], drive=W.DRIVE_CURRENT), load=False)
