"""Electrode drives on the GPU (Sections 3.2 and 3.3): a vacuum gap behind a
series capacitor, driven by a current source, or by the two-harmonic
waveform follows its closed form; a floating electrode collecting a sheet
of charges ends at -(w / eps0) sum x_p; one argon step with a capacitor
matches the oracle from identical states, circuit charge included; and a
run resumed from a checkpoint continues bit for bit."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_helpers import small_argon, to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import paper_2609_17151_amd as P
    return P


def _vacuum(pic, drive, waveform=0, cap=0.0, j_amp=0.0, V=3.0, f=1.3, phase=0.4, nc=20, L=2.0, eps0=1.7, dt=0.01):
    sp = W.species(-1.0, 1.0, 1.0, 0, 1.0, capacity=4096, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=nc, bc=1, field_solve=1, length=L, dt=dt, eps0=eps0, v_amp=V, v_freq=f,
                        v_phase=phase, species=[sp], drive=drive, waveform=waveform, cap=cap, j_amp=j_amp)
    return pic.Sim(cfg), cfg


def _check_linear(sim, cfg, p0):
    nn = cfg["n_cells"] + 1
    np.testing.assert_allclose(sim.phi(), p0 * (1.0 - np.arange(nn) / (nn - 1)), atol=1e-12 * max(1.0, abs(p0)))
    np.testing.assert_allclose(sim.efield(), p0 / cfg["length"], atol=1e-12 * max(1.0, abs(p0)))
    assert sim.circuit()[0] == pytest.approx(p0, abs=1e-12 * max(1.0, abs(p0)))


def test_vacuum_drives_follow_their_closed_forms(pic):
    V, w, th, dt, L, e0 = 3.0, 2 * math.pi * 1.3, 0.4, 0.01, 2.0, 1.7
    C, J = 0.6, 0.25
    cap, _ = _vacuum(pic, W.DRIVE_CAPACITOR, cap=C)
    cur, cfg = _vacuum(pic, W.DRIVE_CURRENT, j_amp=J)
    two, _ = _vacuum(pic, W.DRIVE_VOLTAGE, waveform=W.WAVE_TWO_HARMONIC)
    v0 = V * math.sin(th)
    done = 0
    for n in (5, 37, 64):
        for s in (cap, cur, two):
            s.step(n - done)
        done = n
        t = n * dt
        _check_linear(cap, cfg, (C * V * math.sin(w * t + th) + e0 * v0 / L) / (C + e0 / L))
        q = J / w * (math.cos(th) - math.cos(w * t + th))
        _check_linear(cur, cfg, L / e0 * q)
        assert cur.circuit()[1] == pytest.approx(q, abs=1e-14)
        _check_linear(two, cfg, V * (math.cos(w * t + th) + math.cos(2 * w * t)))


def test_floating_electrode_collects_a_sheet(pic):
    n, L, e0, wgt = 4096, 1.0, 1.0, 1e-7
    sp = W.species(-1.0, 1.0, wgt, 0, 1.0, capacity=n, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=50, bc=1, field_solve=1, length=L, dt=0.01, eps0=e0, species=[sp],
                        drive=W.DRIVE_CAPACITOR, cap=0.0)
    sim = pic.Sim(cfg)
    rng = np.random.default_rng(2)
    cell = rng.integers(0, 50, n).astype(np.int32)
    off = rng.random(n).astype(np.float32)
    x = (cell + off.astype(np.float64)) * (L / 50)
    sim.set_particles(0, cell, off, -np.ones(n, np.float32), np.zeros(n, np.float32), np.zeros(n, np.float32),
                      np.arange(n, dtype=np.uint32), n, 0)
    assert sim.circuit()[0] == pytest.approx(0.0, abs=1e-12)
    sim.step(int(L / 0.01) + 2)
    assert sim.counts()["count"][0] == 0 and sim.wall()["absorbed"][0][0] == n
    assert sim.circuit()[0] == pytest.approx(-wgt / e0 * x.sum(), rel=1e-6)


def test_argon_step_with_capacitor_matches_oracle(pic):
    cfg, tabs = small_argon(n_init=20000)
    cfg.update(drive=W.DRIVE_CAPACITOR, cap=2e-3)
    sim = pic.Sim(cfg, tabs)
    sim.step(300)
    o = to_oracle(sim, cfg, tabs)
    o.set_circuit(sim.circuit()[1])
    o.refresh_field()
    np.testing.assert_allclose(sim.phi(), o.field()[1], rtol=0, atol=1e-6 * np.max(np.abs(o.field()[1])))
    for _ in range(3):
        sim.step(1)
        o.step(1)
        pg, qg = sim.circuit()
        po, qo = o.circuit()
        assert qg == pytest.approx(qo, rel=1e-9, abs=1e-12 * abs(qo) + 1e-30)
        assert pg == pytest.approx(po, rel=1e-5, abs=1e-5 * cfg["v_amp"])
        ph = o.field()[1]
        np.testing.assert_allclose(sim.phi(), ph, rtol=0, atol=1e-5 * np.max(np.abs(ph)))


def test_checkpoint_resume_with_circuit(pic, tmp_path):
    from paper_2609_17151_amd import checkpoint as K
    cfg, tabs = small_argon(n_init=20000)
    cfg.update(drive=W.DRIVE_CAPACITOR, cap=2e-3, waveform=W.WAVE_TWO_HARMONIC)
    a = pic.Sim(cfg, tabs)
    a.step(150)
    path = str(tmp_path / "circ.npz")
    K.save(a, path)
    a.step(60)
    b = K.load(path)
    b.step(60)
    for s in range(2):
        pa, pb = a.get_particles(s), b.get_particles(s)
        for k in ("cell", "off", "vx", "vy", "vz", "id"):
            assert np.array_equal(pa[k], pb[k]), (s, k)
    assert np.array_equal(a.phi(), b.phi())
    assert a.circuit()[1] == b.circuit()[1]
    b.close()


def test_circuit_rules(pic):
    s, _ = _vacuum(pic, W.DRIVE_VOLTAGE)
    with pytest.raises(RuntimeError):
        s.set_circuit(0.0)
    sp = W.species(-1.0, 1.0, 1.0, 0, 1.0, capacity=16, load=W.LOAD_NONE)
    for bad in (dict(bc=0, drive=W.DRIVE_CURRENT), dict(bc=1, drive=3), dict(bc=1, waveform=2),
                dict(bc=1, drive=W.DRIVE_CAPACITOR, cap=-1.0)):
        with pytest.raises(RuntimeError):
            pic.Sim(W.base_config(species=[sp], **bad))
