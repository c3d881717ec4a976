"""RF windows closed on the device (pic_set_windows / pic_get_windows) equal
the time averages read and cleared by the host at the same steps, bit for
bit, in a batch whose discharges have different window lengths; a retired
discharge closes no more windows; and the sweep driver's device mode
reaches the same windows as its host mode."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import paper_2609_17151_amd as P
    return P


def _batch():
    return [W.argon_rf(n_init=n, n_cells=nc, gap=g, v_amp=v, seed=300 + i, capacity=4 * n, weight=3e13 / n)
            for i, (n, nc, g, v) in enumerate(((8000, 200, 0.015, 150.0), (15000, 317, 0.021, 320.0)))]


def test_device_windows_equal_host_windows(pic):
    cfgs, tabs = _batch(), W.argon_tables()
    lens = [96, 160]
    a = pic.Sim(cfgs, tabs)
    a.set_diag(True)
    a.step(40)
    for b in range(2):
        a.set_windows(b, lens[b])
    a.step(480)
    h = pic.Sim(cfgs, tabs)
    h.set_diag(True)
    h.step(40)
    for b in range(2):
        h.reset_avg(b)
    host = [[], []]
    for t in range(1, 481):
        h.step(1)
        for b in range(2):
            if t % lens[b] == 0:
                host[b].append(h.avg(b))
                h.reset_avg(b)
    for b in range(2):
        dev = a.windows(b)
        assert len(dev) == 480 // lens[b] == len(host[b])
        for wd, wh in zip(dev, host[b]):
            assert wd["samples"] == wh["samples"] == lens[b]
            for k in ("density", "phi", "mean_energy"):
                assert np.array_equal(wd[k], wh[k]), (b, k)
    # a retired discharge closes no more windows
    a.retire(0)
    a.step(200)
    assert len(a.windows(0)) == 5 and len(a.windows(1)) == 680 // 160
    with pytest.raises(RuntimeError):
        a.windows(1, first=10, count=1)


def test_sweep_device_mode_matches_host_mode(pic):
    from paper_2609_17151_amd.sweep import Sweep
    cfgs, tabs = _batch(), W.argon_tables()
    out = []
    for chunk in (0, 64):
        sim = pic.Sim(cfgs, tabs)
        sw = Sweep(sim, [48, 40], window_periods=2, max_periods=12, chunk=chunk, progress=0).run()
        out.append(sw)
    for b in range(2):
        assert out[0].window_step[b] == out[1].window_step[b]
        for w0, w1 in zip(out[0].windows[b], out[1].windows[b]):
            assert np.array_equal(w0, w1)


def test_tuned_sweep_matches_untuned(pic):
    # the autotuner's steps come before the first window and change no
    # result: an untuned batch stepped as far first closes the same windows
    from paper_2609_17151_amd.sweep import Sweep
    cfgs, tabs = _batch(), W.argon_tables()
    sim_t = pic.Sim(cfgs, tabs)
    sw_t = Sweep(sim_t, [48, 40], window_periods=2, max_periods=6, chunk=64, progress=0, tune=True).run()
    assert sw_t.schedule is not None
    start = sw_t.window_step[0][0] - sw_t.window_steps(0)
    assert start > 0
    sim_u = pic.Sim(cfgs, tabs)
    sim_u.step(start)
    sw_u = Sweep(sim_u, [48, 40], window_periods=2, max_periods=6, chunk=64, progress=0).run()
    for b in range(2):
        assert sw_t.window_step[b] == sw_u.window_step[b]
        for w0, w1 in zip(sw_t.windows[b], sw_u.windows[b]):
            assert np.array_equal(w0, w1)
