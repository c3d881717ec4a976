"""Time-averaged profiles of independent runs, GPU against oracle: from one
identical argon state (collisions, walls, secondaries) both sides run 600
steps on their own.  The runs decorrelate chaotically after the first
differing collision, so only statistics compare: the time-mean densities,
potential and bulk EEPF agree point by point within 2 % of their maximum or
three standard errors of the difference, the errors taken from block means
(six blocks of 100 steps on each side)."""
import numpy as np
import pytest

from gpu_helpers import small_argon, to_oracle

pytestmark = pytest.mark.gpu

BLOCKS, BLOCK = 6, 100


def _blocks(x, step, read, reset):
    out = []
    for _ in range(BLOCKS):
        reset()
        step(BLOCK)
        out.append(read())
    return out


def _within(g, o, what, frac=0.98):
    """Per point: |mean_g - mean_o| <= max(2 % of the max, 3 sigma)."""
    g, o = np.asarray(g), np.asarray(o)
    mg, mo = g.mean(axis=0), o.mean(axis=0)
    se = np.sqrt(g.var(axis=0, ddof=1) / len(g) + o.var(axis=0, ddof=1) / len(o))
    bar = np.maximum(0.02 * np.max(np.abs(mo)), 3.0 * se)
    ok = np.abs(mg - mo) <= bar
    assert ok.mean() >= frac, (what, ok.mean(), np.max(np.abs(mg - mo) / np.max(np.abs(mo))))


def test_independent_runs_agree_in_time_average():
    import paper_2609_17151_amd as P
    cfg, tabs = small_argon(n_init=20000)
    sim = P.Sim(cfg, tabs)
    sim.step(400)
    o = to_oracle(sim, cfg, tabs)
    sim.set_diag(True, eepf_emax=30.0)
    o.set_diag(True, eepf_emax=30.0)

    def g_read():
        a, h = sim.avg(), sim.eepf()
        return np.concatenate([a["density"][0], a["density"][1], a["phi"], h["bulk"] / max(h["samples"], 1.0)])

    def o_read():
        a, h = o.avg(), o.eepf()
        return np.concatenate([a["density"][0], a["density"][1], a["phi"], h["bulk"] / max(h["samples"], 1.0)])

    def g_reset():
        sim.reset_avg()

    def o_reset():
        o.reset_avg()

    bg = _blocks(sim, sim.step, g_read, g_reset)
    bo = _blocks(o, o.step, o_read, o_reset)
    nn = sim.n_nodes[0]
    g, oo = np.array(bg), np.array(bo)
    _within(g[:, :nn], oo[:, :nn], "electron density")
    _within(g[:, nn:2 * nn], oo[:, nn:2 * nn], "ion density")
    _within(g[:, 2 * nn:3 * nn], oo[:, 2 * nn:3 * nn], "potential")
    _within(g[:, 3 * nn:], oo[:, 3 * nn:], "bulk EEPF")
