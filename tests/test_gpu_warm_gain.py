"""What the trained warm-start network gains over the method without it.

Everything runs in the test, on the GPU: cold runs of 28 argon RF draws
from a narrow family (one batch, 240 RF periods; each draw's reference is
the mean of its last 50 periods), the network trained on 24 of them by the
library's own BF16 kernels, and the 4 held-out draws started from its
prediction.  The held-out draws' first 5-period window lies much closer to
their cold runs' references than the first window of the cold start does:
the network starts them near their periodic steady state instead of from a
uniform plasma; and, under the convergence rule of the sweeps (10 windows in
a row within max(2 %, 3 sigma) of the reference), they converge in fewer RF
periods than their cold runs did.
"""
import numpy as np
import pytest

import workloads as W
from paper_2609_17151_amd import steady

pytestmark = pytest.mark.gpu


def _draws(n, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        gap = rng.uniform(0.020, 0.030)
        out.append(dict(gap=gap, n_cells=int(round(gap / 6.25e-5)), pressure_mtorr=rng.uniform(30.0, 80.0),
                        v_amp=rng.uniform(150.0, 300.0), freq=13.56e6, see_gamma=0.1))
    return out


def test_warm_start_starts_near_the_steady_state():
    import paper_2609_17151_amd as P
    from paper_2609_17151_amd import warm
    from paper_2609_17151_amd.sweep import Sweep
    draws = _draws(28)
    weight = 4.0 * W.PILOT_WEIGHT
    tabs = W.argon_tables()
    cold_cfgs = [warm.config(d, weight=weight, seed=500 + i, n_init=50_000, capacity=1 << 19)
                 for i, d in enumerate(draws)]
    sim = P.Sim(cold_cfgs, tabs)
    spp = [warm.steps_per_period(d) for d in draws]
    sw = Sweep(sim, spp, window_periods=5, max_periods=240, progress=0).run()
    alive = [b for b in range(len(draws)) if all(c > 0 for c in sim.counts(b)["count"])]
    refs = {b: sw.reference(b, span=50) for b in alive}
    sim.close()
    train = [b for b in alive if b < 24]
    held = [b for b in alive if b >= 24]
    assert len(train) >= 20 and len(held) >= 3
    X = np.array([warm.inputs(draws[b]) for b in train])
    Y = np.array([steady.to_features(refs[b]) for b in train])
    model = warm.Model().fit(X, Y, steps=2000, lr=1e-3, batch=len(train))
    assert model.loss(X, Y) < 0.05
    feats = model.predict(np.array([warm.inputs(draws[b]) for b in held]))
    warm_cfgs = [warm.config(draws[b], weight=weight, seed=900 + b, capacity=1 << 19, cold=False) for b in held]
    sim2 = P.Sim(warm_cfgs, tabs)
    for j in range(len(held)):
        warm.start_from_features(sim2, j, warm_cfgs[j], feats[j])
    tols = {b: steady.noise_tolerance([steady.distance(w, refs[b]) for w in sw.windows[b]]) for b in held}

    def stop(j, s):
        return steady.converged_at(s.windows[j], refs[held[j]], tol=tols[held[j]]) is not None

    sw2 = Sweep(sim2, [spp[b] for b in held], window_periods=5, max_periods=150, progress=0).run(stop=stop)
    d_warm = [steady.distance(sw2.windows[j][0], refs[b]) for j, b in enumerate(held)]
    d_cold = [steady.distance(sw.windows[b][0], refs[b]) for b in held]
    sim2.close()
    # the network's start is at least three times closer than the cold start
    assert np.median(d_warm) < np.median(d_cold) / 3.0, (d_warm, d_cold)
    # and reaches the steady state in fewer RF periods (a run that does not
    # converge counts with its whole length)
    per = lambda i, n: 5 * (i + 1) if i is not None else n
    p_cold = [per(steady.converged_at(sw.windows[b], refs[b], tol=tols[b]), 240) for b in held]
    p_warm = [per(steady.converged_at(sw2.windows[j], refs[b], tol=tols[b]), 150) for j, b in enumerate(held)]
    print("periods to convergence, cold:", p_cold, "warm:", p_warm, flush=True)
    assert np.median(p_warm) < np.median(p_cold), (p_warm, p_cold)
