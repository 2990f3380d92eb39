"""GPU: the paper's Section-4 mono- vs multi-morphology networks (the size
group of 20 neurons with spread 700 and mean 300, and its mono-morphology
counterpart of 300-compartment neurons) run for a few epochs under plain,
compartment-count and learned packing: the three packings give bitwise
identical voltages and spikes, and a subset of the multi-morphology neurons,
replayed in the oracle from the GPU's recorded spikes, matches it."""
import sys

import numpy as np
import pytest

from paper_2005_06332_amd import workload as W

pytestmark = pytest.mark.gpu

N_NEURONS = 2000
STEPS = 120


@pytest.fixture(scope="module")
def S():
    from paper_2005_06332_amd import sim
    sim.lib()
    return sim


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cost_model(S):
    from paper_2005_06332_amd import costmodel
    return costmodel.load_or_train(solver=S.SOLVE_CONTRACT)


@pytest.mark.parametrize("mono", [False, True])
def test_section4_networks_pack_three_ways_identically(S, orc, cost_model, mono):
    prob = W.size_group(7, N_NEURONS, mono=mono, n_steps=STEPS)
    assert int(prob["comp_off"][-1]) == N_NEURONS * 300
    outs = {}
    for name, kw in (("plain", dict(packing=S.PACK_PLAIN)),
                     ("count", dict(packing=S.PACK_COUNT)),
                     ("learned", dict(packing=S.PACK_LEARNED, cost_model=cost_model))):
        with S.Simulation(prob, solver=S.SOLVE_CONTRACT, **kw) as g:
            say(f"case section4 mono={mono} {name}: {g.config}")
            g.step(STEPS)
            outs[name] = (g.voltages(), g.spikes())
    v0, s0 = outs["plain"]
    for name in ("count", "learned"):
        assert np.array_equal(outs[name][0], v0), name
        assert np.array_equal(outs[name][1], s0), name
    assert len(s0) > 0
    # a neuron subset against the oracle, replayed from the GPU's spikes
    rng = np.random.default_rng(3)
    targets = np.sort(rng.choice(N_NEURONS, 12, replace=False))
    rep = orc.Sim(W.replay_subset(prob, targets), max_steps=STEPS)
    rep.set_input_raster(W.spike_raster(s0, N_NEURONS, STEPS))
    rep.step(STEPS)
    vr, sr = rep.voltages(), rep.spikes()
    rep.close()
    off = prob["comp_off"]
    want = np.concatenate([v0[off[j]:off[j + 1]] for j in targets])
    pos = {int(j): k for k, j in enumerate(targets)}
    gsp = np.array(sorted((pos[int(n)], int(t)) for n, t in s0 if int(n) in pos),
                   np.int64).reshape(-1, 2)
    osp = np.array(sorted(map(tuple, sr.tolist())), np.int64).reshape(-1, 2)
    d = float(np.abs(want - vr).max())
    say(f"  replay of {len(targets)} neurons: max|dV| {d:.3e} mV, spikes {len(gsp)} vs {len(osp)}")
    assert d <= 1e-4
    assert np.array_equal(gsp, osp)
