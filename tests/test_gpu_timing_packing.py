"""GPU: launch timing and best-fit packing.

- Launch timing (sim_set_kernel_timing) counts every epoch, whether it ran
  from a graph replay or as a direct (partial-epoch) launch. It reports
  per-class launch spans that fit inside their epochs. It changes no result.
- Best-fit packing puts more compartments in each pack than the plain
  consecutive packing. Both give bitwise identical results.
"""
import sys

import numpy as np
import pytest

from paper_2005_06332_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2005_06332_amd import sim
    sim.lib()
    return sim


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def field(config, key):
    return config.split(key + "=")[1].split()[0]


def test_launch_timing_counts_epochs_and_changes_nothing(S):
    prob = W.subset(W.make(3), np.arange(600))  # sizes up to ~2,000: two size classes
    E = 40
    steps = 3 * E + 7  # three whole epochs (graph replays), then a partial epoch
    with S.Simulation(prob, solver=1) as g:
        say("config:", g.config)
        wg = [int(x) for x in field(g.config, "wg").split("+")]
        g.step(E)
        g.set_kernel_timing(True)
        g.step(steps)
        ms, launches = g.kernel_time()
        cls = [g.class_time(c) for c in range(3)]
        v_timed, s_timed = g.voltages(), g.spikes()
    say(f"epochs {launches}, {ms:.3f} ms; classes {cls}")
    assert launches == 4
    assert ms > 0
    for c in range(3):
        c_ms, c_n, c_comps, c_upd = cls[c]
        if wg[c] == 0:
            assert c_n == 0 and c_upd == 0
            continue
        assert c_n == 4 and c_comps > 0
        # the units of the timed launches: the class's compartments times the
        # steps each launch ran (three whole epochs and a partial one)
        assert c_upd == c_comps * steps
        assert 0 < c_ms <= ms * 1.02  # each launch lies inside its epoch
    with S.Simulation(prob, solver=1) as g:
        g.step(E + steps)
        assert np.array_equal(g.voltages(), v_timed)
        assert np.array_equal(g.spikes(), s_timed)


def test_best_fit_packs_are_fuller_than_plain_and_change_nothing(S):
    prob = W.subset(W.make(3), np.arange(2048))
    out = {}
    for packing in (S.PACK_PLAIN, S.PACK_COUNT):
        with S.Simulation(prob, solver=1, packing=packing) as g:
            g.step(80)
            out[packing] = (int(field(g.config, "packs")), g.voltages(), g.spikes())
            say(packing, g.config)
    n_plain, v_plain, s_plain = out[S.PACK_PLAIN]
    n_count, v_count, s_count = out[S.PACK_COUNT]
    assert n_count < n_plain
    assert np.array_equal(v_plain, v_count)
    assert np.array_equal(s_plain, s_count)
