"""sim_step_noalloc (the stepping entry point that allocates nothing) against
sim_step on twin simulations, through the C ABI.

Layouts are forced to keep their larger packs' state in global memory (small
LDS budgets), so the fixed scratch array is what the kernels use. Results must
be bitwise identical (same kernels, same order of operations); spikes of the
allocation-free calls come back through the caller's buffer. Two calls in a
row, the second on a smaller network, then one simulation stepped twice."""
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


def n_global(config):
    return int(config.split("global_packs=")[1].split()[0])


@pytest.mark.parametrize("solver", [0, 1, 2])
def test_noalloc_matches_step_two_calls_second_smaller(S, solver):
    kw = dict(solver=solver, pack_comps=600, lds_comps=120, lds_classes=1)
    for prob, steps in ((W.mini(seed=11, n_neurons=48, n_steps=200), 200),
                        (W.mini(seed=12, n_neurons=20, n_steps=90), 90)):
        say(f"case noalloc solver={solver} N={prob['n_comp'].shape[0]} steps={steps}")
        with S.Simulation(prob, **kw) as a:
            say("  config:", a.config)
            assert n_global(a.config) > 0
            a.step(steps)
            va, sa = a.voltages(), a.spikes()
        with S.Simulation(prob, **kw) as b:
            sb = b.step_noalloc(steps)
            vb = b.voltages()
            assert b.step_count == steps
            assert b.spikes().shape[0] == 0  # the call's spikes went to its buffer
        say(f"  spikes {len(sa)} vs {len(sb)}, max|dV| {np.abs(va - vb).max():.3e}")
        assert np.array_equal(va, vb)
        assert np.array_equal(sa, sb)
        assert len(sa) > 0


def test_noalloc_continues_a_simulation(S):
    prob = W.mini(seed=13, n_neurons=32, n_steps=170)
    kw = dict(solver=1, pack_comps=600, lds_comps=120, lds_classes=1)
    with S.Simulation(prob, **kw) as a:
        a.step(170)
        va, sa = a.voltages(), a.spikes()
    with S.Simulation(prob, **kw) as b:
        b.step(50)                  # graph-replayed and direct epochs first
        s1 = b.spikes()
        s2 = b.step_noalloc(77)     # then allocation-free, ending mid-epoch
        s3 = b.step_noalloc(43)
        vb = b.voltages()
    sb = np.concatenate([s1, s2, s3])
    assert np.array_equal(va, vb)
    assert np.array_equal(sa, sb)


def test_noalloc_reports_a_short_buffer(S):
    prob = W.mini(seed=11, n_neurons=48, n_steps=200)
    with S.Simulation(prob, solver=1) as g:
        with pytest.raises(S.SimError) as e:
            g.step_noalloc(200, cap=1)
        assert e.value.code == S.SIM_ENOMEM
        assert g.step_count == 200
