"""The seeded synthetic workloads: structure, recipe and determinism.

These arrays are the only inputs of both the GPU library and the oracle, so
a change in them changes every benchmark and parity case. The tests check
that every problem is a valid set of Hines trees with valid synapses, that
the generated statistics follow the stated recipe (log-normal compartment
counts, tapering diameters, fixed soma, branch counts), and that the
benchmark network is exactly the one measured (its size is pinned).
"""
import numpy as np
import pytest

from paper_2005_06332_amd import workload as W


def neuron_of(prob):
    off = prob["comp_off"]
    return np.repeat(np.arange(off.shape[0] - 1), np.diff(off))


def check_valid(prob):
    off, par = prob["comp_off"], prob["parent"]
    n_comp = prob["n_comp"]
    N, C = n_comp.shape[0], int(off[-1])
    assert off[0] == 0 and np.all(np.diff(off) == n_comp) and np.all(n_comp >= 1)
    for k in ("parent", "length_um", "diam_um", "mech"):
        assert prob[k].shape[0] == C, k
    nid = neuron_of(prob)
    local = np.arange(C) - off[nid]
    root = local == 0
    # Hines numbering: a root per neuron, every other parent earlier in the neuron
    assert np.all(par[root] == -1)
    assert np.all((par[~root] >= 0) & (par[~root] < local[~root]))
    assert np.all(np.isfinite(prob["length_um"])) and np.all(prob["length_um"] > 0)
    assert np.all(np.isfinite(prob["diam_um"])) and np.all(prob["diam_um"] > 0)
    assert prob["detector"].shape[0] == N and np.all(prob["detector"] < n_comp)
    assert prob["iext_nA"].shape[0] == N and np.all(prob["iext_nA"] >= 0)
    S = prob["syn_pre"].shape[0]
    for k in ("syn_post", "syn_comp", "syn_delay", "syn_w"):
        assert prob[k].shape[0] == S, k
    assert np.all((prob["syn_pre"] >= 0) & (prob["syn_pre"] < N))
    assert np.all((prob["syn_post"] >= 0) & (prob["syn_post"] < N))
    assert np.all((prob["syn_comp"] >= 0) & (prob["syn_comp"] < n_comp[prob["syn_post"]]))
    assert np.all(prob["syn_delay"] >= 1) and np.all(prob["syn_w"] >= 0)
    return nid, local


def branch_counts(prob, nid, local):
    """Branches per neuron: compartments whose parent is the soma or a fork."""
    off, par = prob["comp_off"], prob["parent"]
    C = int(off[-1])
    glob_par = np.where(par >= 0, off[nid] + par, -1)
    kids = np.bincount(glob_par[glob_par >= 0], minlength=C)
    starts = (par >= 0) & ((par == 0) | (kids[np.maximum(glob_par, 0)] >= 2))
    return np.bincount(nid[starts], minlength=off.shape[0] - 1)


@pytest.mark.parametrize("cfg", [1, 2, 3, "mini"])
def test_problems_are_valid_hines_networks(cfg):
    prob = W.mini() if cfg == "mini" else W.make(cfg)
    check_valid(prob)


def test_benchmark_network_is_pinned_and_follows_its_recipe():
    prob = W.make(3)
    nid, local = check_valid(prob)
    n = prob["n_comp"]
    # the measured network, exactly
    assert n.shape[0] == 16384 and int(prob["comp_off"][-1]) == 9293129
    assert prob["syn_pre"].shape[0] == 100 * 16384
    assert prob["params"]["precision"] == 1
    # log-normal counts, median 500, sigma 0.5 in log space, clipped to [50, 8000]
    assert 480 <= np.median(n) <= 520
    assert n.min() >= 50 and n.max() <= 8000
    assert abs(np.std(np.log(n)) - 0.5) < 0.02
    # a 20 um x 20 um soma at compartment 0, 10 um dendritic compartments
    soma = local == 0
    assert np.all(prob["length_um"][soma] == 20.0) and np.all(prob["diam_um"][soma] == 20.0)
    assert np.all(prob["length_um"][~soma] == 10.0)
    assert prob["diam_um"][~soma].min() >= 0.5 and prob["diam_um"][~soma].max() <= 3.0
    # HH everywhere; one synapse count and delay for all
    assert np.all(prob["mech"] == 1)
    assert np.all(np.bincount(prob["syn_post"], minlength=16384) == 100)
    assert np.all(prob["syn_delay"] == 40)
    # an even number of branches, at least 4, at most 256, at least 2 compartments each
    nb = branch_counts(prob, nid, local)
    assert np.all(nb % 2 == 0) and nb.min() >= 4 and nb.max() <= 256
    assert np.all(2 * nb <= n - 1)


def test_generation_is_deterministic_and_seeded():
    a, b = W.mini(seed=5), W.mini(seed=5)
    for k in ("comp_off", "parent", "length_um", "diam_um", "syn_pre", "syn_comp", "syn_w",
              "iext_nA"):
        assert np.array_equal(a[k], b[k]), k
    c = W.mini(seed=6)
    assert not (np.array_equal(a["comp_off"], c["comp_off"])
                and np.array_equal(a["syn_pre"], c["syn_pre"]))


def test_variable_delays_cover_their_range():
    prob = W.mini(seed=17, n_neurons=64, delay_lo=40, delay_hi=200)
    check_valid(prob)
    d = prob["syn_delay"]
    assert d.min() >= 40 and d.max() <= 200 and len(np.unique(d)) > 100


def test_subset_keeps_only_synapses_among_the_kept_neurons():
    prob = W.mini(seed=3, n_neurons=40)
    keep = np.array([0, 7, 8, 21, 39])
    sub = W.subset(prob, keep)
    check_valid(sub)
    assert np.array_equal(sub["n_comp"], prob["n_comp"][keep])
    kept = np.isin(prob["syn_pre"], keep) & np.isin(prob["syn_post"], keep)
    assert sub["syn_pre"].shape[0] == int(kept.sum())


def test_size_group_matches_the_section4_recipe():
    """The Section-4 group: 20 sizes, spread exactly 700, mean exactly 300,
    smallest at least 12; the multi-morphology network holds equally many
    copies of each member, so it has exactly the mono network's
    compartments."""
    for seed in range(7, 17):
        g = W.group_sizes(np.random.default_rng(seed))
        assert g.shape == (20,)
        assert g.max() - g.min() == 700
        assert g.sum() == 20 * 300
        assert g.min() >= 12
    multi = W.size_group(7, 2000)
    mono = W.size_group(7, 2000, mono=True)
    assert multi["comp_off"][-1] == mono["comp_off"][-1] == 2000 * 300
    sizes, counts = np.unique(multi["n_comp"], return_counts=True)
    assert sizes.max() - sizes.min() == 700
    assert abs(multi["n_comp"].mean() - 300.0) < 1e-12
    assert set(mono["n_comp"].tolist()) == {300}


def test_star_network_has_high_fanout_somata():
    prob = W.star_network()
    off = prob["comp_off"]
    for j in range(prob["n_comp"].shape[0]):
        p = prob["parent"][off[j]:off[j + 1]]
        assert p[0] == -1 and np.all(p[1:] < np.arange(1, p.shape[0]))
        assert int(np.sum(p == 0)) in (64, 5)


def test_shared_workloads_hand_out_isolated_read_only_problems(orc):
    """The GPU suite's session caches: one generation per workload, equal to a
    fresh one; every call a new dict whose params and channels are its own; the
    arrays read-only; and the shared oracle run equal to a direct one, made
    once per (workload, steps, precision)."""
    from conftest import SharedOracleRuns, SharedWorkloads
    fw = SharedWorkloads()
    a, b = fw(1), fw(1)
    fresh = W.make(1)
    assert a is not b and a["params"] is not b["params"] and a["channels"] is not b["channels"]
    for k, v in fresh.items():
        if isinstance(v, np.ndarray):
            assert a[k] is b[k] and np.array_equal(a[k], v) and not a[k].flags.writeable
            with pytest.raises(ValueError):
                a[k][...] = 0
        else:
            assert a[k] == v
    a["params"]["theta"] = 1.0
    assert fw(1)["params"]["theta"] == fresh["params"]["theta"]
    runs = SharedOracleRuns(orc, fw)
    v1, s1 = runs(1, 40, 1)
    v2, s2 = runs(1, 40, 1)
    assert v1 is v2 and s1 is s2 and not v1.flags.writeable
    ref = orc.Sim(fresh, max_steps=40, precision=1)
    ref.step(40)
    assert np.array_equal(v1, ref.voltages()) and np.array_equal(s1, ref.spikes())
    ref.close()
