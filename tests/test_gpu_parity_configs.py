"""GPU parity at full size for the remaining workload variants, and the error
of FP32 gating against the FP64 oracle per workload.

- cfg2 (8192 identical neurons of 1000 compartments) with FP32 gating and
  FP64 Hines, all three solvers, every voltage and spike after 80 steps.
- cfg4 (32768 multi-morphology neurons) with learned packing (the MLP cost
  model trained on kernel timings), all three solvers, every voltage and
  spike after 80 steps.
- Full-length per-neuron replay: the GPU runs a whole network for 4000 steps
  in the configuration bench.py times (contraction solver, FP32 gating); 34 of its
  neurons (32 drawn with a fixed seed, the largest and the smallest) are
  rerun in the oracle fed with the GPU's recorded presynaptic spikes:
    * in the FP32-gating oracle: voltages within 1e-4 mV, identical spikes;
    * in the FP64 oracle: the error of FP32 gating itself. Reported per
      workload: max|dV| at the end, and the crossing margins of the FP64
      run, min |V_det - theta_s| over the two voltages of every upward
      threshold crossing and over every step. Identical spikes are asserted
      wherever the FP64 run's voltage stays further from the threshold than
      the stated bound of 0.5 mV; a spike that differs must sit within it.
- cfg5 (1e5 neurons, delays 40..200 steps) replayed over 480 steps with the
  exact solver, so that every delay class delivers at full size.
"""
import sys

import numpy as np
import pytest

from paper_2005_06332_amd import workload as W

pytestmark = pytest.mark.gpu

TOL_MV = 1e-9
TOL_FAST_FP32_MV = 1e-4
# End-state error of FP32 gating against the FP64 oracle after a full run:
# the gates' float rounding (relative 6e-8 per step) shifts spike timing by
# well under a microsecond over 100 ms, and a neuron caught on an action
# potential's upstroke (up to about 500 mV/ms) turns a shift of 1 us into
# 0.5 mV. (cfg2 measured 0.086 mV with every spike identical.)
FP32_VS_FP64_BOUND_MV = 0.5


def tol(precision, solver):
    return TOL_FAST_FP32_MV if (solver != 0 and precision == 1) else TOL_MV


@pytest.fixture(scope="module")
def S():
    from paper_2005_06332_amd import sim
    sim.lib()
    return sim


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(tag, v_gpu, v_ref, s_gpu, s_ref, tol_mv):
    d = np.abs(v_gpu - v_ref)
    say(f"{tag}: max|dV|={d.max():.3e} mV, differing={int(np.count_nonzero(d))}/{d.size}, "
        f"spikes gpu={len(s_gpu)} ref={len(s_ref)}")
    assert np.all(np.isfinite(v_gpu))
    assert d.max() <= tol_mv, tag
    assert s_gpu.shape == s_ref.shape and np.array_equal(s_gpu, s_ref), tag


def full_pair(S, full_workload, oracle_full, cfg, steps, precision, **kw):
    """The GPU run of a full-size workload and the oracle's run of it (shared
    by every variant of one workload, step count and precision)."""
    prob = full_workload(cfg)
    say(f"case {prob['name']} N={prob['n_comp'].shape[0]} C={int(prob['comp_off'][-1])} "
        f"steps={steps} prec={precision} {sorted(k for k in kw if k != 'cost_model')}")
    with S.Simulation(prob, precision=precision, **kw) as g:
        say("  config:", g.config)
        g.step(steps)
        v, s = g.voltages(), g.spikes()
    vr, sr = oracle_full(cfg, steps, precision)
    return v, s, vr, sr


@pytest.mark.parametrize("solver", [0, 1, 2])
def test_cfg2_fp32_gating_full_size(S, full_workload, oracle_full, solver):
    v, s, vr, sr = full_pair(S, full_workload, oracle_full, 2, 80, 1, solver=solver,
                             autotune=(solver != 0))
    compare(f"full cfg2 FP32 gating solver={solver}", v, vr, s, sr, tol(1, solver))


@pytest.fixture(scope="module")
def cost_model(S):
    from paper_2005_06332_amd import costmodel
    return costmodel.load_or_train()


@pytest.mark.parametrize("solver", [0, 1, 2])
def test_cfg4_learned_packing_full_size(S, full_workload, oracle_full, cost_model, solver):
    v, s, vr, sr = full_pair(S, full_workload, oracle_full, 4, 80, 1, solver=solver,
                             packing=S.PACK_LEARNED, cost_model=cost_model)
    compare(f"full cfg4 learned packing solver={solver}", v, vr, s, sr, tol(1, solver))
    assert len(sr) > 1000


def replay_targets(prob, n=32, seed=7):
    N = prob["n_comp"].shape[0]
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.choice(N, n, replace=False),
                                     [int(np.argmax(prob["n_comp"])),
                                      int(np.argmin(prob["n_comp"]))]]))


def gpu_spikes_of(s, targets):
    pos = {int(j): k for k, j in enumerate(targets)}
    return np.array(sorted((pos[int(n)], int(t)) for n, t in s if int(n) in pos),
                    np.int64).reshape(-1, 2)


def replay(orc, prob, targets, raster, steps, precision, track=False):
    """The target neurons rerun in the oracle from the recorded raster.
    Returns (V, spikes [(target index, step)], detector voltages
    [(steps+1), targets] when tracked)."""
    sub = W.replay_subset(prob, targets)
    rep = orc.Sim(sub, max_steps=steps, precision=precision)
    rep.set_input_raster(raster)
    vdet = None
    if track:
        det = sub["comp_off"][:-1] + sub["detector"]
        vdet = np.empty((steps + 1, len(targets)))
        vdet[0] = rep.voltages()[det]
        for n in range(steps):
            rep.step(1)
            vdet[n + 1] = rep.voltages()[det]
    else:
        rep.step(steps)
    v, sp = rep.voltages(), rep.spikes()
    rep.close()
    return v, np.array(sorted(map(tuple, sp.tolist())), np.int64).reshape(-1, 2), vdet


def crossing_margins(vdet, thr):
    """min(thr - V^n, V^{n+1} - thr) over every upward crossing
    V^n < thr <= V^{n+1} of every target, and min |V - thr| over all steps."""
    a, b = vdet[:-1], vdet[1:]
    up = (a < thr) & (b >= thr)
    m = np.minimum(thr - a, b - thr)[up]
    return (float(m.min()) if m.size else float("inf"), int(up.sum()),
            float(np.abs(vdet - thr).min()))


def fp32_error_report(S, orc, name, prob, steps=4000, **kw):
    targets = replay_targets(prob)
    N = prob["n_comp"].shape[0]
    say(f"case {name} full-length replay steps={steps} targets={len(targets)}")
    with S.Simulation(prob, precision=1, solver=2, **kw) as g:
        say("  config:", g.config)
        g.step(steps)
        v, s = g.voltages(), g.spikes()
    raster = W.spike_raster(s, N, steps)
    off = prob["comp_off"]
    want = np.concatenate([v[off[j]:off[j + 1]] for j in targets])
    gsp = gpu_spikes_of(s, targets)
    # FP32-gating oracle: parity
    v32, sp32, _ = replay(orc, prob, targets, raster, steps, 1)
    compare(f"{name} replay contract vs FP32-gating oracle", want, v32, gsp, sp32,
            TOL_FAST_FP32_MV)
    # FP64 oracle: the error of FP32 gating
    v64, sp64, vdet = replay(orc, prob, targets, raster, steps, 0, track=True)
    thr = prob["params"]["v_thresh"]
    cmin, ncross, gmin = crossing_margins(vdet, thr)
    sub_off = W.replay_subset(prob, targets)["comp_off"]
    same, worst = [], 0.0
    for k in range(len(targets)):
        a = gsp[gsp[:, 0] == k][:, 1]
        b = sp64[sp64[:, 0] == k][:, 1]
        if a.shape == b.shape and np.array_equal(a, b):
            same.append(k)
            worst = max(worst, float(np.abs(want[sub_off[k]:sub_off[k + 1]]
                                            - v64[sub_off[k]:sub_off[k + 1]]).max()))
        else:
            # a differing spike train: the FP64 run must have come within the
            # stated bound of the threshold at the first differing step
            diff = np.setxor1d(a, b)
            n0 = int(diff.min())
            near = np.abs(vdet[max(n0 - 1, 0):n0 + 1, k] - thr).min()
            say(f"  target {k}: spikes differ first at step {n0}, FP64 |V-thr| there "
                f"{near:.3e} mV")
            assert near <= FP32_VS_FP64_BOUND_MV
    say(f"P11 {name}: FP32 gating vs FP64 oracle over {steps} steps, {len(targets)} neurons: "
        f"max|dV| {worst:.3e} mV (neurons with identical spikes: {len(same)}/{len(targets)}), "
        f"{ncross} crossings, min crossing margin {cmin:.3e} mV, min |V-thr| {gmin:.3e} mV")
    assert worst <= FP32_VS_FP64_BOUND_MV
    if gmin > FP32_VS_FP64_BOUND_MV:
        assert len(same) == len(targets)
    assert len(s) > 1000
    return worst, cmin, gmin


def test_fp32_error_cfg2_full_length(S, orc, full_workload):
    fp32_error_report(S, orc, "cfg2", full_workload(2, precision=1), autotune=True)


def test_fp32_error_cfg4_full_length(S, orc, full_workload, cost_model):
    fp32_error_report(S, orc, "cfg4", full_workload(4), packing=S.PACK_LEARNED,
                      cost_model=cost_model)


def test_fp32_error_cfg5_full_length(S, orc, full_workload):
    """cfg5 over 4000 steps (every delay class 40..200 steps delivers many
    times), default layout with its largest neurons in global scratch."""
    fp32_error_report(S, orc, "cfg5", full_workload(5))


def test_cfg5_exact_replay_delivers_every_delay(S, orc, full_workload):
    """cfg5 with the exact solver over 480 steps (12 epochs, so delays of up to
    200 steps deliver at full size), replayed per neuron: bitwise in
    practice, 1e-9 mV stated."""
    prob = full_workload(5)
    steps = 480
    N = prob["n_comp"].shape[0]
    targets = replay_targets(prob)
    with S.Simulation(prob, solver=0) as g:
        say("  config:", g.config)
        g.step(steps)
        v, s = g.voltages(), g.spikes()
    raster = W.spike_raster(s, N, steps)
    off = prob["comp_off"]
    want = np.concatenate([v[off[j]:off[j + 1]] for j in targets])
    vr, sr, _ = replay(orc, prob, targets, raster, steps, 1)
    compare("cfg5 exact replay 480 steps", want, vr, gpu_spikes_of(s, targets), sr, TOL_MV)
    # events did arrive through the longest delays: spikes of steps >= 200
    # exist and fed the targets' synapses
    rp = W.replay_subset(prob, targets)
    assert rp["syn_delay"].max() >= 190 and len(s) > 1000


def test_fp32_error_cfg3_full_length(S, orc):
    fp32_error_report(S, orc, "cfg3", W.make(3), autotune=True)
