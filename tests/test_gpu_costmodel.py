"""GPU tests of the cost model: the library's MLP kernels against the float64
reference, and the learned packing (results unchanged, predictions better
than the compartment count)."""
import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_2005_06332_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2005_06332_amd import sim
    sim.lib()
    return sim


def data(n=300, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 800, (n, M.F)).astype(np.float32)
    t = (0.8 * np.log1p(x[:, 0]) + 0.3 * np.log1p(x[:, 5]) + rng.normal(0, 0.05, n)).astype(np.float32)
    return x, t


def test_mlp_forward_matches_reference(S):
    x, t = data()
    p = M.init(x, t, seed=4).astype(np.float32)
    got = S.mlp_forward(p, x)
    ref, _ = M.forward(p.astype(np.float64), x.astype(np.float64))
    assert np.max(np.abs(got - ref)) <= 2e-5 * max(1.0, np.max(np.abs(ref)))


def test_mlp_gradient_matches_reference(S):
    x, t = data()
    p = M.init(x, t, seed=6).astype(np.float32)
    L, g = S.mlp_loss_grad(p, x, t)
    Lr, gr = M.loss_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    assert L == pytest.approx(Lr, rel=1e-4)
    scale = np.max(np.abs(gr))
    assert np.max(np.abs(g - gr)) <= 1e-4 * scale
    assert np.all(g[:M.OW1] == 0) and np.all(g[M.OYM:] == 0)


def test_mlp_training_matches_reference_adam(S):
    x, t = data(200, seed=2)
    p0 = M.init(x, t, seed=8).astype(np.float32)
    p_gpu, loss_gpu = S.mlp_train(p0, x, t, epochs=25, lr=2e-3)
    p_ref = M.adam(p0.astype(np.float64), x.astype(np.float64), t.astype(np.float64), 25, 2e-3)
    assert np.max(np.abs(p_gpu - p_ref)) <= 2e-4
    assert loss_gpu == pytest.approx(M.loss(p_ref, x.astype(np.float64), t.astype(np.float64)),
                                     rel=1e-3)


def test_mlp_init_standardisation(S):
    x, t = data(500, seed=3)
    p = S.mlp_init(x, t, seed=1)
    lx = np.log1p(x.astype(np.float64))
    assert np.allclose(p[M.OXM:M.OXS], lx.mean(0), rtol=1e-5)
    assert np.allclose(p[M.OXS:M.OW1], lx.std(0), rtol=1e-4)
    assert p[M.OYM] == pytest.approx(float(np.mean(t)), rel=1e-5)


def test_learned_packing_changes_no_result(S):
    from paper_2005_06332_amd import costmodel
    prob = W.mini(n_neurons=96, n_steps=160, seed=31)
    f, y = costmodel.calibrate(prob, epochs=1)
    p, _ = costmodel.train(f, y, epochs=200)
    outs = []
    for kw in (dict(packing=S.PACK_COUNT), dict(packing=S.PACK_LEARNED, cost_model=p)):
        with S.Simulation(prob, **kw) as g:
            g.step(160)
            outs.append((g.voltages(), g.spikes(), g.config))
    print(outs[1][2], flush=True)
    assert "learned" in outs[1][2]
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_cost_model_predicts_kernel_time_better_than_count(S):
    """Calibrate on 2048 neurons of the 16384-neuron recipe, train on half,
    evaluate on the held-out half: the MLP must explain the measured
    per-neuron time better than the compartment count does."""
    from paper_2005_06332_amd import costmodel
    prob = W.subset(W.make(3), np.arange(2048))
    f, y = costmodel.calibrate(prob, epochs=2)
    tr, te = np.arange(0, 2048, 2), np.arange(1, 2048, 2)
    p, loss = costmodel.train(f[tr], y[tr], epochs=3000)
    q = costmodel.fit_quality(p, f[te], y[te])
    print(f"held-out: r(log MLP, log t)={q['r_log_mlp']:.3f} "
          f"r(log count, log t)={q['r_log_count']:.3f} MAPE={q['mape_mlp']:.3f} "
          f"train loss={loss:.4f}", flush=True)
    assert q["r_log_mlp"] >= q["r_log_count"]
