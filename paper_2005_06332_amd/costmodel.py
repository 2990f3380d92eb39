"""Learned cost model for neuron-to-workgroup packing.

The simulator records, in the epoch kernel itself, the wall-clock time each
pack takes. A calibration run gives every neuron its own pack, so each
neuron's time is measured in isolation; the 16 morphology features of the
library (compartments, branches, levels, critical path, serial sweep
lengths, synapses, ...) and log(time) then train the 16-64-64-1 MLP with the
library's GPU kernels (forward, backward, Adam). The trained parameters drive
SIM_PACK_LEARNED; the compartment count (SIM_PACK_COUNT) is the fallback and
the yardstick. The model changes which workgroup runs which neuron and in
what order, never what is computed.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

from . import sim as S
from . import workload as W


def calibrate(prob: dict, epochs: int = 2, threads: int = 256, solver: int = S.SOLVE_EXACT):
    """Per-neuron kernel time (ns per epoch) with one neuron per pack, under
    the tree solver the packing is for (a neuron's cost depends on it: serial
    sweeps for the exact solver, level counts for the fast one, contraction
    rounds for the contraction solver).
    Returns (features [N,16] float32, log time [N] float32)."""
    with S.Simulation(prob, packing=S.PACK_COUNT, sched=S.SCHED_PERSISTENT, pack_comps=1,
                      threads=threads, record_timings=True, autotune=False,
                      use_graph=False, solver=solver) as g:
        E = int(g.config.split("E=")[1].split()[0])
        g.step(E)
        g.neuron_timings(reset=True)
        g.step(epochs * E)
        t = g.neuron_timings() / epochs
        f = g.features()
    return f, np.log(np.maximum(t, 1.0)).astype(np.float32)


def train(features: np.ndarray, log_t: np.ndarray, epochs: int = 3000, lr: float = 3e-3,
          seed: int = 1234):
    p = S.mlp_init(features, log_t, seed)
    p, loss = S.mlp_train(p, features, log_t, epochs, lr)
    return p, loss


def fit_quality(params: np.ndarray, features: np.ndarray, log_t: np.ndarray) -> dict:
    pred = S.mlp_forward(params, features)
    t = np.exp(log_t)
    r = np.corrcoef(pred, log_t)[0, 1]
    n = features[:, 0]
    rc = np.corrcoef(np.log(n), log_t)[0, 1]
    return dict(r_log_mlp=float(r), r_log_count=float(rc),
                mape_mlp=float(np.mean(np.abs(np.exp(pred) - t) / t)))


def load_or_train(prob_like: dict | None = None, n_neurons: int = 4096,
                  cache_dir: str | None = None, solver: int = S.SOLVE_EXACT):
    """Parameters trained on a calibration run of the 16384-neuron
    multi-morphology recipe (seed 3, first n_neurons neurons) under the given
    tree solver, cached per solver."""
    cache_dir = cache_dir or os.environ.get("MMHINES_CACHE", "/tmp/mmhines_cache")
    key = hashlib.sha1(repr(("cm", 3, n_neurons, 1, int(solver))).encode()).hexdigest()[:12]
    path = os.path.join(cache_dir, f"costmodel_{key}.npy")
    if os.path.exists(path):
        return np.load(path)
    calib = W.make(3)
    calib = W.subset(calib, np.arange(min(n_neurons, calib["n_comp"].shape[0])))
    f, y = calibrate(calib, solver=solver)
    p, _ = train(f, y)
    try:
        os.makedirs(cache_dir, exist_ok=True)
        np.save(path, p)
    except OSError:
        pass
    return p
