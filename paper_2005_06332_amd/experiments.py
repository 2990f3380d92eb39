"""The paper's multi-morphology load-balance experiment on one GPU.

Section 4 of the paper simulates 10,000 neurons whose sizes come from a group
of 20 randomly sized neurons (largest minus smallest: 700) and compares them
with a mono-morphology run of the same number of neurons; on the CPU cluster
the size mix costs about 12 % extra time, and scheduling large neurons first
(task priorities, then an initial sort by size) brings it down to about 3 %.

Here the same two networks (workload.size_group) run through the library
with plain packing (generation order), compartment-count packing (sort by
size, the analogue of the paper's sorting) and learned packing (the MLP cost
model). Time is the device time of whole epochs (HIP events); it is reported
per compartment-update so that the two networks, whose compartment totals
differ slightly, compare directly.

  python -m paper_2005_06332_amd.experiments [--steps 400] [--neurons 10000]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import costmodel
from . import sim as S
from . import workload as W


def _time(prob: dict, packing: int, steps: int, warmup: int, solver: int,
          cost_model=None, neuron_cost=None) -> dict:
    g = S.Simulation(prob, packing=packing, solver=solver, cost_model=cost_model,
                     neuron_cost=neuron_cost)
    try:
        g.step(warmup)
        g.set_kernel_timing(True)
        g.step(steps)
        ms, epochs = g.kernel_time()
        config = g.config
    finally:
        g.close()
    C = int(prob["comp_off"][-1])
    out = dict(ms_per_step=ms / steps, ns_per_update=ms * 1e6 / (C * steps),
               compartments=C, epochs=epochs, launch=config)
    print(f"experiments: {prob['name']} packing={packing} "
          f"{out['ns_per_update']:.5f} ns per update", file=sys.stderr, flush=True)
    return out


def imbalance(n_neurons: int = 10000, steps: int = 400, warmup: int = 40, seed: int = 7,
              solver: int = S.SOLVE_FAST) -> dict:
    """Mono vs multi-morphology under plain, count and learned packing."""
    mono = W.size_group(seed, n_neurons, mono=True)
    multi = W.size_group(seed, n_neurons, mono=False)
    print("experiments: cost model", file=sys.stderr, flush=True)
    model = costmodel.load_or_train(solver=solver)
    runs = {
        "mono_plain": _time(mono, S.PACK_PLAIN, steps, warmup, solver),
        "mono_count": _time(mono, S.PACK_COUNT, steps, warmup, solver),
        "multi_plain": _time(multi, S.PACK_PLAIN, steps, warmup, solver),
        "multi_count": _time(multi, S.PACK_COUNT, steps, warmup, solver),
        "multi_learned": _time(multi, S.PACK_LEARNED, steps, warmup, solver, model),
    }
    for base in ("mono_plain", "mono_count"):
        b = runs[base]["ns_per_update"]
        for r in runs.values():
            r[f"extra_vs_{base}"] = r["ns_per_update"] / b - 1.0
    sizes = multi["n_comp"]
    return dict(experiment="mono vs multi-morphology (paper Section 4)", neurons=n_neurons,
                steps=steps, group_sizes=sorted(set(int(x) for x in sizes)),
                group_mean=float(sizes.mean()), mono_size=int(mono["n_comp"][0]),
                compartments=dict(mono=int(mono["comp_off"][-1]),
                                  multi=int(multi["comp_off"][-1])),
                runs=runs)


def measured_pack_costs(prob: dict, steps: int, solver: int) -> np.ndarray:
    """Per neuron: the measured kernel time of its pack under count packing
    (the pack's summed per-neuron times from the in-kernel recorder)."""
    with S.Simulation(prob, packing=S.PACK_COUNT, solver=solver, record_timings=True) as g:
        E = int(g.config.split("E=")[1].split()[0])
        g.step(E)
        g.neuron_timings(reset=True)
        g.step(steps)
        t = g.neuron_timings()
        cost = np.empty(prob["n_comp"].shape[0])
        for p in range(g.pack_count()):
            ids = g.pack_neurons(p)
            cost[ids] = t[ids].sum()
    return np.maximum(cost, 1e-9)


def packing_bound(prob: dict, steps: int = 400, warmup: int = 40, reps: int = 3,
                  solver: int = S.SOLVE_CONTRACT) -> dict:
    """Count packing against learned packing, with the cost model's
    predictions and with the measured time of each neuron's pack under count
    packing as the neuron's cost. Learned packing forms the same best-fit
    packs and dispatches them in decreasing cost, so the measured costs give
    the dispatch order that the packs' real times call for: what no
    prediction from neuron features can improve on. Runs alternate, reps
    times each."""
    print("experiments: cost model", file=sys.stderr, flush=True)
    model = costmodel.load_or_train(solver=solver)
    print("experiments: measured pack times", file=sys.stderr, flush=True)
    measured = measured_pack_costs(prob, steps, solver)
    runs = {"count": [], "learned (model)": [], "learned (measured pack times)": []}
    for _ in range(reps):
        runs["count"].append(_time(prob, S.PACK_COUNT, steps, warmup, solver))
        runs["learned (model)"].append(_time(prob, S.PACK_LEARNED, steps, warmup, solver, model))
        runs["learned (measured pack times)"].append(
            _time(prob, S.PACK_LEARNED, steps, warmup, solver, neuron_cost=measured))
    out = {k: dict(ns_per_update=[r["ns_per_update"] for r in v], launch=v[0]["launch"])
           for k, v in runs.items()}
    base = np.mean(out["count"]["ns_per_update"])
    for v in out.values():
        v["mean_vs_count"] = float(np.mean(v["ns_per_update"]) / base - 1.0)
    return dict(experiment="count vs learned packing, with a bound from measured pack times",
                workload=prob["name"], steps=steps, reps=reps, runs=out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--neurons", type=int, default=10000)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--solver", default="fast", choices=["exact", "fast", "contract"])
    ap.add_argument("--bound", default=None, help="workload (cfgN): count vs learned packing "
                    "and the measured-pack-time bound instead of the Section 4 experiment")
    args = ap.parse_args()
    solver = dict(exact=S.SOLVE_EXACT, fast=S.SOLVE_FAST, contract=S.SOLVE_CONTRACT)[args.solver]
    if args.bound:
        out = packing_bound(W.make(int(args.bound.replace("cfg", ""))), args.steps, args.warmup,
                            solver=solver)
    else:
        out = imbalance(args.neurons, args.steps, args.warmup, solver=solver)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
