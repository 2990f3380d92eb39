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

from . import costmodel
from . import sim as S
from . import workload as W


def _time(prob: dict, packing: int, steps: int, warmup: int, solver: int,
          cost_model=None) -> dict:
    g = S.Simulation(prob, packing=packing, solver=solver, cost_model=cost_model)
    try:
        g.step(warmup)
        g.set_kernel_timing(True)
        g.step(steps)
        ms, epochs = g.kernel_time()
        config = g.config
    finally:
        g.close()
    C = int(prob["comp_off"][-1])
    return dict(ms_per_step=ms / steps, ns_per_update=ms * 1e6 / (C * steps),
                compartments=C, epochs=epochs, launch=config)


def imbalance(n_neurons: int = 10000, steps: int = 400, warmup: int = 40, seed: int = 7,
              solver: int = S.SOLVE_FAST) -> dict:
    """Mono vs multi-morphology under plain, count and learned packing."""
    mono = W.size_group(seed, n_neurons, mono=True)
    multi = W.size_group(seed, n_neurons, mono=False)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--neurons", type=int, default=10000)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--solver", default="fast", choices=["exact", "fast", "contract"])
    args = ap.parse_args()
    solver = dict(exact=S.SOLVE_EXACT, fast=S.SOLVE_FAST, contract=S.SOLVE_CONTRACT)[args.solver]
    out = imbalance(args.neurons, args.steps, args.warmup, solver=solver)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
