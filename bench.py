"""Benchmark: compartment-updates/s of the multi-morphology network on one GPU.

  python bench.py [--steps K] [--warmup W] [--workload cfg3] [--packing count]

One step = one time step dt of the whole network (every compartment of every
neuron advanced once: delivery, gating, assembly, Hines solve, detection).
Inputs are generated and copied to the GPU before the timed region; the timed
region covers exactly K steps bracketed by device synchronisation and HIP
events on the simulator's stream. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2005_06332_amd import workload as W  # noqa: E402

PEAK_HBM_GBS = 8000.0
# Non-packed vector FMA rate: 256 CUs x 64 lanes x 2 flop x 2.4 GHz. Packed
# FP32 is not used, so float and double arithmetic share this peak.
PEAK_VALU_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12

# Algorithmic bytes per compartment-update of a per-step streaming update
# (state V f64 read+write 16 B, gates read+write 24 B in FP32 / 48 B in FP64,
# per-compartment constants 24 B when morphologies differ, synaptic
# conductance read+write per synapse).
def bytes_per_update(precision: int, multi: bool, syn_per_comp: float) -> float:
    gates = 24.0 if precision == 1 else 48.0
    const = 24.0 if multi else 0.0
    g = syn_per_comp * (8.0 if precision == 1 else 16.0)
    return 16.0 + gates + const + g


# Floating-point operations per compartment-update as the path evaluates them
# (each exp is a Cody-Waite reduction plus a Taylor polynomial: 1 mul, 2 fma,
# 7 fma in float / 13 in double, 1 scaling mul; fma = 2 flops).
def flops_per_update(precision: int) -> float:
    exp_f = 1 + 4 + (14 if precision == 1 else 26) + 1
    rates = 6 * 2 + 6 * exp_f + 2 + 4 + 1 + 1 + 1  # 6 rates: argument, exp, scaling
    gates = 3 * (exp_f + 6)
    current = 21
    assembly = 10
    sweep = 8
    return float(rates + gates + current + assembly + sweep)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in ("kernels.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_2005_06332_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def make_workload(name: str, neurons: int | None, precision: str | None = None):
    kw = {}
    if neurons:
        kw["n_neurons"] = neurons
    if precision:
        kw["precision"] = 0 if precision == "fp64" else 1
    cfg = int(name.replace("cfg", ""))
    prob = W.make(cfg, **kw)
    return prob


def describe(prob: dict) -> str:
    n = prob["n_comp"]
    return (f"{prob['name']}: {n.shape[0]} multi-morphology neurons, compartments log-normal "
            f"(median {int(np.median(n))}, max {n.max()}), {int(prob['comp_off'][-1])} "
            f"compartments, {prob['syn_pre'].shape[0]} synapses, HH everywhere, "
            f"dt {prob['params']['dt']} ms")


def time_run(S, prob, steps, warmup, packing, cost_model=None, autotune=True, stream=None,
             solver=1):
    import torch
    g = S.Simulation(prob, packing=packing, autotune=autotune, cost_model=cost_model,
                     stream=stream.cuda_stream if stream is not None else None, solver=solver)
    torch.cuda.synchronize()
    if warmup:
        g.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # launch timing on: whole epochs replay from the captured graphs, with HIP
    # events around each replay on the simulator's stream, and each
    # size-class launch timing its own span on the device
    g.set_kernel_timing(True)
    with torch.cuda.stream(stream):
        ev0.record(stream)
        g.step(steps)
        ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    return g, ms


def cpu_baseline(prob: dict, target_s: float = 15.0):
    """The oracle on a bounded sample of the same workload: the first neurons
    of the network (with the synapses among them) for a short run."""
    from oracle import oracle as O
    O.build(force=False)
    n_all = prob["n_comp"].shape[0]
    # calibrate the sample size with a small probe
    probe = W.subset(prob, np.arange(min(256, n_all)))
    t0 = time.perf_counter()
    s = O.Sim(probe, max_steps=40)
    s.step(40)
    s.close()
    dt = time.perf_counter() - t0
    rate = probe["comp_off"][-1] * 40 / max(dt, 1e-6)
    steps = 80
    want = rate * target_s / steps
    mean_n = float(prob["comp_off"][-1]) / n_all
    nn = int(min(n_all, max(256, want / mean_n)))
    if nn == n_all:  # the whole network fits the budget: run it longer
        steps = int(min(4000, max(80, rate * target_s / float(prob["comp_off"][-1]))))
    sample = W.subset(prob, np.arange(nn))
    t0 = time.perf_counter()
    s = O.Sim(sample, max_steps=steps)
    s.step(steps)
    s.close()
    el = time.perf_counter() - t0
    upd = float(sample["comp_off"][-1]) * steps
    return dict(value=upd / el, unit="compartment-updates/s", cores=O.num_threads(),
                kind="oracle",
                sample=f"first {nn} neurons of {prob['name']} ({int(sample['comp_off'][-1])} "
                       f"compartments, synapses among them), {steps} steps, {el:.1f} s, "
                       f"precision mode {prob['params']['precision']}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--neurons", type=int, default=0)
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32"],
                    help="override the workload's precision (fp32 = FP32 gating, FP64 Hines)")
    ap.add_argument("--packing", default="count", choices=["plain", "count", "learned"])
    ap.add_argument("--solver", default="fast", choices=["exact", "fast"],
                    help="exact: the elimination in the reference operation order (bitwise "
                         "equal to the CPU oracle); fast: division-free homogeneous form")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-packing comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed run, copy 1 GiB with a plain copy kernel (reference "
                         "for the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: sharding the network over several GPUs "
              "(one RCCL allgather of spike bits per epoch) is designed but not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_06332_amd import sim as S, costmodel

    prob = make_workload(args.workload, args.neurons or None, args.precision)
    C = int(prob["comp_off"][-1])
    N = int(prob["n_comp"].shape[0])
    prec = int(prob["params"]["precision"])
    multi = len(np.unique(prob["n_comp"])) > 1
    stream = torch.cuda.Stream()

    cost_model = None
    packing = dict(plain=S.PACK_PLAIN, count=S.PACK_COUNT, learned=S.PACK_LEARNED)[args.packing]
    if packing == S.PACK_LEARNED:
        cost_model = costmodel.load_or_train(prob)

    solver = S.SOLVE_FAST if args.solver == "fast" else S.SOLVE_EXACT
    g, ms = time_run(S, prob, args.steps, args.warmup, packing, cost_model,
                     autotune=not args.no_autotune, stream=stream, solver=solver)
    config_str = g.config
    E = int(config_str.split("E=")[1].split()[0])
    # the dominant kernel: the launch of size class 0 (most packs), its
    # duration over the timed region from its own device-side span
    cls = [g.class_time(c) for c in range(3)]
    epoch_ms, epochs = g.kernel_time()
    g.close()
    upd = float(C) * args.steps
    value = upd / (ms / 1e3)
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    plain = None
    if not args.no_plain and packing != S.PACK_PLAIN:
        gp, msp = time_run(S, prob, args.steps, args.warmup, S.PACK_PLAIN, autotune=False,
                           stream=stream, solver=solver)
        gp.close()
        plain = upd / (msp / 1e3)

    syn_per_comp = prob["syn_pre"].shape[0] / C
    b_alg = bytes_per_update(prec, multi, syn_per_comp)
    k_ms, k_n, k_comps = cls[0]
    kernel_ms = k_ms / max(k_n, 1)
    upd_per_launch = float(k_comps) * E
    achieved_gbs = b_alg * upd_per_launch / (kernel_ms / 1e3) / 1e9
    flops = flops_per_update(prec)
    achieved_tf = flops * upd_per_launch / (kernel_ms / 1e3) / 1e12

    # HBM bytes per launch measured with rocprofv3 counters on this kernel
    # source (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known
    # size); reported only while the kernel source is unchanged.
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{prob['name']}.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            rec = json.load(f)
        if rec.get("kernel_source_sha1") == kernel_source_hash():
            traffic = rec.get("bytes_per_launch")

    out = {
        "metric": "compartment-updates/s at 1 GPU (multi-morphology)",
        "value": value,
        "unit": "compartment-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 gating + f64 Hines" if prec == 1 else "f64",
        "data": "synthetic",
        "config": {
            "workload": describe(prob),
            "neurons": N, "compartments": C, "synapses": int(prob["syn_pre"].shape[0]),
            "precision": "fp32-gating/fp64-hines" if prec == 1 else "fp64",
            "packing": args.packing, "solver": args.solver, "launch": config_str,
            "plain_packing_value": plain,
            "speedup_vs_plain_packing": (value / plain) if plain else None,
            "hbm_roofline_frac_streaming": value * b_alg / (PEAK_HBM_GBS * 1e9),
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tf,
            "peak": PEAK_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tf / PEAK_VALU_TFLOPS,
            "traffic": traffic,
            "kernel": "k_epoch, size class 0 launch",
            "kernel_ms": kernel_ms,
            "kernel_launches": k_n,
            "compartments_per_launch_step": k_comps,
            "updates_per_launch": upd_per_launch,
            "epoch_ms": epoch_ms / max(epochs, 1),
            "class_ms": [c[0] / max(c[1], 1) for c in cls],
            "class_compartments": [c[2] for c in cls],
            "flops_per_update": flops,
            "streaming_bytes_per_update": b_alg,
            "streaming_hbm_GBps": achieved_gbs,
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
