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

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "compartment-updates/s at 1 GPU (multi-morphology) + % HBM roofline vs plain packing"

# Algorithmic bytes per compartment-update of a per-step streaming update
# (state V f64 read+write 16 B, gates read+write 24 B in FP32 / 48 B in FP64,
# per-compartment constants 24 B when morphologies differ, synaptic
# conductance read+write per synapse).
def bytes_per_update(precision: int, multi: bool, syn_per_comp: float) -> float:
    gates = 24.0 if precision == 1 else 48.0
    const = 24.0 if multi else 0.0
    g = syn_per_comp * (8.0 if precision == 1 else 16.0)
    return 16.0 + gates + const + g


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
             solver=1, lds_classes=0):
    import torch
    g = S.Simulation(prob, packing=packing, autotune=autotune, cost_model=cost_model,
                     stream=stream.cuda_stream if stream is not None else None, solver=solver,
                     lds_classes=lds_classes)
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


def host_info() -> dict:
    """CPU model, logical CPUs usable by this process and RAM of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    ram = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()
    return dict(host_cpu=model, host_logical_cpus=ncpu, host_ram_gib=ram)


def copy_bandwidth(stream) -> float:
    """HBM bandwidth of a plain device copy (1 GiB read + 1 GiB written), GB/s:
    the best of 5 timed copies after a warm-up copy."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = None
    with torch.cuda.stream(stream):
        b.copy_(a)
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.copy_(a)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.synchronize()
    return 2.0 * 4 * n / (best / 1e3) / 1e9


def cpu_baseline(prob: dict, target_s: float = 20.0):
    """The oracle on a bounded sample of the same workload: the first neurons
    of the network (with the synapses among them) for a short run, sized for
    about target_s seconds. The short probe that sizes it includes the
    oracle's set-up, so on many cores it underestimates the rate (by 42% on
    16 threads): a 20 s target keeps the run between 10 and 30 s either way."""
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
                kind="oracle", **host_info(),
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
    ap.add_argument("--solver", default="contract", choices=["exact", "fast", "contract"],
                    help="exact: the elimination in the reference operation order (bitwise "
                         "equal to the CPU oracle); fast: division-free homogeneous form; "
                         "contract: tree contraction")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-packing comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--lds-classes", type=int, default=0,
                    help="fix the number of LDS size classes (1..3) instead of autotuning the "
                         "layout (the counter runs use it to reproduce the benchmarked layout)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed run, copy 1 GiB with a plain copy kernel (reference "
                         "for the HBM byte counters)")
    ap.add_argument("--no-kbw", action="store_true", help="skip the copy-bandwidth probe")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: sharding the network over several GPUs "
              "(one RCCL allgather of spike bits per epoch) is designed but not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_06332_amd import sim as S, costmodel

    print(f"bench: generating {args.workload}", file=sys.stderr, flush=True)
    prob = make_workload(args.workload, args.neurons or None, args.precision)
    print(f"bench: {args.workload} ready; creating the simulation "
          f"({'fixed layout' if (args.no_autotune or args.lds_classes) else 'autotuning'})",
          file=sys.stderr, flush=True)
    C = int(prob["comp_off"][-1])
    N = int(prob["n_comp"].shape[0])
    prec = int(prob["params"]["precision"])
    multi = len(np.unique(prob["n_comp"])) > 1
    stream = torch.cuda.Stream()

    cost_model = None
    packing = dict(plain=S.PACK_PLAIN, count=S.PACK_COUNT, learned=S.PACK_LEARNED)[args.packing]
    solver = dict(exact=S.SOLVE_EXACT, fast=S.SOLVE_FAST, contract=S.SOLVE_CONTRACT)[args.solver]
    if packing == S.PACK_LEARNED:
        cost_model = costmodel.load_or_train(prob, solver=solver)

    g, ms = time_run(S, prob, args.steps, args.warmup, packing, cost_model,
                     autotune=not (args.no_autotune or args.lds_classes), stream=stream,
                     solver=solver, lds_classes=args.lds_classes)
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
    # the dominant kernel: the size-class-0 launch; its units are the
    # compartment-updates its launches performed over the timed region
    # (class compartments x the steps each launch ran), its time the launches'
    # own device spans
    k_ms, k_n, k_comps, k_upd = cls[0]
    kernel_ms = k_ms / max(k_n, 1)
    upd_per_launch = k_upd / max(k_n, 1)
    steps_per_launch = upd_per_launch / max(k_comps, 1)
    achieved_gbs = b_alg * upd_per_launch / (kernel_ms / 1e3) / 1e9
    kbw = None if args.no_kbw else copy_bandwidth(stream)

    # HBM bytes per launch measured with rocprofv3 counters on this kernel
    # source (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known
    # size), one record per profiled layout; reported only while the kernel
    # source is unchanged, for the same layout and a launch of the profiled
    # length.
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{prob['name']}.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            rec = json.load(f)
        if rec.get("kernel_source_sha1") == kernel_source_hash():
            for lay in rec.get("layouts", []):
                if (abs(lay.get("steps_per_launch", -1) - steps_per_launch) < 1e-9
                        and lay.get("launch") == config_str):
                    traffic = lay.get("bytes_per_launch")

    out = {
        "metric": METRIC,
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
            "hbm_roofline_frac_whole_run": value * b_alg / (PEAK_HBM_GBS * 1e9),
            "plain_packing_hbm_roofline_frac": (plain * b_alg / (PEAK_HBM_GBS * 1e9)
                                                if plain else None),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / PEAK_HBM_GBS,
            "traffic": traffic,
            "kernel": "k_epoch, size class 0 launch",
            "algorithmic_bytes_per_update": b_alg,
            "updates_per_launch": upd_per_launch,
            "steps_per_launch": steps_per_launch,
            "compartments_per_launch_step": k_comps,
            "kernel_ms": kernel_ms,
            "kernel_launches": k_n,
            "k_bw_GBps": kbw,
            "frac_of_k_bw": (achieved_gbs / kbw) if kbw else None,
            "epoch_ms": epoch_ms / max(epochs, 1),
            "class_ms": [c[0] / max(c[1], 1) for c in cls],
            "class_compartments": [c[2] for c in cls],
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
