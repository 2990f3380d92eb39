"""Seeded synthetic workloads: morphologies, synapses and drive.

This module only draws inputs. It holds none of the simulation's arithmetic
(no areas, conductances, matrix coefficients or channel kinetics): both the
GPU library and the CPU oracle receive the arrays it returns and derive
everything else themselves.

The paper measures on randomly sized neurons (Section 4: a 20-size group with
a spread of 700 and mean 300; later an F-distribution) and never publishes a
morphology dataset, so every workload here is synthetic. The five standard
workloads are:

  cfg1  64 identical neurons, soma + 4 unbranched dendrites x 50 compartments
  cfg2  8192 identical neurons, 1000 compartments, random binary tree, 32 branches
  cfg3  16384 neurons, log-normal sizes (median 500, sigma 0.5, clip 50..8000)
  cfg4  32768 neurons, same distribution as cfg3
  cfg5  100000 neurons, log-normal (median 1000, clip 50..16000), delays 40..200 steps

Problem dictionary (all numpy arrays, neuron-major CSR):
  n_comp[N] i32, comp_off[N+1] i64, parent[C] i32 (neuron-local, -1 at the root,
  0 <= parent[i] < i), length_um[C] f64, diam_um[C] f64, mech[C] u8 (0 passive,
  1 Hodgkin-Huxley), detector[N] i32, iext_nA[N] f64,
  syn_pre[S], syn_post[S], syn_comp[S], syn_delay[S] i32, syn_w[S] f64,
  params (dict), channels (dict), n_steps (int), name (str).
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

# Biophysical constants of the standard workloads (modern Hodgkin-Huxley
# squid-axon values; the paper leaves channel kinetics unspecified).
CHANNELS = dict(cm=1.0, ra=100.0, gnabar=0.12, gkbar=0.036, gl=0.0003,
                ena=50.0, ek=-77.0, el=-54.3, g_pas=1e-4, e_pas=-65.0)

# Soma: one 20 um x 20 um cylinder at compartment 0 of every neuron.
SOMA_L_UM = 20.0
SOMA_D_UM = 20.0
DEND_L_UM = 10.0

# Upper end of the uniform somatic drive U(0, I_max) in nA, one per workload.
# Chosen once so that a fair share (roughly a third to a half) of the neurons
# fire within the first 100 ms; frozen here so the inputs never change.
IEXT_MAX_NA = {1: 0.6, 2: 3.0, 3: 2.0, 4: 2.0, 5: 3.0, "mini": 2.0}


def default_params(precision: int = 0) -> dict:
    return dict(dt=0.025, theta=0.5, tau_syn=2.0, e_syn=0.0, v_thresh=0.0,
                v_init=-65.0, precision=precision)


# ---------------------------------------------------------------------------
# tree construction
# ---------------------------------------------------------------------------

def _random_branch_tree(n_branches: int, u: np.ndarray):
    """Binary branch tree: the soma gets two child branches, then a uniformly
    chosen leaf branch gets two children until n_branches exist.

    ``u`` holds (n_branches - 2) / 2 uniforms in [0, 1). Returns
    (branch_parent[B] with -1 for soma children, children lists) where branch
    ids are in creation order.
    """
    bpar = [-1, -1]
    children = [[], []]
    leaves = [0, 1]
    for x in u:
        k = int(x * len(leaves))
        if k >= len(leaves):
            k = len(leaves) - 1
        b = leaves.pop(k)
        for _ in range(2):
            bpar.append(b)
            children.append([])
            children[b].append(len(bpar) - 1)
            leaves.append(len(bpar) - 1)
    return bpar, children


def _dfs_order(bpar, children):
    """Depth-first order of branches, soma children first, children in
    creation order."""
    roots = [b for b, p in enumerate(bpar) if p < 0]
    order = []
    stack = list(reversed(roots))
    while stack:
        b = stack.pop()
        order.append(b)
        stack.extend(reversed(children[b]))
    return order


def _build_neuron(bpar, children, lens, d0, d1):
    """Compartment arrays of one neuron: soma at 0, then branches in DFS order,
    each branch contiguous from its base (proximal) to its tip (distal).
    lens/d0/d1 are indexed by branch id (creation order); every branch has at
    least one compartment. A branch's diameter tapers linearly from d0 at its
    base to d1 at its tip, sampled at the compartment midpoints."""
    order = np.asarray(_dfs_order(bpar, children), np.int64)
    lens = np.asarray(lens, np.int64)
    L = lens[order]                                   # branch lengths, DFS order
    n = 1 + int(L.sum())
    first = np.empty(lens.shape[0], np.int64)         # first compartment, by branch id
    first[order] = 1 + np.concatenate(([0], np.cumsum(L)[:-1]))
    tip = first + lens - 1
    bp = np.asarray(bpar, np.int64)
    base_parent = np.where(bp < 0, 0, tip[np.maximum(bp, 0)])
    br = np.repeat(order, L)                          # branch of compartments 1..n-1
    local = np.arange(1, n, dtype=np.int64) - first[br]
    parent = np.empty(n, np.int32)
    parent[0] = -1
    parent[1:] = np.where(local == 0, base_parent[br], np.arange(n - 1, dtype=np.int64))
    length = np.full(n, DEND_L_UM, np.float64)
    length[0] = SOMA_L_UM
    diam = np.empty(n, np.float64)
    diam[0] = SOMA_D_UM
    frac = (local + 0.5) / lens[br]
    diam[1:] = d0[br] + (d1[br] - d0[br]) * frac
    return parent, length, diam


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def _assemble(name, seed, morphs, mech_fn, rng, syn_per_neuron, delay_fn,
              iext_max, n_steps, precision):
    N = len(morphs)
    n_comp = np.array([m[0].shape[0] for m in morphs], np.int32)
    comp_off = np.zeros(N + 1, np.int64)
    comp_off[1:] = np.cumsum(n_comp)
    parent = np.concatenate([m[0] for m in morphs])
    length = np.concatenate([m[1] for m in morphs])
    diam = np.concatenate([m[2] for m in morphs])
    mech = np.concatenate([mech_fn(m[0].shape[0]) for m in morphs]).astype(np.uint8)

    S = syn_per_neuron
    post = np.repeat(np.arange(N, dtype=np.int32), S)
    if N > 1:
        pre = rng.integers(0, N - 1, size=N * S).astype(np.int32)
        pre = pre + (pre >= post).astype(np.int32)          # no autapses
    else:
        pre = np.zeros(N * S, np.int32)
    comp = np.floor(rng.random(N * S) * np.repeat(n_comp, S)).astype(np.int32)
    comp = np.minimum(comp, np.repeat(n_comp, S) - 1)
    w = rng.random(N * S) * 0.01
    delay = delay_fn(N * S).astype(np.int32)
    iext = rng.random(N) * iext_max
    return dict(
        name=name, seed=seed, n_steps=int(n_steps),
        n_comp=n_comp, comp_off=comp_off, parent=parent.astype(np.int32),
        length_um=length, diam_um=diam, mech=mech,
        detector=np.zeros(N, np.int32), iext_nA=iext,
        syn_pre=pre, syn_post=post, syn_comp=comp, syn_delay=delay, syn_w=w,
        params=default_params(precision), channels=dict(CHANNELS),
    )


def config1(seed: int = 1, precision: int = 0) -> dict:
    """64 identical neurons: soma + 4 dendrites of 50 compartments (d U(1,2) um,
    one draw per dendrite compartment shared by all neurons, L 10 um). HH on
    the soma, leak on the dendrites; 10 synapses per neuron, delay 40 steps."""
    rng = np.random.default_rng(seed)
    dend_d = rng.uniform(1.0, 2.0, size=200)
    n = 201
    parent = np.empty(n, np.int32)
    parent[0] = -1
    for k in range(4):
        b0 = 1 + 50 * k
        parent[b0] = 0
        parent[b0 + 1:b0 + 50] = np.arange(b0, b0 + 49)
    length = np.full(n, DEND_L_UM)
    length[0] = SOMA_L_UM
    diam = np.concatenate([[SOMA_D_UM], dend_d])
    morphs = [(parent, length, diam)] * 64

    def mech(nc):
        m = np.zeros(nc, np.uint8)
        m[0] = 1
        return m
    return _assemble("cfg1", seed, morphs, mech, rng, 10,
                     lambda s: np.full(s, 40), IEXT_MAX_NA[1], 400, precision)


def _taper(rng, B):
    d0 = rng.uniform(0.5, 3.0, size=B)
    d1 = 0.5 + rng.random(B) * (d0 - 0.5)
    return d0, d1


def _hh_all(nc):
    return np.ones(nc, np.uint8)


def config2(seed: int = 2, precision: int = 0, n_neurons: int = 8192,
            n_steps: int = 4000) -> dict:
    """Identical neurons of 1000 compartments: random binary tree of 32
    branches, 999 dendritic compartments split equally (31-32 per branch);
    one morphology shared by every neuron. HH everywhere; 50 synapses per
    neuron, delay 40 steps."""
    rng = np.random.default_rng(seed)
    B = 32
    bpar, ch = _random_branch_tree(B, rng.random((B - 2) // 2))
    lens = np.full(B, 999 // B)
    lens[:999 - lens.sum()] += 1
    d0, d1 = _taper(rng, B)
    morph = _build_neuron(bpar, ch, lens, d0, d1)
    morphs = [morph] * n_neurons
    return _assemble("cfg2", seed, morphs, _hh_all, rng, 50,
                     lambda s: np.full(s, 40), IEXT_MAX_NA[2], n_steps,
                     precision)


def _lognormal_neurons(rng, N, median, lo, hi):
    n = np.rint(np.exp(np.log(median) + 0.5 * rng.standard_normal(N)))
    n = np.clip(n, lo, hi).astype(np.int64)
    bmax = np.minimum(256, 2 * ((n - 1) // 4))
    nb_choices = (bmax - 4) // 2 + 1
    nb = 4 + 2 * np.floor(rng.random(N) * nb_choices).astype(np.int64)
    nb = np.minimum(nb, bmax)
    morphs = []
    for j in range(N):
        B = int(nb[j])
        bpar, ch = _random_branch_tree(B, rng.random((B - 2) // 2))
        extra = int(n[j]) - 1 - 2 * B
        lens = 2 + rng.multinomial(extra, np.full(B, 1.0 / B))
        d0, d1 = _taper(rng, B)
        morphs.append(_build_neuron(bpar, ch, lens, d0, d1))
    return morphs


def multi_morphology(name: str, seed: int, n_neurons: int, median: float,
                     lo: int, hi: int, syn_per_neuron: int, delay_lo: int,
                     delay_hi: int, n_steps: int, iext_max: float,
                     precision: int = 1) -> dict:
    """Multi-morphology network: per-neuron compartment count log-normal
    (sigma 0.5 in log space, clipped), an even number of branches uniform in
    [4, min(256, 2*floor((n-1)/4))], at least 2 compartments per branch with
    the rest split multinomially, diameters tapering linearly per branch from
    U(0.5, 3) um to U(0.5, start) um. HH everywhere."""
    rng = np.random.default_rng(seed)
    morphs = _lognormal_neurons(rng, n_neurons, median, lo, hi)
    if delay_lo == delay_hi:
        dfn = (lambda s: np.full(s, delay_lo))
    else:
        dfn = (lambda s: rng.integers(delay_lo, delay_hi + 1, size=s))
    return _assemble(name, seed, morphs, _hh_all, rng, syn_per_neuron, dfn,
                     iext_max, n_steps, precision)


def config3(seed: int = 3, precision: int = 1, n_neurons: int = 16384,
            n_steps: int = 4000) -> dict:
    return multi_morphology("cfg3", seed, n_neurons, 500, 50, 8000, 100, 40,
                            40, n_steps, IEXT_MAX_NA[3], precision)


def config4(seed: int = 4, precision: int = 1, n_neurons: int = 32768,
            n_steps: int = 4000) -> dict:
    return multi_morphology("cfg4", seed, n_neurons, 500, 50, 8000, 100, 40,
                            40, n_steps, IEXT_MAX_NA[4], precision)


def config5(seed: int = 5, precision: int = 1, n_neurons: int = 100000,
            n_steps: int = 4000) -> dict:
    return multi_morphology("cfg5", seed, n_neurons, 1000, 50, 16000, 200, 40,
                            200, n_steps, IEXT_MAX_NA[5], precision)


def mini(seed: int = 11, n_neurons: int = 48, precision: int = 1,
         n_steps: int = 200, median: float = 120, syn: int = 12,
         delay_lo: int = 40, delay_hi: int = 40) -> dict:
    """Small multi-morphology network with the cfg3 recipe, sized so that
    the oracle finishes in well under a second."""
    return multi_morphology("mini", seed, n_neurons, median, 12, 4 * median,
                            syn, delay_lo, delay_hi, n_steps,
                            IEXT_MAX_NA["mini"], precision)


def group_sizes(rng, count: int = 20, spread: int = 700, mean: int = 300,
                smallest: int = 12) -> np.ndarray:
    """`count` random neuron sizes whose largest minus smallest is exactly
    `spread`, whose mean is exactly `mean` and whose smallest is at least
    `smallest` (the size group of the paper's Section 4 experiment).

    The smallest and largest members sit at m and m + spread; the others are
    m + spread * x with x ~ Beta(1, 2) (skewed small, so that the mean can be
    reached with m >= smallest), redrawn until that holds; integer rounding
    is then corrected by +-1 steps on the inner members so that the sum is
    exactly count * mean."""
    while True:
        x = np.concatenate([[0.0, 1.0], rng.beta(1.0, 2.0, count - 2)])
        m = mean - spread * x.mean()
        if m >= smallest:
            break
    lo = int(np.rint(m))
    sizes = np.concatenate([[lo, lo + spread],
                            np.rint(lo + spread * x[2:]).astype(np.int64)]).astype(np.int64)
    sizes[2:] = np.clip(sizes[2:], lo, lo + spread)
    diff = count * mean - int(sizes.sum())
    k = 2
    while diff != 0:
        step = 1 if diff > 0 else -1
        if lo < sizes[k] + step < lo + spread:
            sizes[k] += step
            diff -= step
        k = 2 + (k - 1) % (count - 2)
    return sizes


def size_group(seed: int = 7, n_neurons: int = 10000, mono: bool = False,
               precision: int = 1, n_steps: int = 400) -> dict:
    """The paper's Section-4 imbalance test: a group of 20 neurons whose sizes
    have a spread (max - min) of exactly 700 compartments and a mean of
    exactly 300 (group_sizes); the network holds n_neurons / 20 copies of each
    member in a random order, so its compartment total equals that of the
    mono-morphology network, n_neurons copies of one 300-compartment neuron.
    The trees follow the cfg3 recipe with at most 32 branches."""
    rng = np.random.default_rng(seed)
    g = group_sizes(rng)

    def one(n):
        B = max(2, int(min(32, 2 * ((n - 1) // 4))))
        bpar, ch = _random_branch_tree(B, rng.random((B - 2) // 2))
        extra = n - 1 - 2 * B
        lens = 2 + rng.multinomial(extra, np.full(B, 1.0 / B))
        d0, d1 = _taper(rng, B)
        return _build_neuron(bpar, ch, lens, d0, d1)

    if mono:
        proto = one(300)
        morphs = [proto] * n_neurons
    else:
        group = [one(int(n)) for n in g]
        pick = np.resize(np.arange(20), n_neurons)
        rng.shuffle(pick)
        morphs = [group[k] for k in pick]
    return _assemble("size_group_mono" if mono else "size_group", seed, morphs,
                     _hh_all, rng, 100, lambda s: np.full(s, 40), 2.0,
                     n_steps, precision)


def star_network(seed: int = 31, n_neurons: int = 16, fanout=(64, 5), branch_len: int = 3,
                 precision: int = 1, n_steps: int = 200) -> dict:
    """Neurons whose soma carries many unbranched dendrites (neuron j has
    fanout[j % len(fanout)] children of branch_len compartments, diameters as
    in the cfg3 recipe): nodes of very high fan-out, a degenerate case of the
    tree solve. HH everywhere, 12 synapses per neuron, delay 40 steps."""
    rng = np.random.default_rng(seed)
    morphs = []
    for j in range(n_neurons):
        B = int(fanout[j % len(fanout)])
        n = 1 + B * branch_len
        parent = np.empty(n, np.int32)
        parent[0] = -1
        length = np.full(n, DEND_L_UM)
        length[0] = SOMA_L_UM
        diam = np.empty(n)
        diam[0] = SOMA_D_UM
        d0, d1 = _taper(rng, B)
        for b in range(B):
            b0 = 1 + b * branch_len
            parent[b0] = 0
            parent[b0 + 1:b0 + branch_len] = np.arange(b0, b0 + branch_len - 1)
            frac = (np.arange(branch_len) + 0.5) / branch_len
            diam[b0:b0 + branch_len] = d0[b] + (d1[b] - d0[b]) * frac
        morphs.append((parent, length, diam))
    return _assemble("star", seed, morphs, _hh_all, rng, 12, lambda s: np.full(s, 40),
                     IEXT_MAX_NA["mini"], n_steps, precision)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def make(cfg, **kw) -> dict:
    """Problem for a numbered workload (1..5) with optional overrides
    (n_neurons, n_steps, precision, seed). Large problems are cached on disk
    under $MMHINES_CACHE (default /tmp/mmhines_cache)."""
    fn = CONFIGS[cfg]
    key = hashlib.sha1(repr((cfg, sorted(kw.items()), _VERSION)).encode()).hexdigest()[:16]
    cdir = os.environ.get("MMHINES_CACHE", "/tmp/mmhines_cache")
    path = os.path.join(cdir, f"cfg{cfg}_{key}.npz")
    if os.path.exists(path):
        return load(path)
    prob = fn(**kw)
    if prob["comp_off"][-1] > 200000:
        try:
            os.makedirs(cdir, exist_ok=True)
            save(prob, path)
        except OSError:
            pass
    return prob


_VERSION = 1
_ARRAYS = ("n_comp", "comp_off", "parent", "length_um", "diam_um", "mech",
           "detector", "iext_nA", "syn_pre", "syn_post", "syn_comp",
           "syn_delay", "syn_w")


def save(prob: dict, path: str) -> None:
    meta = {k: prob[k] for k in ("name", "seed", "n_steps")}
    extra = {f"p_{k}": v for k, v in prob["params"].items()}
    extra.update({f"c_{k}": v for k, v in prob["channels"].items()})
    tmp = path + ".tmp.npz"
    np.savez(tmp, **{k: prob[k] for k in _ARRAYS},
             meta=np.array(repr(meta)), **{k: np.array(v) for k, v in extra.items()})
    os.replace(tmp, path)


def load(path: str) -> dict:
    import ast
    z = np.load(path, allow_pickle=False)
    prob = {k: z[k] for k in _ARRAYS}
    prob.update(ast.literal_eval(str(z["meta"])))
    prob["params"] = {k[2:]: z[k].item() for k in z.files if k.startswith("p_")}
    prob["channels"] = {k[2:]: z[k].item() for k in z.files if k.startswith("c_")}
    return prob


def subset(prob: dict, neurons) -> dict:
    """Sub-network of the given neurons (in the given order): keeps their
    morphologies and the synapses among them, renumbered."""
    neurons = np.asarray(neurons, np.int64)
    N = prob["n_comp"].shape[0]
    remap = np.full(N, -1, np.int64)
    remap[neurons] = np.arange(neurons.shape[0])
    off = prob["comp_off"]
    idx = np.concatenate([np.arange(off[j], off[j + 1]) for j in neurons])
    n_comp = prob["n_comp"][neurons].astype(np.int32)
    comp_off = np.zeros(neurons.shape[0] + 1, np.int64)
    comp_off[1:] = np.cumsum(n_comp)
    keep = (remap[prob["syn_pre"]] >= 0) & (remap[prob["syn_post"]] >= 0)
    order = np.argsort(remap[prob["syn_post"][keep]], kind="stable")
    out = dict(prob)
    out.update(
        n_comp=n_comp, comp_off=comp_off, parent=prob["parent"][idx],
        length_um=prob["length_um"][idx], diam_um=prob["diam_um"][idx],
        mech=prob["mech"][idx], detector=prob["detector"][neurons],
        iext_nA=prob["iext_nA"][neurons],
        syn_pre=remap[prob["syn_pre"][keep]][order].astype(np.int32),
        syn_post=remap[prob["syn_post"][keep]][order].astype(np.int32),
        syn_comp=prob["syn_comp"][keep][order],
        syn_delay=prob["syn_delay"][keep][order],
        syn_w=prob["syn_w"][keep][order],
        params=dict(prob["params"]), channels=dict(prob["channels"]),
    )
    return out


def replay_subset(prob: dict, neurons) -> dict:
    """The given neurons (in the given order) with every synapse onto them,
    for replaying recorded presynaptic spikes: post ids are renumbered, pre
    ids keep the full network's numbering, and the synapses keep their
    relative order."""
    neurons = np.asarray(neurons, np.int64)
    N = prob["n_comp"].shape[0]
    remap = np.full(N, -1, np.int64)
    remap[neurons] = np.arange(neurons.shape[0])
    off = prob["comp_off"]
    idx = np.concatenate([np.arange(off[j], off[j + 1]) for j in neurons])
    n_comp = prob["n_comp"][neurons].astype(np.int32)
    comp_off = np.zeros(neurons.shape[0] + 1, np.int64)
    comp_off[1:] = np.cumsum(n_comp)
    keep = remap[prob["syn_post"]] >= 0
    order = np.argsort(remap[prob["syn_post"][keep]], kind="stable")
    out = dict(prob)
    out.update(
        n_comp=n_comp, comp_off=comp_off, parent=prob["parent"][idx],
        length_um=prob["length_um"][idx], diam_um=prob["diam_um"][idx],
        mech=prob["mech"][idx], detector=prob["detector"][neurons],
        iext_nA=prob["iext_nA"][neurons],
        syn_pre=prob["syn_pre"][keep][order].astype(np.int32),
        syn_post=remap[prob["syn_post"][keep]][order].astype(np.int32),
        syn_comp=prob["syn_comp"][keep][order],
        syn_delay=prob["syn_delay"][keep][order],
        syn_w=prob["syn_w"][keep][order],
        params=dict(prob["params"]), channels=dict(prob["channels"]),
    )
    return out


def spike_raster(spikes: np.ndarray, n_neurons: int, n_steps: int) -> np.ndarray:
    """uint8 [(n_steps+1), n_neurons] from (neuron, step) pairs."""
    r = np.zeros((n_steps + 1, n_neurons), np.uint8)
    sp = np.asarray(spikes).reshape(-1, 2)
    if sp.size:
        r[sp[:, 1], sp[:, 0]] = 1
    return r


def summary(prob: dict) -> str:
    N = prob["n_comp"].shape[0]
    C = int(prob["comp_off"][-1])
    return (f"{prob['name']}: N={N} C={C} S={prob['syn_pre'].shape[0]} "
            f"n_comp[min/med/max]={prob['n_comp'].min()}/"
            f"{int(np.median(prob['n_comp']))}/{prob['n_comp'].max()} "
            f"steps={prob['n_steps']}")
