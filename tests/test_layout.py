"""Host layout on the CPU (no GPU): sim_plan_create lays a problem out exactly
as sim_create would for a given LDS size and CU count, without a device.

- every neuron sits in exactly one pack, every pack in exactly one workgroup
  list of one size class;
- LDS accounting: each pack's table and state bytes equal the carve-up the
  epoch kernel makes (restated here from the kernel's layout), LDS packs fit
  their class's allocation, and a class allocates what its largest pack needs;
- persistent scheduling is Graham's LPT list schedule: its makespan is at most
  (4/3 - 1/(3m)) times the optimum, checked against brute force on up to 10
  packs (P15);
- the contraction solver's elimination schedule eliminates every compartment
  once, each round's compartments are at distance >= 3 in the contracted
  tree and have degree <= 2, and executing it solves the tree system (checked
  against a dense solve); so do the pack-level items in the epoch kernel's
  own encoding.
"""
import itertools

import numpy as np
import pytest

from paper_2005_06332_amd import workload as W


@pytest.fixture(scope="module")
def S():
    from paper_2005_06332_amd import sim
    sim.lib()
    return sim


def plan(S, prob, lds=160 * 1024, n_cu=256, **kw):
    return S.Simulation(prob, plan=(lds, n_cu), **kw)


def align(x, a):
    return (x + a - 1) // a * a


def table_bytes(info, tsize):
    """Tables as the kernel carves them: branch records (16 B), synapse
    weights, level offsets (4 B, 4-aligned), forward order and child list
    (2 B each), synapse targets and run lengths (2 B each); the contraction
    solver stages no branch records, levels, forward order or child list,
    but its round offsets (4 B) and the items staged in LDS (8 B, 8-aligned;
    the others stay in global memory); the whole rounded to 16 B."""
    # (the contraction solver, n_rounds > 0, stages no branch tables)
    nbr, nlev, nch = info["n_branches"], info["n_levels"], info["n_child_entries"]
    if info["n_rounds"] > 0:
        nbr = nlev = nch = 0
    b = 16 * nbr + tsize * info["n_syn"]
    b = align(b, 4) + 4 * nlev
    b += 2 * nbr + 2 * nch + 4 * info["n_syn"]
    if info["n_rounds"] > 0:
        b = align(b, 4) + 4 * (info["n_rounds"] + 1)
    if info["n_staged_items"] > 0:
        b = align(b, 8) + 8 * info["n_staged_items"]
    return align(b, 16)


def state_bytes(info, tsize):
    """V, the off-diagonal, R and D (8 B per compartment each; the
    contraction solver's arrays have one spare entry more), synapse event
    masks (8 B), spike masks, detector voltages, external currents and
    detector indices (8 B per neuron each), synaptic conductances
    (16-aligned), 64 B of sweep slack."""
    n, s, k = info["n_comp"], info["n_syn"], info["n_neurons"]
    if info["n_rounds"] > 0:
        n += 1
    return 32 * n + 8 * s + 32 * k + align(tsize * s, 16) + 64


CASES = [
    ("mini count", lambda: W.mini(), dict()),
    ("mini plain", lambda: W.mini(), dict(packing=0)),
    ("mini contract", lambda: W.mini(), dict(solver=2)),
    ("mini fp64 small lds", lambda: W.mini(precision=0), dict(lds_comps=120, solver=2)),
    ("cfg3 subset persistent", lambda: W.subset(W.make(3), np.arange(3000)),
     dict(sched=1, lds_classes=3)),
    ("cfg1 contract", lambda: W.config1(), dict(solver=2, sched=1)),
]


@pytest.mark.parametrize("name,mk,kw", CASES, ids=[c[0] for c in CASES])
def test_layout_places_every_neuron_once_and_fits_lds(S, name, mk, kw):
    prob = mk()
    N = prob["n_comp"].shape[0]
    tsize = 4 if prob["params"]["precision"] == 1 and kw.get("precision", 1) == 1 else 8
    lds = 160 * 1024
    with plan(S, prob, lds=lds, **kw) as g:
        npk = g.pack_count()
        seen = np.zeros(N, np.int64)
        infos = []
        for p in range(npk):
            info = g.pack_info(p)
            infos.append(info)
            ids = g.pack_neurons(p)
            seen[ids] += 1
            assert info["n_comp"] == int(prob["n_comp"][ids].sum())
            assert info["table_bytes"] == table_bytes(info, tsize), (name, p, info)
            assert info["state_bytes"] == state_bytes(info, tsize), (name, p, info)
        assert np.all(seen == 1)
        ran = np.zeros(npk, np.int64)
        for c in range(3):
            n_wg, threads, cls_lds = g.class_launch(c)
            assert cls_lds <= lds
            need = 256
            for w in range(n_wg):
                for p in g.workgroup_packs(c, w):
                    ran[p] += 1
                    info = infos[p]
                    assert info["size_class"] == c
                    b = info["table_bytes"] + (0 if info["in_global"] else info["state_bytes"])
                    assert b <= cls_lds
                    need = max(need, b)
            if n_wg:
                assert need == cls_lds
        assert np.all(ran == 1)


def test_plan_refuses_what_needs_the_device(S):
    prob = W.mini()
    with pytest.raises(S.SimError):
        plan(S, prob, autotune=True)
    with plan(S, prob) as g:
        with pytest.raises(S.SimError) as e:
            g.step(1)
        assert e.value.code == S.SIM_ESTATE
        with pytest.raises(S.SimError):
            g.voltages()


def opt_makespan(costs, m):
    """Minimum over all assignments of the largest machine load (branch and
    bound over the items in decreasing order)."""
    costs = sorted(costs, reverse=True)
    best = [sum(costs)]
    loads = [0.0] * m

    def rec(i):
        if i == len(costs):
            best[0] = min(best[0], max(loads))
            return
        seen = set()
        for w in range(m):
            if loads[w] in seen or loads[w] + costs[i] >= best[0]:
                continue
            seen.add(loads[w])
            loads[w] += costs[i]
            rec(i + 1)
            loads[w] -= costs[i]
    rec(0)
    return best[0]


@pytest.mark.parametrize("seed,n,threads,lds", [
    (41, 10, 1024, 64 * 1024), (42, 9, 640, 64 * 1024), (43, 10, 512, 160 * 1024),
    (44, 8, 640, 64 * 1024), (45, 10, 1024, 64 * 1024), (46, 7, 512, 160 * 1024),
])
def test_persistent_schedule_is_within_graham_lpt_bound(S, seed, n, threads, lds):
    """P15: one neuron per pack (pack_comps = 1), one CU, so the class-0
    launch has m = 2..4 persistent workgroups; the static lists must be
    Graham's LPT schedule, whose makespan is at most (4/3 - 1/(3m)) OPT."""
    prob = W.mini(seed=seed, n_neurons=n, median=60)
    with plan(S, prob, lds=lds, n_cu=1, sched=1, pack_comps=1, threads=threads) as g:
        n_wg, _, _ = g.class_launch(0)
        assert g.class_launch(1)[0] == 0
        costs = [g.pack_info(p)["cost"] for p in range(g.pack_count())]
        assert len(costs) == n
        loads = [sum(costs[p] for p in g.workgroup_packs(0, w)) for w in range(n_wg)]
    m = n_wg
    assert 2 <= m <= 4
    lpt = max(loads)
    opt = opt_makespan(costs, m)
    assert lpt <= (4.0 / 3.0 - 1.0 / (3 * m)) * opt + 1e-9, (lpt, opt, m)
    # and it is the list schedule: packs by decreasing cost, each to the
    # least loaded workgroup (ties to the lowest index)
    order = sorted(range(n), key=lambda p: -costs[p])
    sim_loads = [0.0] * m
    for p in order:
        w = min(range(m), key=lambda w: (sim_loads[w], w))
        sim_loads[w] += costs[p]
    assert sorted(sim_loads) == sorted(loads)


def contracted_neighbours(parent_cur, children_cur, k):
    nb = set(children_cur[k])
    if parent_cur[k] >= 0:
        nb.add(parent_cur[k])
    return nb


def execute_schedule(items, ro, p, e, d, r):
    """The elimination the schedule describes, in numpy (test-side), then back
    substitution in reverse round order. As in the kernel, a coupling is read
    from the slot the fills write (EW, which starts with no valid entry) when
    the item flags it as made by an earlier elimination, else from the
    off-diagonal e."""
    n = len(p)
    D, R, V, EW = d.copy(), r.copy(), np.zeros(n), np.full(n, np.nan)
    for q in range(len(items)):
        k, n1, n2, fl = items[q]
        up = fl & 1
        y = 1.0 / D[k]
        a1 = ((EW if fl & 2 else e)[k if up else n1]) if n1 >= 0 else 0.0
        a2 = (EW if fl & 4 else e)[n2] if n2 >= 0 else 0.0
        if n1 >= 0:
            D[n1] -= a1 * a1 * y
            R[n1] -= a1 * R[k] * y
        if n2 >= 0:
            D[n2] -= a2 * a2 * y
            R[n2] -= a2 * R[k] * y
            if n1 >= 0:
                EW[n2] = -a1 * a2 * y
        R[k], EW[k], V[k] = R[k] * y, a1 * y, a2 * y
    for rr in range(len(ro) - 2, -1, -1):
        for q in range(ro[rr], ro[rr + 1]):
            k, n1, n2, _ = items[q]
            x = R[k]
            if n1 >= 0:
                x -= EW[k] * V[n1]
            if n2 >= 0:
                x -= V[k] * V[n2]
            V[k] = x
    return V


@pytest.mark.parametrize("which", ["mini", "cfg1", "star", "cfg3"])
def test_contraction_schedule_is_a_valid_elimination(S, which):
    prob = {"mini": lambda: W.mini(), "cfg1": W.config1, "star": W.star_network,
            "cfg3": lambda: W.subset(W.make(3), np.arange(24))}[which]()
    rng = np.random.default_rng(5)
    off = prob["comp_off"]
    with plan(S, prob, solver=2) as g:
        for j in range(min(prob["n_comp"].shape[0], 12)):
            p = prob["parent"][off[j]:off[j + 1]].astype(np.int64)
            n = p.shape[0]
            items, ro = g.contraction_schedule(j, n)
            assert sorted(items[:, 0].tolist()) == list(range(n))
            assert ro[0] == 0 and ro[-1] == n and np.all(np.diff(ro) > 0)
            # replay the contraction on the tree and check each round
            made = np.zeros(n, bool)  # coupling to the current parent made by a fill
            par = p.copy()
            ch = [set() for _ in range(n)]
            for i in range(1, n):
                ch[p[i]].add(i)
            for rr in range(len(ro) - 1):
                closed = set()
                for q in range(ro[rr], ro[rr + 1]):
                    k, n1, n2, fl = (int(x) for x in items[q])
                    up = fl & 1
                    nb = contracted_neighbours(par, ch, k)
                    assert len(nb) <= 2
                    assert nb == {x for x in (n1, n2) if x >= 0}
                    assert (up == 1) == (n1 >= 0 and par[k] == n1)
                    # which couplings are fills, which the off-diagonal
                    if n1 >= 0:
                        assert bool(fl & 2) == bool(made[k] if up else made[n1])
                    if n2 >= 0:
                        assert bool(fl & 4) == bool(made[n2])
                    ball = nb | {k}
                    assert not (ball & closed), "round members closer than 3"
                    closed |= ball
                for q in range(ro[rr], ro[rr + 1]):
                    k, n1, n2, up = (int(x) for x in items[q])
                    if par[k] >= 0:
                        ch[par[k]].discard(k)
                    for c in list(ch[k]):
                        par[c] = -1
                    if n1 >= 0 and n2 >= 0:  # n2 hangs off n1 from now on
                        par[n2] = n1
                        ch[n1].add(n2)
                        made[n2] = True
                    ch[k] = set()
                    par[k] = -2
            # the elimination solves a random symmetric diagonally dominant
            # system on this tree
            e = np.zeros(n)
            e[1:] = -rng.uniform(0.05, 1.0, n - 1)
            dd = np.zeros(n)
            np.add.at(dd, np.arange(1, n), -e[1:])
            np.add.at(dd, p[1:], -e[1:])
            d = dd + rng.uniform(0.2, 1.5, n)
            rhs = rng.normal(size=n)
            A = np.diag(d)
            A[np.arange(1, n), p[1:]] = e[1:]
            A[p[1:], np.arange(1, n)] = e[1:]
            x = execute_schedule(items, ro, p, e, d, rhs)
            ref = np.linalg.solve(A, rhs)
            assert np.max(np.abs(x - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def execute_pack_items(items, n, e, d, r):
    """The epoch kernel's elimination and back substitution over a pack's
    items as it reads them (sim_pack_contraction_items), in numpy: arrays
    of n + 1 entries (the last is the spare compartment, off-diagonal 0),
    couplings read from the working slot W followed by the off-diagonal.
    The items run one after another, the back substitution in reverse: the
    kernel's rounds only group items that touch disjoint slots, so the
    result is the same."""
    m = n + 1
    D, R = np.append(d, 0.0), np.append(r, 0.0)
    WE = np.concatenate([np.zeros(m), np.append(e, 0.0)])  # W, then the off-diagonal
    its = [int(x) for x in items]
    for it in its:
        k, i1, i2 = it & 0x7FFF, (it >> 15) & 0xFFFF, (it >> 31) & 0xFFFF
        u1 = (it >> 47) & 0xFFFF
        u2 = i2 if it >> 63 else i2 + m
        a1, a2 = WE[u1], WE[u2]
        dk, rk = D[k], R[k]
        d1, r1, d2, r2 = D[i1], R[i1], D[i2], R[i2]
        y = 1.0 / dk
        h, g1, g2 = rk * y, a1 * y, a2 * y
        D[i1], R[i1] = d1 - a1 * g1, r1 - a1 * h
        D[i2], R[i2] = d2 - a2 * g2, r2 - a2 * h
        WE[i2] = -(a1 * g2)
        R[k], WE[k], D[k] = h, g1, g2
    V = WE[:m].copy()  # the back substitution writes x over the W slot
    for it in reversed(its):
        k, i1, i2 = it & 0x7FFF, (it >> 15) & 0xFFFF, (it >> 31) & 0xFFFF
        V[k] = R[k] - V[k] * V[i1] - D[k] * V[i2]
    return V[:n]


@pytest.mark.parametrize("which", ["mini", "cfg1", "star", "cfg3"])
def test_pack_items_as_the_kernel_reads_them_solve_the_pack(S, which):
    """Every item of every pack, in the kernel's encoding (absent neighbours
    as the spare compartment, the first coupling by one index into the
    working slot and the off-diagonal), eliminates its compartment once,
    and executing them solves each pack's tree systems (a dense solve of the
    pack's block-diagonal matrix)."""
    prob = {"mini": lambda: W.mini(), "cfg1": W.config1, "star": W.star_network,
            "cfg3": lambda: W.subset(W.make(3), np.arange(200))}[which]()
    rng = np.random.default_rng(17)
    off = prob["comp_off"]
    with plan(S, prob, solver=2) as g:
        for pk in range(g.pack_count()):
            items = g.pack_contraction_items(pk)
            n = g.pack_info(pk)["n_comp"]
            assert items.shape == (n,)
            k = (items & np.uint64(0x7FFF)).astype(np.int64)
            assert sorted(k.tolist()) == list(range(n))
            # the pack's tree: its neurons in pack order, compartments in order
            p = np.empty(n, np.int64)
            base = 0
            for j in g.pack_neurons(pk):
                pj = prob["parent"][off[j]:off[j + 1]].astype(np.int64)
                p[base:base + pj.shape[0]] = np.where(pj >= 0, pj + base, -1)
                base += pj.shape[0]
            assert base == n
            child = np.flatnonzero(p >= 0)
            e = np.zeros(n)
            e[child] = -rng.uniform(0.05, 1.0, child.shape[0])
            dd = np.zeros(n)
            np.add.at(dd, child, -e[child])
            np.add.at(dd, p[child], -e[child])
            d = dd + rng.uniform(0.2, 1.5, n)
            rhs = rng.normal(size=n)
            A = np.diag(d)
            A[child, p[child]] = e[child]
            A[p[child], child] = e[child]
            x = execute_pack_items(items, n, e, d, rhs)
            ref = np.linalg.solve(A, rhs)
            assert np.max(np.abs(x - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref))), pk


@pytest.mark.parametrize("which", ["cfg3 subset", "cfg1", "star"])
def test_contraction_tail_rounds_fit_one_wavefront(S, which):
    """A pack's round r is round r of each of its neurons; rounds from
    n_wide_rounds on (at most 63 of them) hold at most 64 items and are
    staged in LDS whole (one wavefront runs them without workgroup
    barriers), and the round before them holds more, is not staged whole,
    or would make the tail longer than 63 rounds (a soma with 64 children
    needs more than 64 rounds)."""
    prob = {"cfg3 subset": lambda: W.subset(W.make(3), np.arange(400)),
            "cfg1": W.config1, "star": W.star_network}[which]()
    off = prob["comp_off"]
    with plan(S, prob, solver=2) as g:
        for p in range(g.pack_count()):
            info = g.pack_info(p)
            sizes = np.zeros(info["n_rounds"], np.int64)
            for j in g.pack_neurons(p):
                _, ro = g.contraction_schedule(int(j), int(off[j + 1] - off[j]))
                sizes[:len(ro) - 1] += np.diff(ro)
            assert sizes.sum() == info["n_comp"]
            nw = info["n_wide_rounds"]
            assert 0 <= nw <= info["n_rounds"]
            st = info["n_staged_items"]
            nr = info["n_rounds"]
            assert np.all(sizes[nw:] <= 64), (p, nw, sizes)
            assert st >= sizes[nw:].sum()
            # the tail's lanes hold its round offsets: at most 63 rounds
            assert nr - nw <= 63
            if nw > 0:
                assert (sizes[nw - 1] > 64 or st < sizes[nw - 1:].sum()
                        or nr - nw == 63), (p, nw, sizes, st)
            # the staged items are a suffix of the tail rounds (those that
            # hold at most 64 items each)
            small = len(sizes)
            while small > 0 and sizes[small - 1] <= 64:
                small -= 1
            assert 0 <= st <= sizes[small:].sum()


def test_learned_packing_takes_given_neuron_costs(S):
    """Learned packing with per-neuron costs given in place of a model
    dispatches its best-fit packs in decreasing cost, the largest cost among
    a pack's neurons; invalid costs are refused."""
    prob = W.subset(W.make(3), np.arange(600))
    N = prob["n_comp"].shape[0]
    rng = np.random.default_rng(11)
    cost = rng.uniform(1.0, 2.0, N)
    with plan(S, prob, packing=S.PACK_LEARNED, neuron_cost=cost) as g:
        assert "learned(given costs)" in g.config
        pc = [g.pack_info(p)["cost"] for p in range(g.pack_count())]
        for p in range(g.pack_count()):
            assert pc[p] == pytest.approx(cost[g.pack_neurons(p)].max())
        # class by class, the dispatch (workgroup) order is decreasing cost
        for c in range(3):
            n_wg = g.class_launch(c)[0]
            order = [q for w in range(n_wg) for q in g.workgroup_packs(c, w)]
            cs = [pc[q] for q in order]
            assert cs == sorted(cs, reverse=True)
    for bad in (np.zeros(N), np.full(N, np.nan)):
        with pytest.raises(S.SimError):
            plan(S, prob, packing=S.PACK_LEARNED, neuron_cost=bad)
