// Host side of the simulator: input validation, morphology analysis
// (branches, levels, features), packing of neurons into workgroup packs,
// device layout, epoch launches (optionally replayed from a hipGraph) and the
// C ABI of include/sim.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include "../../include/sim.h"
#include "internal.h"

namespace mmh {
hipError_t mlp_forward(const float *params, const float *x, int64_t n, float *out);
hipError_t mlp_loss_grad(const float *params, const float *x, const float *t, int64_t n,
                         float *loss, float *grad);
hipError_t mlp_train(float *params, const float *x, const float *t, int64_t n, int epochs,
                     float lr, float *final_loss);
}  // namespace mmh

using namespace mmh;

namespace {

// Failure text of calls without a simulation handle (sim_create, the cost
// model calls); one per calling thread, so concurrent callers do not race.
thread_local std::string g_create_error;

struct Error {
    int code;
    std::string msg;
};

Error fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return Error{code, buf};
}

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            throw fail(SIM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));      \
    } while (0)

// ---------------------------------------------------------------------------
// Morphology analysis of one neuron.
// ---------------------------------------------------------------------------
struct NeuronTopo {
    int32_t n = 0;
    std::vector<int32_t> b0, b1, bpar, height, depth;  // per branch
    std::vector<int32_t> child_off, child;             // CSR of child branch ids
    std::vector<int32_t> branch_of;                    // per compartment
    int32_t max_height = 0, max_depth = 0;
};

void analyse(const int32_t *p, int32_t n, NeuronTopo &t) {
    t.n = n;
    std::vector<int32_t> nchild(n, 0);
    for (int32_t i = 1; i < n; ++i) nchild[p[i]]++;
    t.b0.clear();
    t.b1.clear();
    t.branch_of.assign(n, 0);
    for (int32_t i = 0; i < n; ++i) {
        bool start = (i == 0) || !(p[i] == i - 1 && nchild[i - 1] == 1);
        if (start) {
            if (!t.b0.empty()) t.b1.push_back(i - 1);
            t.b0.push_back(i);
        }
        t.branch_of[i] = (int32_t)t.b0.size() - 1;
    }
    t.b1.push_back(n - 1);
    const int32_t nb = (int32_t)t.b0.size();
    t.bpar.assign(nb, -1);
    std::vector<int32_t> cnt(nb, 0);
    for (int32_t b = 1; b < nb; ++b) {
        t.bpar[b] = t.branch_of[p[t.b0[b]]];
        cnt[t.bpar[b]]++;
    }
    t.child_off.assign(nb + 1, 0);
    for (int32_t b = 0; b < nb; ++b) t.child_off[b + 1] = t.child_off[b] + cnt[b];
    t.child.assign(t.child_off[nb], 0);
    std::vector<int32_t> fill(nb, 0);
    for (int32_t b = 1; b < nb; ++b) {
        const int32_t q = t.bpar[b];
        t.child[t.child_off[q] + fill[q]++] = b;  // ascending b, hence ascending base
    }
    t.height.assign(nb, 0);
    for (int32_t b = nb - 1; b >= 0; --b)
        for (int32_t c = t.child_off[b]; c < t.child_off[b + 1]; ++c)
            t.height[b] = std::max(t.height[b], t.height[t.child[c]] + 1);
    t.depth.assign(nb, 0);
    for (int32_t b = 1; b < nb; ++b) t.depth[b] = t.depth[t.bpar[b]] + 1;
    t.max_height = *std::max_element(t.height.begin(), t.height.end());
    t.max_depth = *std::max_element(t.depth.begin(), t.depth.end());
}

// ---------------------------------------------------------------------------
// Elimination schedule of the contraction solver for one neuron.
//
// The tree system is solved by Gaussian elimination in an order that
// contracts the tree in rounds (parallel tree contraction, Miller and Reif:
// "rake" leaves and "compress" chains). A round eliminates a set of
// compartments of current degree <= 2 whose pairwise distance in the current
// tree is at least 3, so that every surviving compartment has at most one
// eliminated neighbour in the round: one barrier per round suffices, and each
// update of a survivor has a single writer. Eliminating k with neighbours n1,
// n2 adds -A[n,k]^2/A[k,k] to each neighbour's diagonal, -A[n,k] r_k/A[k,k]
// to its right-hand side, and, when both exist, links n1 and n2 with the
// coupling -A[n1,k] A[k,n2]/A[k,k] (n2 becomes a child of n1). Back
// substitution visits the rounds in reverse. The order depends only on the
// neuron's parent vector, so results do not depend on packing.
// ---------------------------------------------------------------------------
struct Elim {
    int32_t k, n1, n2;  // neuron-local; n1 / n2 = -1 when absent
    bool n1_parent;     // n1 is k's current parent (else a child, or absent)
    bool f1, f2;        // the coupling to n1 / n2 was made by an earlier
                        // elimination (else it is the off-diagonal)
};

void contraction_schedule(const int32_t *p, int32_t n, std::vector<Elim> &items,
                          std::vector<int32_t> &round_off) {
    items.clear();
    round_off.assign(1, 0);
    std::vector<int32_t> cp(p, p + n), fc(n, -1), ns(n, -1), ps(n, -1), nch(n, 0), stamp(n, 0);
    std::vector<uint8_t> filled(n, 0);  // coupling to the current parent made by a fill
    auto link = [&](int32_t c, int32_t par) {  // c becomes the first child of par
        cp[c] = par;
        ps[c] = -1;
        ns[c] = fc[par];
        if (fc[par] >= 0) ps[fc[par]] = c;
        fc[par] = c;
        nch[par]++;
    };
    auto unlink = [&](int32_t c) {  // detach c from its parent
        const int32_t par = cp[c];
        if (ps[c] >= 0) ns[ps[c]] = ns[c]; else fc[par] = ns[c];
        if (ns[c] >= 0) ps[ns[c]] = ps[c];
        nch[par]--;
        cp[c] = -1;
        ps[c] = ns[c] = -1;
    };
    for (int32_t i = n - 1; i >= 1; --i) link(i, p[i]);  // children in ascending order
    std::vector<int32_t> alive(n), next, sel;
    for (int32_t i = 0; i < n; ++i) alive[i] = n - 1 - i;  // descending index
    int32_t round = 0;
    auto deg = [&](int32_t v) { return nch[v] + (cp[v] >= 0 ? 1 : 0); };
    auto mark = [&](int32_t v) {  // v and every compartment within distance 2
        auto mark1 = [&](int32_t u) {
            stamp[u] = round;
            if (cp[u] >= 0) stamp[cp[u]] = round;
            for (int32_t c = fc[u]; c >= 0; c = ns[c]) stamp[c] = round;
        };
        mark1(v);
        if (cp[v] >= 0) mark1(cp[v]);
        for (int32_t c = fc[v]; c >= 0; c = ns[c]) mark1(c);
    };
    while (!alive.empty()) {
        ++round;
        sel.clear();
        for (int pass = 0; pass < 2; ++pass)  // leaves (and lone roots) first, then chains
            for (int32_t v : alive) {
                if (stamp[v] == round) continue;
                const int d = deg(v);
                if (pass == 0 ? d <= 1 : d == 2) {
                    sel.push_back(v);
                    mark(v);
                }
            }
        for (int32_t k : sel) {
            Elim e{k, -1, -1, false, false, false};
            const int32_t par = cp[k];
            const int32_t c1 = fc[k], c2 = c1 >= 0 ? ns[c1] : -1;
            if (par >= 0) {
                e.n1 = par;
                e.n1_parent = true;
                e.n2 = c1;  // at most one child
                e.f1 = filled[k];
                e.f2 = c1 >= 0 && filled[c1];
                unlink(k);
                if (c1 >= 0) {
                    unlink(c1);
                    link(c1, par);
                    filled[c1] = 1;
                }
            } else if (c1 >= 0) {
                if (c2 >= 0) {  // a root with two children: c2 hangs off c1
                    e.n1 = c1;
                    e.n2 = c2;
                    e.f1 = filled[c1];
                    e.f2 = filled[c2];
                    unlink(c1);
                    unlink(c2);
                    link(c2, c1);
                    filled[c2] = 1;
                } else {  // a root with one child: the child becomes the root
                    e.n2 = c1;
                    e.f2 = filled[c1];
                    unlink(c1);
                }
            }
            items.push_back(e);
            stamp[k] = -1;  // eliminated
        }
        next.clear();
        for (int32_t v : alive)
            if (stamp[v] != -1) next.push_back(v);
        alive.swap(next);
        round_off.push_back((int32_t)items.size());
    }
}

void features(const NeuronTopo &t, const uint8_t *mech, int32_t nsyn, int32_t nseg,
              float *f) {
    const int32_t nb = (int32_t)t.b0.size();
    int32_t maxlen = 0, leaves = 0, maxch = 0;
    double sumsq = 0;
    std::vector<int32_t> bw(t.max_height + 1, 0), fw(t.max_depth + 1, 0),
        width(t.max_depth + 1, 0);
    std::vector<int64_t> path(nb, 0);
    int64_t crit = 0;
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t len = t.b1[b] - t.b0[b] + 1;
        const int32_t nc = t.child_off[b + 1] - t.child_off[b];
        maxlen = std::max(maxlen, len);
        maxch = std::max(maxch, nc);
        if (nc == 0) leaves++;
        sumsq += (double)len * len;
        bw[t.height[b]] = std::max(bw[t.height[b]], len + nc);
        fw[t.depth[b]] = std::max(fw[t.depth[b]], len);
        width[t.depth[b]]++;
        path[b] = len + (t.bpar[b] >= 0 ? path[t.bpar[b]] : 0);
        crit = std::max(crit, path[b]);
    }
    int64_t sbw = 0, sfw = 0;
    for (int32_t v : bw) sbw += v;
    for (int32_t v : fw) sfw += v;
    int32_t nhh = 0;
    for (int32_t i = 0; i < t.n; ++i) nhh += mech[i] ? 1 : 0;
    f[0] = (float)t.n;
    f[1] = (float)nb;
    f[2] = (float)(t.max_depth + 1);
    f[3] = (float)maxlen;
    f[4] = (float)t.n / (float)nb;
    f[5] = (float)crit;
    f[6] = (float)sbw;
    f[7] = (float)sfw;
    f[8] = (float)leaves;
    f[9] = (float)nsyn;
    f[10] = (float)nseg;
    f[11] = (float)nhh;
    f[12] = (float)maxch;
    f[13] = (float)*std::max_element(width.begin(), width.end());
    f[14] = (float)(sumsq / nb);
    f[15] = (float)(t.child_off[1] - t.child_off[0]);
}

// ---------------------------------------------------------------------------
// Launch variant and device buffers.
// ---------------------------------------------------------------------------
constexpr int kClasses = 3;
constexpr int64_t kRingMin = 32;  // spike ring rows (epochs) at least

// One launch of the epoch kernel over the packs of one size class: its
// workgroup count, dynamic LDS, and where its lists start in the shared
// offset / list arrays.
struct Launch {
    int n_wg = 0;
    int threads = 256;
    size_t lds = 256;
    int32_t off0 = 0, list0 = 0;
    bool resident = false;  // every pack in LDS with every compartment register-resident
};

struct Variant {
    int threads = 256;
    int pack_comps = 1024;  // plain packing: target compartments per pack
    int comp_cap = 0;       // count / learned packing: cap on a pack's compartments, 0 = none
    int lds_limit = 64 * 1024;  // bytes of LDS per workgroup
    int sched = SIM_SCHED_PERSISTENT;
    int nclass = 2;  // LDS size classes in use (1..kClasses)
    int cls_thr = 1;  // class c launches threads << (c * cls_thr) (at most the launch bound)
    bool res_cap = false;  // count / learned packing: no pack of class c holds more
                           // compartments than its threads' register slots
                           // (kResident per thread), so its launch keeps every
                           // compartment's gates and constants in registers

};

template <typename X>
struct DBuf {
    X *p = nullptr;
    int64_t n = 0;
    void free_() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(int64_t count) {
        free_();
        n = count;
        HIPCHK(hipMalloc((void **)&p, sizeof(X) * (count > 0 ? count : 1)));
    }
    void upload(const std::vector<X> &v) {
        alloc((int64_t)v.size());
        if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), sizeof(X) * v.size(), hipMemcpyHostToDevice));
    }
};

}  // namespace

struct sim {
    // inputs (copied)
    sim_params_t P{};
    sim_channels_t CH{};
    int32_t N = 0;
    int64_t C = 0, S = 0;
    std::vector<int64_t> off;
    std::vector<int32_t> parent, detector, pre, post, pcomp, delay;
    std::vector<double> length, diam, iext, weight;
    std::vector<uint8_t> mech;
    std::vector<float> cost_model;
    std::vector<double> ncost;  // per-neuron costs given for learned packing
    int precision = 1;
    int solver = 0;
    int E = 40;
    int tsize = 4;  // sizeof gating type

    // analysis
    std::vector<NeuronTopo> topo;
    std::vector<float> feat;           // [N][16]
    std::vector<int32_t> nsyn_of;      // synapses per post neuron
    std::vector<int64_t> syn_by_post;  // synapse ids grouped by post, ascending id
    std::vector<int64_t> syn_post_off; // [N+1]
    std::vector<double> cost;          // packing cost per neuron
    // contraction solver: per neuron, its items (neuron-local, in round
    // order, at the neuron's compartment offsets) and round offsets
    std::vector<uint64_t> citems;
    std::vector<int32_t> croff;
    std::vector<int64_t> croff0;       // [N+1] into croff

    // layout: the host arrays build_layout produces, held until uploaded
    struct HostLayout {
        std::vector<uint32_t> topo, cnb;
        std::vector<int32_t> lparent, nid, ndet, lvl, spre, sdel;
        std::vector<double> len, dia, w64, iext64;
        std::vector<int64_t> ncomp0;
        std::vector<uint16_t> scomp, sseg, chl, fws;
        std::vector<Branch> brs;
        std::vector<uint64_t> cit;
    } hl;
    bool planned_only = false;  // laid out on the host, no device (sim_plan_create)
    Variant var;
    std::vector<int32_t> order;        // packed position -> input neuron
    std::vector<int64_t> comp_perm;    // packed compartment -> input compartment
    std::vector<int64_t> syn_perm;     // packed synapse -> input synapse id
    std::vector<PackDesc> packs;
    std::vector<double> pack_cost;
    std::vector<int32_t> pack_of_neuron;  // input neuron -> pack
    std::vector<int32_t> wg_off, wg_list;
    int n_wg = 0;
    size_t lds_bytes = 0;
    Launch launch[kClasses];     // one launch per size class
    hipStream_t side[kClasses] = {};  // streams of classes 1.. (class 0: main stream)
    hipEvent_t ev_fork = nullptr, ev_join[kClasses] = {};
    int64_t scratch_bytes = 0;
    int max_lds = 64 * 1024;
    int n_cu = 256;

    // device
    hipStream_t stream = nullptr;
    bool own_stream = false;
    DBuf<PackDesc> d_packs;
    DBuf<int32_t> d_wg_off, d_wg_list, d_spre, d_sdelay, d_nid, d_ndet, d_lvl, d_lparent;
    DBuf<double> d_V, d_cdt, d_e, d_len, d_diam, d_w64, d_iext64, d_q;
    DBuf<char> d_gm, d_gh, d_gn, d_af, d_sg, d_sw, d_niext, d_scratch;
    DBuf<uint32_t> d_topo, d_cnb;
    DBuf<uint16_t> d_scomp, d_sseg, d_chl;
    DBuf<Branch> d_br;
    DBuf<uint16_t> d_fw;
    DBuf<uint64_t> d_cit;
    DBuf<int64_t> d_ncomp0, d_epoch;
    DBuf<uint64_t> d_ring, d_ptime;
    double q = 0;

    // spike history: a device ring of ring_rows epoch rows (enough for the
    // longest delay), drained after every stretch of at most ring_rows epochs
    // into pinned staging (two slots, so the host reads one while the device
    // fills the other) and from there into the host spike list
    int32_t ring_rows = 0;
    uint64_t *h_stage[2] = {nullptr, nullptr};
    hipEvent_t ev_stage[2] = {};
    struct Drain {
        int64_t first_epoch = 0;
        int32_t rows = 0;
        int64_t lo = 0, hi = 0;  // spikes of steps (lo, hi]
        bool pending = false;
    } drain[2];
    int drain_slot = 0;
    std::vector<sim_spike_t> spikes;      // sorted by (step, neuron)
    // sim_step_noalloc: the call's spikes go to the caller's buffer instead
    sim_spike_t *sink = nullptr;
    int64_t sink_cap = 0, sink_n = 0;
    void *na_scratch = nullptr;       // this device's fixed scratch array
    char *scratch_override = nullptr;  // global-pack state base for the launches
    int64_t scratch_total = 0;         // bytes the global packs' slices need
    std::vector<std::vector<int32_t>> by_t;  // scan scratch, one list per epoch step

    // time
    int64_t step = 0;
    hipGraph_t graph1 = nullptr, graphK = nullptr;
    hipGraphExec_t exec1 = nullptr, execK = nullptr;
    int graphK_epochs = 8;
    bool kt_on = false;
    double kt_ms = 0;
    int64_t kt_launches = 0;
    // launch timing: HIP event pairs around each epoch (or graph replay of
    // kt_ep[u] epochs) on the simulator's stream, taken from a pool and read
    // back once per sim_step; each size-class launch times itself on the
    // device (d_ktimer, 8 words per class, see EpochArgs::ktimer)
    std::vector<hipEvent_t> kt_pool;
    std::vector<int> kt_ep;
    int kt_used = 0;
    DBuf<uint64_t> d_ktimer;
    double kt_cls_ms[kClasses] = {};
    int64_t kt_cls_n[kClasses] = {};
    int64_t cls_comps[kClasses] = {};  // compartments of each size class
    int64_t kt_cls_upd[kClasses] = {};  // compartment-updates launched while timing is on
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double tick_ns = 10.0;

    std::string err, config;
};

namespace {

// ---------------------------------------------------------------------------
// Validation: everything is checked before any device allocation.
// ---------------------------------------------------------------------------
void validate(const sim_params_t *P, const sim_morphology_t *M, const sim_channels_t *CH,
              const sim_synapses_t *SY) {
    if (!P || !M || !CH || !SY) throw fail(SIM_EINVAL, "null argument");
    if (!(P->dt_ms > 0) || !std::isfinite(P->dt_ms)) throw fail(SIM_EINVAL, "dt_ms must be > 0");
    if (!(P->theta == 0.5 || P->theta == 1.0))
        throw fail(SIM_EINVAL, "theta must be 0.5 or 1.0 (got %g)", P->theta);
    if (!(P->tau_syn_ms > 0) || !std::isfinite(P->tau_syn_ms))
        throw fail(SIM_EINVAL, "tau_syn_ms must be > 0");
    for (double v : {P->e_syn_mV, P->v_thresh_mV, P->v_init_mV, CH->cm_uF_cm2, CH->ra_ohm_cm,
                     CH->gnabar, CH->gkbar, CH->gl, CH->ena, CH->ek, CH->el, CH->g_pas, CH->e_pas})
        if (!std::isfinite(v)) throw fail(SIM_EINVAL, "non-finite parameter");
    if (!(CH->cm_uF_cm2 > 0) || !(CH->ra_ohm_cm > 0))
        throw fail(SIM_EINVAL, "cm and ra must be > 0");
    if (P->precision != SIM_FP64 && P->precision != SIM_FP32_GATING)
        throw fail(SIM_EINVAL, "unknown precision %d", P->precision);
    if (P->solver != SIM_SOLVE_EXACT && P->solver != SIM_SOLVE_FAST &&
        P->solver != SIM_SOLVE_CONTRACT)
        throw fail(SIM_EINVAL, "unknown solver %d", P->solver);
    if (P->packing < SIM_PACK_PLAIN || P->packing > SIM_PACK_LEARNED)
        throw fail(SIM_EINVAL, "unknown packing %d", P->packing);
    if (P->sched < SIM_SCHED_AUTO || P->sched > SIM_SCHED_DISPATCH)
        throw fail(SIM_EINVAL, "unknown sched %d", P->sched);
    if (P->threads != 0 && (P->threads < 64 || P->threads > 1024 || P->threads % 64))
        throw fail(SIM_EINVAL, "threads must be a multiple of 64 in [64, 1024]");
    if (P->pack_comps < 0 || P->lds_comps < 0) throw fail(SIM_EINVAL, "negative size");
    if (P->lds_classes < 0 || P->lds_classes > 3)
        throw fail(SIM_EINVAL, "lds_classes must be 0 (default) or 1..3");
    if (M->n_neurons < 1) throw fail(SIM_EINVAL, "n_neurons must be >= 1");
    if (!M->comp_offset || !M->parent || !M->length_um || !M->diam_um || !M->mech ||
        !M->detector || !M->i_ext_nA)
        throw fail(SIM_EINVAL, "null morphology array");
    const int32_t N = M->n_neurons;
    if (M->comp_offset[0] != 0) throw fail(SIM_EINVAL, "comp_offset[0] must be 0");
    for (int32_t j = 0; j < N; ++j) {
        const int64_t b = M->comp_offset[j], e = M->comp_offset[j + 1];
        const int64_t n = e - b;
        if (n < 1) throw fail(SIM_EINVAL, "neuron %d has no compartments", j);
        if (n > 32767) throw fail(SIM_EINVAL, "neuron %d has %lld > 32767 compartments", j, (long long)n);
        if (M->parent[b] != -1) throw fail(SIM_EINVAL, "neuron %d: parent[0] must be -1", j);
        for (int64_t i = 1; i < n; ++i) {
            const int32_t p = M->parent[b + i];
            if (p < 0 || p >= i)
                throw fail(SIM_EINVAL, "neuron %d compartment %lld: parent %d not in [0, %lld)", j,
                           (long long)i, p, (long long)i);
        }
        for (int64_t i = 0; i < n; ++i) {
            const double L = M->length_um[b + i], d = M->diam_um[b + i];
            if (!(L > 0) || !(d > 0) || !std::isfinite(L) || !std::isfinite(d))
                throw fail(SIM_EINVAL, "neuron %d compartment %lld: bad geometry", j, (long long)i);
            if (M->mech[b + i] > 1) throw fail(SIM_EINVAL, "mech must be 0 or 1");
        }
        if (M->detector[j] < 0 || M->detector[j] >= n)
            throw fail(SIM_EINVAL, "neuron %d: detector out of range", j);
        if (!std::isfinite(M->i_ext_nA[j])) throw fail(SIM_EINVAL, "non-finite i_ext");
    }
    if (SY->n < 0) throw fail(SIM_EINVAL, "negative synapse count");
    if (SY->n > 0 && (!SY->pre || !SY->post || !SY->post_comp || !SY->delay_steps || !SY->weight_uS))
        throw fail(SIM_EINVAL, "null synapse array");
    int64_t mind = INT64_MAX;
    for (int64_t k = 0; k < SY->n; ++k) {
        const int32_t a = SY->pre[k], b = SY->post[k];
        if (a < 0 || a >= N || b < 0 || b >= N) throw fail(SIM_EINVAL, "synapse %lld: neuron out of range", (long long)k);
        const int64_t nb = M->comp_offset[b + 1] - M->comp_offset[b];
        if (SY->post_comp[k] < 0 || SY->post_comp[k] >= nb)
            throw fail(SIM_EINVAL, "synapse %lld: compartment out of range", (long long)k);
        if (SY->delay_steps[k] < 1) throw fail(SIM_EINVAL, "synapse %lld: delay must be >= 1 step", (long long)k);
        if (!(SY->weight_uS[k] >= 0) || !std::isfinite(SY->weight_uS[k]))
            throw fail(SIM_EINVAL, "synapse %lld: weight must be finite and >= 0", (long long)k);
        mind = std::min<int64_t>(mind, SY->delay_steps[k]);
    }
    if (P->epoch_steps < 0 || P->epoch_steps > 64)
        throw fail(SIM_EINVAL, "epoch_steps must be in [0, 64]");
    if (P->epoch_steps > 0 && SY->n > 0 && P->epoch_steps > mind)
        throw fail(SIM_EINVAL, "epoch_steps %d exceeds the smallest delay %lld", P->epoch_steps,
                   (long long)mind);
    if (P->packing == SIM_PACK_LEARNED && P->cost_model) {
        for (int64_t i = 0; i < kMlpParams; ++i)
            if (!std::isfinite(P->cost_model[i])) throw fail(SIM_EINVAL, "non-finite cost model");
    }
    if (P->packing == SIM_PACK_LEARNED && P->neuron_cost) {
        for (int32_t j = 0; j < M->n_neurons; ++j)
            if (!std::isfinite(P->neuron_cost[j]) || !(P->neuron_cost[j] > 0.0))
                throw fail(SIM_EINVAL, "neuron %d: cost must be finite and > 0", j);
    }
}

void copy_inputs(sim_t *s, const sim_params_t *P, const sim_morphology_t *M,
                 const sim_channels_t *CH, const sim_synapses_t *SY) {
    s->P = *P;
    s->CH = *CH;
    s->N = M->n_neurons;
    s->C = M->comp_offset[s->N];
    s->S = SY->n;
    s->off.assign(M->comp_offset, M->comp_offset + s->N + 1);
    s->parent.assign(M->parent, M->parent + s->C);
    s->length.assign(M->length_um, M->length_um + s->C);
    s->diam.assign(M->diam_um, M->diam_um + s->C);
    s->mech.assign(M->mech, M->mech + s->C);
    s->detector.assign(M->detector, M->detector + s->N);
    s->iext.assign(M->i_ext_nA, M->i_ext_nA + s->N);
    if (s->S) {
        s->pre.assign(SY->pre, SY->pre + s->S);
        s->post.assign(SY->post, SY->post + s->S);
        s->pcomp.assign(SY->post_comp, SY->post_comp + s->S);
        s->delay.assign(SY->delay_steps, SY->delay_steps + s->S);
        s->weight.assign(SY->weight_uS, SY->weight_uS + s->S);
    }
    if (P->cost_model) s->cost_model.assign(P->cost_model, P->cost_model + kMlpParams);
    if (P->packing == SIM_PACK_LEARNED && P->neuron_cost)
        s->ncost.assign(P->neuron_cost, P->neuron_cost + s->N);
    s->P.neuron_cost = nullptr;  // copied; the caller's array need not outlive the call
    s->precision = P->precision;
    s->solver = P->solver;
    s->tsize = P->precision == SIM_FP64 ? 8 : 4;
    int64_t mind = 64;
    for (int64_t k = 0; k < s->S; ++k) mind = std::min<int64_t>(mind, s->delay[k]);
    s->E = P->epoch_steps > 0 ? P->epoch_steps : (int)mind;
    // ring rows: delivery in epoch k reads epochs k - ceil((delay + 1) / E)
    // .. k - 1 while epoch k writes its own row, so that many + 1 rows must be
    // distinct; at least kRingMin so that draining stays rare
    int64_t maxd = 0;
    for (int64_t k = 0; k < s->S; ++k) maxd = std::max<int64_t>(maxd, s->delay[k]);
    const int64_t need = (maxd + 1 + s->E - 1) / s->E + 1;
    const int64_t rows = std::max<int64_t>(need, kRingMin);
    if (rows * (int64_t)s->N * 8 > (int64_t)16 << 30)
        throw fail(SIM_ENOMEM, "spike ring of %lld epochs x %d neurons exceeds 16 GiB (longest delay "
                   "%lld steps)", (long long)rows, s->N, (long long)maxd);
    s->ring_rows = (int32_t)rows;
}

void analyse_all(sim_t *s) {
    s->topo.resize(s->N);
    s->nsyn_of.assign(s->N, 0);
    for (int64_t k = 0; k < s->S; ++k) s->nsyn_of[s->post[k]]++;
    s->syn_post_off.assign(s->N + 1, 0);
    for (int32_t j = 0; j < s->N; ++j) s->syn_post_off[j + 1] = s->syn_post_off[j] + s->nsyn_of[j];
    s->syn_by_post.assign(s->S, 0);
    std::vector<int64_t> fill(s->N, 0);
    for (int64_t k = 0; k < s->S; ++k) {
        const int32_t j = s->post[k];
        s->syn_by_post[s->syn_post_off[j] + fill[j]++] = k;
    }
    s->feat.assign((size_t)s->N * kFeat, 0.0f);
    std::vector<int32_t> seen;
    for (int32_t j = 0; j < s->N; ++j) {
        const int64_t b = s->off[j];
        const int32_t n = (int32_t)(s->off[j + 1] - b);
        analyse(s->parent.data() + b, n, s->topo[j]);
        // distinct target compartments
        seen.clear();
        for (int64_t q = s->syn_post_off[j]; q < s->syn_post_off[j + 1]; ++q)
            seen.push_back(s->pcomp[s->syn_by_post[q]]);
        std::sort(seen.begin(), seen.end());
        const int32_t nseg = (int32_t)(std::unique(seen.begin(), seen.end()) - seen.begin());
        features(s->topo[j], s->mech.data() + b, s->nsyn_of[j], nseg, &s->feat[(size_t)j * kFeat]);
    }
    s->citems.clear();
    s->croff.clear();
    s->croff0.assign(1, 0);
    if (s->solver == SIM_SOLVE_CONTRACT) {
        s->citems.resize(s->C);
        std::vector<Elim> items;
        std::vector<int32_t> roff;
        for (int32_t j = 0; j < s->N; ++j) {
            const int64_t b = s->off[j];
            const int32_t n = (int32_t)(s->off[j + 1] - b);
            contraction_schedule(s->parent.data() + b, n, items, roff);
            for (int32_t q = 0; q < n; ++q) {
                const Elim &e = items[q];
                s->citems[b + q] = make_item((uint32_t)e.k, e.n1_parent,
                                             e.n1 < 0 ? kNoNb : (uint32_t)e.n1,
                                             e.n2 < 0 ? kNoNb : (uint32_t)e.n2, e.f1, e.f2);
            }
            s->croff.insert(s->croff.end(), roff.begin(), roff.end());
            s->croff0.push_back((int64_t)s->croff.size());
        }
    }
}

int32_t contraction_rounds(const sim_t *s, int32_t j) {
    return s->croff0.size() > (size_t)j + 1 ? (int32_t)(s->croff0[j + 1] - s->croff0[j] - 1) : 0;
}

bool learned_costs(const sim_t *s) {
    return s->P.packing == SIM_PACK_LEARNED && (!s->cost_model.empty() || !s->ncost.empty());
}

void compute_cost(sim_t *s) {
    s->cost.assign(s->N, 0.0);
    if (s->P.packing == SIM_PACK_LEARNED && !s->ncost.empty()) {
        s->cost = s->ncost;
    } else if (learned_costs(s)) {
        std::vector<float> pred(s->N);
        hipError_t e = mlp_forward(s->cost_model.data(), s->feat.data(), s->N, pred.data());
        if (e != hipSuccess) throw fail(SIM_EDEVICE, "cost model inference failed: %s", hipGetErrorString(e));
        for (int32_t j = 0; j < s->N; ++j) s->cost[j] = std::exp((double)pred[j]);
    } else {
        for (int32_t j = 0; j < s->N; ++j) s->cost[j] = (double)(s->off[j + 1] - s->off[j]);
    }
}

// ---------------------------------------------------------------------------
// Packing and layout.
// ---------------------------------------------------------------------------
int64_t state_bytes(const sim_t *s, int64_t n, int64_t ns, int64_t k) {
    if (s->solver == SIM_SOLVE_CONTRACT) ++n;  // the spare compartment (make_citem)
    return s->tsize == 8 ? pack_state_bytes<double>(n, ns, k) : pack_state_bytes<float>(n, ns, k);
}
// LDS bytes of a pack's tables. The contraction solver stages no branch
// records, forward order, child list or level offsets: it reads none of them
// in its steps (its assembly takes the children word, and its rare fallbacks
// read the branch tables from global memory).
int64_t table_bytes(const sim_t *s, int64_t nbr, int64_t nch, int64_t nlev, int64_t ns,
                    int64_t n, int64_t nrnd, int64_t nst) {
    if (s->solver == SIM_SOLVE_CONTRACT) nbr = nch = nlev = 0;
    return s->tsize == 8 ? pack_table_bytes<double>(nbr, nch, nlev, ns, n, nrnd, nst)
                         : pack_table_bytes<float>(nbr, nch, nlev, ns, n, nrnd, nst);
}

void build_layout(sim_t *s, Variant v) {
    v.threads = std::min(v.threads, s->tsize == 8 ? kMaxThreadsF64 : kMaxThreadsF32);
    s->var = v;
    const int32_t N = s->N;
    // neuron order
    s->order.resize(N);
    std::iota(s->order.begin(), s->order.end(), 0);
    // count and learned packing fill their packs in decreasing compartment
    // count (ties by cost); the cost then orders the packs
    const bool learned = learned_costs(s);
    if (s->P.packing != SIM_PACK_PLAIN)
        std::stable_sort(s->order.begin(), s->order.end(), [&](int32_t a, int32_t b) {
            const int64_t na = s->off[a + 1] - s->off[a], nb = s->off[b + 1] - s->off[b];
            return na != nb ? na > nb : s->cost[a] > s->cost[b];
        });
    struct P0 {
        int32_t first, count;
        int64_t ncomp, nsyn;
        int32_t nbr;
    };
    std::vector<P0> pk;
    // size classes: LDS budgets lds_limit, 2x, 4x, ... capped at the CU's LDS;
    // the last class in use also takes the packs that fit nowhere (their
    // state in global scratch, their tables in LDS)
    const int ncls = std::max(1, std::min(kClasses, v.nclass));
    int64_t cls_budget[kClasses];
    for (int c = 0; c < kClasses; ++c)
        cls_budget[c] = std::min<int64_t>((int64_t)v.lds_limit << c, s->max_lds);
    if (s->P.packing == SIM_PACK_PLAIN) {
        // consecutive neurons in generation order, up to pack_comps compartments
        P0 cur{0, 0, 0, 0, 0};
        for (int32_t q = 0; q < N; ++q) {
            const int32_t j = s->order[q];
            const int64_t n = s->off[j + 1] - s->off[j];
            const int32_t nb = (int32_t)s->topo[j].b0.size();
            const bool fits = cur.count == 0 ||
                              (cur.ncomp + n <= v.pack_comps && cur.count < 1024 &&
                               cur.ncomp + n <= 32766 && cur.nbr + nb <= 32766);
            if (!fits) {
                pk.push_back(cur);
                cur = P0{q, 0, 0, 0, 0};
            }
            cur.count++;
            cur.ncomp += n;
            cur.nsyn += s->nsyn_of[j];
            cur.nbr += nb;
        }
        pk.push_back(cur);
    } else {
        // Best-fit decreasing: neurons by decreasing size, each into the open
        // pack with the least LDS left that still holds it (tables and
        // state, exactly as the kernel lays them out); a neuron that fits no
        // open pack opens one in the smallest size class that holds it
        // alone. A pack's workgroup allocates its class's budget whatever it
        // holds, so filling packs to the budget raises the compartments
        // resident per CU. Packs are then ordered by decreasing cost (the
        // dispatch order of the workgroups, and the LPT order of persistent
        // ones): summed compartment counts, or, with the learned model, the
        // largest predicted time among the pack's neurons (its neurons run
        // side by side, so the slowest one bounds the pack's sweeps).
        struct Bin {
            std::vector<int32_t> members;
            int64_t n = 0, ns = 0;
            int32_t nbr = 0, nch = 0, maxh = 0, maxd = 0, maxr = 0;
            int cls = 0;
            double cost = 0.0;
        };
        // (contraction: room for the staged tail items, about one in
        // kTailShare compartments)
#ifndef MMH_TAIL_SHARE
#define MMH_TAIL_SHARE 8
#endif
        const int64_t tail_share = MMH_TAIL_SHARE;
        const int thr_max = s->tsize == 8 ? kMaxThreadsF64 : kMaxThreadsF32;
        auto res_cap_of = [&](int cls) -> int64_t {
            return v.res_cap ? (int64_t)kResident * std::min(v.threads << (cls * v.cls_thr), thr_max)
                             : INT64_MAX;
        };
        auto bytes_of = [&](int64_t n, int64_t ns, int32_t nbr, int32_t nch, int32_t maxh,
                            int32_t maxd, int32_t maxr, int64_t k) -> int64_t {
            const int64_t nlev = (int64_t)maxh + maxd + 4;
            const int64_t nst = (maxr > 0 && tail_share > 0) ? n / tail_share : 0;
            return table_bytes(s, nbr, nch, nlev, ns, n, maxr, nst) + state_bytes(s, n, ns, k);
        };
        std::vector<Bin> bins;
        std::multimap<int64_t, int32_t> open;  // LDS bytes left -> bin
        std::vector<std::multimap<int64_t, int32_t>::iterator> where;
        const int64_t base_bytes = bytes_of(0, 0, 0, 0, 0, 0, 0, 0);
        for (int32_t q = 0; q < N; ++q) {
            const int32_t j = s->order[q];
            const NeuronTopo &t = s->topo[j];
            const int64_t n = s->off[j + 1] - s->off[j], ns = s->nsyn_of[j];
            const int32_t nb = (int32_t)t.b0.size();
            const int32_t nr = contraction_rounds(s, j);
            const int64_t alone = bytes_of(n, ns, nb, nb - 1, t.max_height, t.max_depth, nr, 1);
            int32_t chosen = -1;
            int tries = 0;
            for (auto it = open.lower_bound(alone - base_bytes); it != open.end() && tries < 32;
                 ++it, ++tries) {
                const Bin &B = bins[it->second];
                if (B.members.size() >= 1024 || B.n + n > 32766 || B.nbr + nb > 32766 ||
                    (v.comp_cap > 0 && B.n + n > v.comp_cap) || B.n + n > res_cap_of(B.cls))
                    continue;
                const int64_t with = bytes_of(B.n + n, B.ns + ns, B.nbr + nb, B.nch + nb - 1,
                                              std::max(B.maxh, t.max_height),
                                              std::max(B.maxd, t.max_depth), std::max(B.maxr, nr),
                                              (int64_t)B.members.size() + 1);
                if (with <= cls_budget[B.cls]) {
                    chosen = it->second;
                    break;
                }
            }
            if (chosen < 0) {
                Bin B;
                while (B.cls + 1 < ncls && (alone > cls_budget[B.cls] || n > res_cap_of(B.cls)))
                    ++B.cls;
                bins.push_back(B);
                where.push_back(open.end());
                chosen = (int32_t)bins.size() - 1;
            } else {
                open.erase(where[chosen]);
                where[chosen] = open.end();
            }
            Bin &B = bins[chosen];
            B.members.push_back(j);
            B.n += n;
            B.ns += ns;
            B.nbr += nb;
            B.nch += nb - 1;
            B.maxh = std::max(B.maxh, t.max_height);
            B.maxd = std::max(B.maxd, t.max_depth);
            B.maxr = std::max(B.maxr, nr);
            B.cost = learned ? std::max(B.cost, s->cost[j]) : B.cost + s->cost[j];
            const int64_t used = bytes_of(B.n, B.ns, B.nbr, B.nch, B.maxh, B.maxd, B.maxr,
                                          (int64_t)B.members.size());
            if (used <= cls_budget[B.cls])  // (a pack too large for LDS stays alone)
                where[chosen] = open.emplace(cls_budget[B.cls] - used, chosen);
        }
        std::vector<int32_t> bo(bins.size());
        std::iota(bo.begin(), bo.end(), 0);
        std::stable_sort(bo.begin(), bo.end(),
                         [&](int32_t a, int32_t b) { return bins[a].cost > bins[b].cost; });
        int32_t q = 0;
        for (int32_t b : bo) {
            P0 cur{q, 0, 0, 0, 0};
            for (int32_t j : bins[b].members) {
                s->order[q++] = j;
                cur.count++;
                cur.ncomp += s->off[j + 1] - s->off[j];
                cur.nsyn += s->nsyn_of[j];
                cur.nbr += (int32_t)s->topo[j].b0.size();
            }
            pk.push_back(cur);
        }
    }
    const int npk = (int)pk.size();
    s->packs.assign(npk, PackDesc{});
    s->pack_cost.assign(npk, 0.0);
    s->pack_of_neuron.assign(N, 0);

    s->hl = sim_t::HostLayout{};
    auto &topo = s->hl.topo;
    auto &cnb = s->hl.cnb;  // children words (make_children)
    auto &lparent = s->hl.lparent, &nid = s->hl.nid, &ndet = s->hl.ndet, &lvl = s->hl.lvl;
    auto &len = s->hl.len, &dia = s->hl.dia, &w64 = s->hl.w64, &iext64 = s->hl.iext64;
    auto &ncomp0 = s->hl.ncomp0;
    auto &spre = s->hl.spre, &sdel = s->hl.sdel;
    auto &scomp = s->hl.scomp, &sseg = s->hl.sseg, &chl = s->hl.chl;
    auto &brs = s->hl.brs;
    auto &fws = s->hl.fws;  // forward order: record ids
    auto &cit = s->hl.cit;  // contraction items, pack-local, by pack and round
    std::vector<int32_t> member_base;  // compartment base of each neuron in the pack
    // per-pack branch scratch (pack-local branch index = br_base + local)
    std::vector<int32_t> tb0, tb1, tpar, tch_off, tch, pos, child0;
    topo.reserve(s->C);
    cnb.reserve(s->C);
    lparent.reserve(s->C);
    len.reserve(s->C);
    dia.reserve(s->C);
    s->comp_perm.clear();
    s->comp_perm.reserve(s->C);
    s->syn_perm.clear();
    s->syn_perm.reserve(s->S);
    int64_t scratch = 0;
    int64_t lds_cls[kClasses];
    for (int c = 0; c < kClasses; ++c) lds_cls[c] = 0;
    std::vector<int> pclass(npk, 0);
    std::vector<std::pair<int64_t, int64_t>> segs;  // (local comp, synapse id)


    for (int p = 0; p < npk; ++p) {
        PackDesc d{};
        d.comp0 = (int64_t)topo.size();
        d.syn0 = (int64_t)spre.size();
        d.ncomp = (int32_t)pk[p].ncomp;
        d.nsyn = (int32_t)pk[p].nsyn;
        d.neur0 = pk[p].first;
        d.nneur = pk[p].count;
        d.br0 = (int32_t)brs.size();
        d.nbr = pk[p].nbr;
        d.ch0 = (int32_t)chl.size();
        d.lv0 = (int32_t)lvl.size();
        member_base.clear();
        tb0.clear();
        tb1.clear();
        tpar.clear();
        tch.clear();
        tch_off.assign(1, 0);
        int32_t maxh = 0, maxd = 0;
        int32_t comp_base = 0, br_base = 0;
        segs.clear();
        std::vector<int32_t> bh, bd;  // height, depth of pack-local branches
        for (int32_t k = 0; k < pk[p].count; ++k) {
            const int32_t q = pk[p].first + k;
            const int32_t j = s->order[q];
            s->pack_of_neuron[j] = p;
            s->pack_cost[p] = learned ? std::max(s->pack_cost[p], s->cost[j])
                                      : s->pack_cost[p] + s->cost[j];
            const NeuronTopo &t = s->topo[j];
            const int64_t b = s->off[j];
            const int32_t n = t.n;
            const int32_t nb = (int32_t)t.b0.size();
            maxh = std::max(maxh, t.max_height);
            maxd = std::max(maxd, t.max_depth);
            // branch-end marker per local compartment
            std::vector<int32_t> end_branch(n, -1);
            for (int32_t bb = 0; bb < nb; ++bb) end_branch[t.b1[bb]] = bb;
            // children of each compartment, ascending (parent[i] < i)
            std::vector<int32_t> nch_of(n, 0), ch1(n, -1), ch2(n, -1);
            for (int32_t i = 1; i < n; ++i) {
                const int32_t pp = s->parent[b + i];
                if (nch_of[pp] == 0) ch1[pp] = i; else if (nch_of[pp] == 1) ch2[pp] = i;
                nch_of[pp]++;
            }
            for (int32_t i = 0; i < n; ++i) {
                const bool root = i == 0;
                const uint32_t par = root ? (uint32_t)k : (uint32_t)(comp_base + s->parent[b + i]);
                const uint32_t bid = end_branch[i] >= 0 ? (uint32_t)(br_base + end_branch[i]) : kNone;
                topo.push_back(make_topo(par, s->mech[b + i] != 0, bid, root));
                cnb.push_back(nch_of[i] > 2 ? kManyChildren
                                            : make_children(ch1[i] >= 0 ? comp_base + ch1[i] : kNoNb,
                                                            ch2[i] >= 0 ? comp_base + ch2[i] : kNoNb));
                lparent.push_back(s->parent[b + i]);
                len.push_back(s->length[b + i]);
                dia.push_back(s->diam[b + i]);
                s->comp_perm.push_back(b + i);
            }
            for (int32_t bb = 0; bb < nb; ++bb) {
                tb0.push_back(comp_base + t.b0[bb]);
                tb1.push_back(comp_base + t.b1[bb]);
                tpar.push_back(bb == 0 ? (int32_t)kRootPar : comp_base + s->parent[b + t.b0[bb]]);
                for (int32_t c = t.child_off[bb]; c < t.child_off[bb + 1]; ++c)
                    tch.push_back(br_base + t.child[c]);
                tch_off.push_back((int32_t)tch.size());
                bh.push_back(t.height[bb]);
                bd.push_back(t.depth[bb]);
            }
            nid.push_back(j);
            ndet.push_back(comp_base + s->detector[j]);
            iext64.push_back(s->iext[j]);
            ncomp0.push_back(d.comp0 + comp_base);
            for (int64_t qq = s->syn_post_off[j]; qq < s->syn_post_off[j + 1]; ++qq) {
                const int64_t sid = s->syn_by_post[qq];
                segs.emplace_back((int64_t)comp_base + s->pcomp[sid], sid);
            }
            member_base.push_back(comp_base);
            comp_base += n;
            br_base += nb;
        }
        if ((int64_t)chl.size() + (int64_t)tch.size() > INT32_MAX)
            throw fail(SIM_ENOMEM, "child list too large");
        if (tch.size() > 65535) throw fail(SIM_EINVAL, "pack child list too large");
        // synapses by (local compartment, id)
        std::sort(segs.begin(), segs.end());
        for (size_t u = 0; u < segs.size(); ++u) {
            const int64_t sid = segs[u].second;
            s->syn_perm.push_back(sid);
            spre.push_back(s->pre[sid]);
            sdel.push_back(s->delay[sid]);
            w64.push_back(s->weight[sid]);
            scomp.push_back((uint16_t)segs[u].first);
            int32_t run = 0;
            if (u == 0 || segs[u].first != segs[u - 1].first) {
                size_t w = u;
                while (w < segs.size() && segs[w].first == segs[u].first) ++w;
                run = (int32_t)(w - u);
            }
            if (run > 65535) throw fail(SIM_EINVAL, "too many synapses on one compartment");
            sseg.push_back((uint16_t)run);
        }
        // levels: branches by height (backward), by depth (forward); within a
        // level, longest chains first so that the lanes of a wave finish
        // together. The backward order is also the order of the branch
        // records (a branch's id is its position).
        d.nbw = maxh + 1;
        d.nfw = maxd + 1;
        const int32_t nbr = d.nbr;
        auto nchild = [&](int32_t bb) { return tch_off[bb + 1] - tch_off[bb]; };
        auto chain_len = [&](int32_t bb, bool with_children) {
            return (tb1[bb] - tb0[bb]) + (with_children ? nchild(bb) : 0);
        };
        std::vector<int32_t> lev, order;
        order.clear();
        lvl.push_back(0);
        for (int h = 0; h < d.nbw; ++h) {
            lev.clear();
            for (int32_t bb = 0; bb < nbr; ++bb)
                if (bh[bb] == h) lev.push_back(bb);
            std::stable_sort(lev.begin(), lev.end(), [&](int32_t x, int32_t y) {
                return chain_len(x, true) > chain_len(y, true);
            });
            order.insert(order.end(), lev.begin(), lev.end());
            lvl.push_back((int32_t)order.size());
        }
        pos.assign(nbr, 0);
        for (int32_t k = 0; k < nbr; ++k) pos[order[k]] = k;
        // child entries (base compartments) in record order
        child0.assign(nbr, 0);
        {
            int32_t acc = 0;
            for (int32_t k = 0; k < nbr; ++k) {
                const int32_t bb = order[k];
                child0[k] = acc;
                for (int32_t r = 0; r < nchild(bb); ++r)
                    chl.push_back((uint16_t)tb0[tch[tch_off[bb] + r]]);
                acc += nchild(bb);
            }
        }
        for (int32_t k = 0; k < nbr; ++k) {
            const int32_t bb = order[k];
            Branch r{};
            r.b0 = (uint16_t)tb0[bb];
            r.b1 = (uint16_t)tb1[bb];
            r.child0 = (uint16_t)child0[k];
            r.nchild = (uint16_t)nchild(bb);
            r.par = (uint16_t)tpar[bb];
            for (int32_t c = 0; c < 2; ++c)
                r.cb[c] = c < nchild(bb) ? (uint16_t)tb0[tch[tch_off[bb] + c]] : 0;
            brs.push_back(r);
        }
        // branch ids in the compartment words: positions in record order
        for (int64_t c = d.comp0; c < (int64_t)topo.size(); ++c) {
            const uint32_t w = topo[c];
            const uint32_t bid = (w >> 16) & 0x7FFFu;
            if (bid != kNone) topo[c] = (w & ~(0x7FFFu << 16)) | ((uint32_t)pos[bid] << 16);
        }
        lvl.push_back(0);
        for (int h = 0; h < d.nfw; ++h) {
            lev.clear();
            for (int32_t bb = 0; bb < nbr; ++bb)
                if (bd[bb] == h) lev.push_back(bb);
            std::stable_sort(lev.begin(), lev.end(), [&](int32_t x, int32_t y) {
                return chain_len(x, false) > chain_len(y, false);
            });
            for (int32_t bb : lev)
                fws.push_back((uint16_t)pos[bb]);
            lvl.push_back((int32_t)(fws.size() - d.br0));
        }
        d.nch = (int32_t)chl.size() - d.ch0;
        d.it0 = 0;
        d.nrnd = 0;
        d.nrw = 0;
        d.nst = 0;
        if (s->solver == SIM_SOLVE_CONTRACT) {
            // round r of the pack: round r of each of its neurons, in pack
            // order, renumbered pack-locally; offsets follow the levels
            d.it0 = (int32_t)cit.size();
            int32_t maxr = 0;
            for (int32_t k = 0; k < pk[p].count; ++k)
                maxr = std::max(maxr, contraction_rounds(s, s->order[pk[p].first + k]));
            d.nrnd = maxr;
            lvl.push_back(0);
            for (int32_t r = 0; r < maxr; ++r) {
                for (int32_t k = 0; k < pk[p].count; ++k) {
                    const int32_t j = s->order[pk[p].first + k];
                    if (r >= contraction_rounds(s, j)) continue;
                    const int32_t *ro = s->croff.data() + s->croff0[j];
                    const uint32_t base = (uint32_t)member_base[k];
                    // pack-local, absent neighbours as the spare compartment
                    const uint32_t spare = (uint32_t)d.ncomp, m = spare + 1;
                    for (int32_t q = ro[r]; q < ro[r + 1]; ++q) {
                        const uint64_t it = s->citems[s->off[j] + q];
                        const uint32_t kk = base + (uint32_t)(it & 0x7FFFu);
                        const bool up = (it >> 15) & 1u;
                        const uint32_t n1 = (uint32_t)(it >> 16) & 0xFFFFu;
                        const uint32_t n2 = (uint32_t)(it >> 32) & 0xFFFFu;
                        const bool f1 = (it >> 49) & 1u, f2 = (it >> 50) & 1u;
                        const uint32_t i1 = n1 == kNoNb ? spare : base + n1;
                        const uint32_t i2 = n2 == kNoNb ? spare : base + n2;
                        // the coupling to n1 sits with the child of the pair
                        const uint32_t c1 = up ? kk : i1;
                        const uint32_t u1 = (n1 != kNoNb && f1) ? c1 : m + c1;
                        cit.push_back(make_citem(kk, i1, i2, u1, n2 != kNoNb && f2));
                    }
                }
                lvl.push_back((int32_t)(cit.size() - d.it0));
            }
            if ((int64_t)cit.size() - d.it0 != d.ncomp)
                throw fail(SIM_EINVAL, "internal: contraction schedule does not cover the pack");
            // the tail of rounds that one wavefront can take: every round
            // from nrw on has at most kWave items
            const int32_t *ro = lvl.data() + (lvl.size() - (size_t)maxr - 1);
            d.nrw = maxr;
            while (d.nrw > 0 && ro[d.nrw] - ro[d.nrw - 1] <= kWave) --d.nrw;
            if (cit.size() > (size_t)INT32_MAX) throw fail(SIM_ENOMEM, "contraction table too large");
        }
        d.tbytes = (int32_t)table_bytes(s, d.nbr, d.nch, d.nbw + d.nfw + 2, d.nsyn, d.ncomp, d.nrnd,
                                        0);
        // size class: 0 = fits the small LDS budget (many workgroups per CU),
        // 1 = needs a larger LDS allocation (its own concurrent launch), or
        // does not fit LDS at all (state in global scratch, same launch)
        const int64_t bytes = state_bytes(s, d.ncomp, d.nsyn, d.nneur);
        if (d.tbytes > s->max_lds) throw fail(SIM_EINVAL, "pack topology tables exceed LDS");
        int c = 0;
        while (c + 1 < ncls &&
               (d.tbytes + bytes > cls_budget[c] ||
                (v.res_cap && s->P.packing != SIM_PACK_PLAIN &&
                 d.ncomp > (int64_t)kResident *
                               std::min(v.threads << (c * v.cls_thr),
                                        s->tsize == 8 ? kMaxThreadsF64 : kMaxThreadsF32))))
            ++c;
        d.global_mem = d.tbytes + bytes <= cls_budget[c] ? 0 : 1;
        if (s->solver == SIM_SOLVE_CONTRACT && d.nrnd > 0) {
            // stage the single-wavefront tail of the schedule in LDS, as much
            // of it as the class budget leaves room for: those rounds are
            // short, so an item read from global memory would stall each one
            const int32_t *ro = lvl.data() + (lvl.size() - (size_t)d.nrnd - 1);
            const int64_t in_lds = d.global_mem ? 0 : bytes;
            auto tb_with = [&](int64_t nst) {
                return table_bytes(s, d.nbr, d.nch, d.nbw + d.nfw + 2, d.nsyn, d.ncomp, d.nrnd, nst);
            };
            int64_t nst = d.ncomp - ro[d.nrw];
            const int64_t room = (cls_budget[c] - in_lds - d.tbytes) / 8 + 2;
            nst = std::max<int64_t>(0, std::min(nst, room));
            while (nst > 0 && tb_with(nst) + in_lds > std::max<int64_t>(cls_budget[c], d.tbytes))
                --nst;
            d.nst = (int32_t)nst;
            d.tbytes = (int32_t)tb_with(nst);
            // the single-wavefront tail reads its items from LDS only: it
            // starts at the first round whose items are all staged; and its
            // lanes hold its round offsets, one per lane, so it spans at
            // most kWave - 1 rounds (a soma of high fan-out loses one child
            // per round and can need many more)
            while (d.nrw < d.nrnd && ro[d.nrw] < d.ncomp - d.nst) ++d.nrw;
            d.nrw = std::max(d.nrw, d.nrnd - (kWave - 1));
        }
        if (!d.global_mem) {
            lds_cls[c] = std::max(lds_cls[c], d.tbytes + bytes);
        } else {
            lds_cls[c] = std::max<int64_t>(lds_cls[c], d.tbytes);
            scratch = std::max(scratch, bytes);
        }
        pclass[p] = c;
        s->packs[p] = d;
    }
    ncomp0.push_back((int64_t)topo.size());
    s->scratch_bytes = scratch;

    for (int c = 0; c < kClasses; ++c) s->cls_comps[c] = 0;
    for (int p = 0; p < npk; ++p) s->cls_comps[pclass[p]] += s->packs[p].ncomp;

    // workgroup lists, one per size class
    s->wg_off.clear();
    s->wg_list.clear();
    int sched_mode = v.sched;
    if (s->P.packing == SIM_PACK_PLAIN) sched_mode = SIM_SCHED_DISPATCH;
    for (int c = 0; c < kClasses; ++c) {
        Launch &L = s->launch[c];
        L.lds = (size_t)std::max<int64_t>(lds_cls[c], 256);
        L.threads = std::min(v.threads << (c * v.cls_thr),
                             s->tsize == 8 ? kMaxThreadsF64 : kMaxThreadsF32);
        L.off0 = (int32_t)s->wg_off.size();
        L.list0 = (int32_t)s->wg_list.size();
        std::vector<int32_t> mine;  // in pack order (cost order for sorted packings)
        for (int p = 0; p < npk; ++p)
            if (pclass[p] == c) mine.push_back(p);
        const int np = (int)mine.size();
        // the resident-only kernel applies when every pack of the class keeps
        // its state in LDS and each thread's compartments fit its register
        // slots (FP32 gating, contraction solver)
        L.resident = np > 0 && s->tsize == 4 && s->solver == SIM_SOLVE_CONTRACT;
        for (int p : mine)
            if (s->packs[p].global_mem || s->packs[p].ncomp > kResident * L.threads)
                L.resident = false;
        if (np == 0) {
            L.n_wg = 0;
            s->wg_off.push_back(0);
            continue;
        }
        if (sched_mode == SIM_SCHED_DISPATCH || c > 0) {
            L.n_wg = np;
            for (int q = 0; q <= np; ++q) s->wg_off.push_back(q);
            for (int p : mine) s->wg_list.push_back(p);
        } else {
            // resident workgroups per CU from the LDS footprint and the threads
            const int by_lds = std::max(1, (int)(s->max_lds / std::max<size_t>(L.lds, 1)));
            const int by_thr = std::max(1, 2048 / v.threads);
            const int per_cu = std::max(1, std::min(by_lds, by_thr));
            L.n_wg = std::max(1, std::min(np, per_cu * s->n_cu));
            // LPT: packs by decreasing cost, each to the least loaded workgroup
            std::vector<int32_t> byc = mine;
            std::stable_sort(byc.begin(), byc.end(), [&](int32_t a, int32_t b) {
                return s->pack_cost[a] > s->pack_cost[b];
            });
            using QE = std::pair<double, int32_t>;
            std::priority_queue<QE, std::vector<QE>, std::greater<QE>> heap;
            for (int w = 0; w < L.n_wg; ++w) heap.push({0.0, w});
            std::vector<std::vector<int32_t>> lists(L.n_wg);
            for (int32_t p : byc) {
                QE top = heap.top();
                heap.pop();
                lists[top.second].push_back(p);
                heap.push({top.first + s->pack_cost[p], top.second});
            }
            int32_t acc = 0;
            s->wg_off.push_back(0);
            for (int w = 0; w < L.n_wg; ++w) {
                for (int32_t p : lists[w]) s->wg_list.push_back(p);
                acc += (int32_t)lists[w].size();
                s->wg_off.push_back(acc);
            }
        }
    }
    s->n_wg = 0;
    for (int c = 0; c < kClasses; ++c) s->n_wg += s->launch[c].n_wg;
    s->lds_bytes = s->launch[0].lds;
}

// Device copy of the layout build_layout left in s->hl, and the state arrays.
void upload_layout(sim_t *s) {
    sim_t::HostLayout &h = s->hl;
    const int32_t N = s->N;
    const int npk = (int)s->packs.size();
    s->d_packs.upload(s->packs);
    s->d_wg_off.upload(s->wg_off);
    s->d_wg_list.upload(s->wg_list);
    s->d_topo.upload(h.topo);
    s->d_cnb.upload(h.cnb);
    s->d_lparent.upload(h.lparent);
    s->d_len.upload(h.len);
    s->d_diam.upload(h.dia);
    s->d_ncomp0.upload(h.ncomp0);
    s->d_nid.upload(h.nid);
    s->d_ndet.upload(h.ndet);
    s->d_iext64.upload(h.iext64);
    s->d_spre.upload(h.spre);
    s->d_sdelay.upload(h.sdel);
    s->d_w64.upload(h.w64);
    s->d_scomp.upload(h.scomp);
    s->d_sseg.upload(h.sseg);
    s->d_br.upload(h.brs);
    s->d_fw.upload(h.fws);
    s->d_cit.upload(h.cit);
    s->d_chl.upload(h.chl);
    s->d_lvl.upload(h.lvl);
    const int64_t C = s->C, S = s->S;
    s->d_V.alloc(C);
    s->d_cdt.alloc(C);
    s->d_e.alloc(C);
    s->d_gm.alloc(C * s->tsize);
    s->d_gh.alloc(C * s->tsize);
    s->d_gn.alloc(C * s->tsize);
    s->d_af.alloc(C * s->tsize);
    s->d_sg.alloc(S * s->tsize);
    s->d_sw.alloc(S * s->tsize);
    s->d_niext.alloc((int64_t)N * s->tsize);
    s->d_q.alloc(1);
    s->d_scratch.alloc(256);
    s->d_ptime.alloc(npk);
    HIPCHK(hipMemset(s->d_ptime.p, 0, sizeof(uint64_t) * npk));
    s->hl = sim_t::HostLayout{};  // the device holds it now
}

void init_state(sim_t *s) {
    SetupArgs a{};
    a.n_neurons = s->N;
    a.ncomp0 = s->d_ncomp0.p;
    a.lparent = s->d_lparent.p;
    a.length = s->d_len.p;
    a.diam = s->d_diam.p;
    a.cm = s->CH.cm_uF_cm2;
    a.ra = s->CH.ra_ohm_cm;
    a.dt = s->P.dt_ms;
    a.theta = s->P.theta;
    a.v_init = s->P.v_init_mV;
    a.cdt = s->d_cdt.p;
    a.e = s->d_e.p;
    a.V = s->d_V.p;
    a.af = s->d_af.p;
    a.gm = s->d_gm.p;
    a.gh = s->d_gh.p;
    a.gn = s->d_gn.p;
    a.q_out = s->d_q.p;
    a.tau = s->P.tau_syn_ms;
    HIPCHK(launch_setup(a, s->precision == SIM_FP64 ? 0 : 1, s->stream));
    const int pr = s->precision == SIM_FP64 ? 0 : 1;
    HIPCHK(launch_decay_weights_convert(s->d_w64.p, s->d_sw.p, s->S, pr, s->stream));
    HIPCHK(launch_decay_weights_convert(s->d_iext64.p, s->d_niext.p, s->N, pr, s->stream));
    if (s->S) HIPCHK(hipMemsetAsync(s->d_sg.p, 0, s->S * s->tsize, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    HIPCHK(hipMemcpy(&s->q, s->d_q.p, sizeof(double), hipMemcpyDeviceToHost));
    s->step = 0;
    if (s->d_ring.p && s->d_ring.n) HIPCHK(launch_fill_u64(s->d_ring.p, s->d_ring.n, 0, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->spikes.clear();
    s->drain[0].pending = s->drain[1].pending = false;
    s->drain_slot = 0;
}

void destroy_graphs(sim_t *s) {
    if (s->exec1) (void)hipGraphExecDestroy(s->exec1);
    if (s->execK) (void)hipGraphExecDestroy(s->execK);
    if (s->graph1) (void)hipGraphDestroy(s->graph1);
    if (s->graphK) (void)hipGraphDestroy(s->graphK);
    s->exec1 = s->execK = nullptr;
    s->graph1 = s->graphK = nullptr;
}

EpochArgs make_args(sim_t *s) {
    EpochArgs a{};
    a.packs = s->d_packs.p;
    a.wg_off = s->d_wg_off.p;
    a.wg_list = s->d_wg_list.p;
    a.V = s->d_V.p;
    a.gm = s->d_gm.p;
    a.gh = s->d_gh.p;
    a.gn = s->d_gn.p;
    a.topo = s->d_topo.p;
    a.cnb = s->d_cnb.p;
    a.cdt = s->d_cdt.p;
    a.e = s->d_e.p;
    a.af = s->d_af.p;
    a.sg = s->d_sg.p;
    a.sw = s->d_sw.p;
    a.spre = s->d_spre.p;
    a.sdelay = s->d_sdelay.p;
    a.scomp = s->d_scomp.p;
    a.sseg = s->d_sseg.p;
    a.nid = s->d_nid.p;
    a.ndet = s->d_ndet.p;
    a.niext = s->d_niext.p;
    a.br = s->d_br.p;
    a.fw = s->d_fw.p;
    a.chl = s->d_chl.p;
    a.lvl = s->d_lvl.p;
    a.cit = s->d_cit.p;
    a.ring = s->d_ring.p;
    a.ring_rows = s->ring_rows;
    a.n_neurons = s->N;
    a.E = s->E;
    a.scratch = s->scratch_override ? s->scratch_override : s->d_scratch.p;
    a.scratch_stride = 0;
    a.omt = 1.0 - s->P.theta;
    a.ginv = -1.0 / s->P.theta;
    a.v_thresh = s->P.v_thresh_mV;
    a.gnabar = s->CH.gnabar;
    a.gkbar = s->CH.gkbar;
    a.gl = s->CH.gl;
    a.ena = s->CH.ena;
    a.ek = s->CH.ek;
    a.el = s->CH.el;
    a.g_pas = s->CH.g_pas;
    a.e_pas = s->CH.e_pas;
    a.e_syn = s->P.e_syn_mV;
    a.dt = s->P.dt_ms;
    a.q = s->q;
    {
        const double dc[11] = {a.gnabar, a.gkbar, a.gl,    a.ena, a.ek, a.el,
                               a.g_pas,  a.e_pas, a.e_syn, a.dt,  a.q};
        for (int k = 0; k < 11; ++k) a.fch[k] = (float)dc[k];
    }
    a.pack_time = s->P.record_timings ? s->d_ptime.p : nullptr;
    return a;
}

}  // namespace

namespace {

// Global packs need disjoint scratch slices even when one workgroup runs
// several of them in sequence: the slice is chosen per pack from its ordinal.
// The offsets are folded into the pack table's `global_mem` field (1 + slice
// index in units of the largest global pack).
void assign_scratch(sim_t *s) {
    int64_t maxb = 0;
    int32_t count = 0;
    for (auto &d : s->packs)
        if (d.global_mem) {
            maxb = std::max(maxb, state_bytes(s, d.ncomp, d.nsyn, d.nneur));
            d.global_mem = 1 + count++;
        }
    s->scratch_total = maxb * count;
    if (count) {
        s->d_scratch.alloc(maxb * count);
        s->scratch_bytes = maxb;
        HIPCHK(hipMemcpy(s->d_packs.p, s->packs.data(), sizeof(PackDesc) * s->packs.size(),
                         hipMemcpyHostToDevice));
    }
}

// Two events of the pool for one timed span of `epochs` epochs (created on
// first use).
std::pair<hipEvent_t, hipEvent_t> kt_pair(sim_t *s, int epochs) {
    while ((int)s->kt_pool.size() < s->kt_used + 2) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        s->kt_pool.push_back(e);
    }
    s->kt_ep.resize(s->kt_pool.size() / 2);
    s->kt_ep[s->kt_used / 2] = epochs;
    s->kt_used += 2;
    return {s->kt_pool[s->kt_used - 2], s->kt_pool[s->kt_used - 1]};
}

// Re-arm the device launch timers and clear their totals (stream idle).
void ktimer_reset(sim_t *s) {
    std::vector<uint64_t> init(8 * kClasses, 0);
    for (int c = 0; c < kClasses; ++c) init[8 * c] = ~0ull;
    HIPCHK(hipMemcpy(s->d_ktimer.p, init.data(), sizeof(uint64_t) * init.size(),
                     hipMemcpyHostToDevice));
}

// Read back the epoch spans recorded since the last call (stream idle), and
// the device timers' totals per size class.
void kt_collect(sim_t *s) {
    for (int u = 0; u + 1 < s->kt_used; u += 2) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, s->kt_pool[u], s->kt_pool[u + 1]));
        s->kt_ms += ms;
        s->kt_launches += s->kt_ep[u / 2];
    }
    s->kt_used = 0;
    uint64_t t[8 * kClasses];
    HIPCHK(hipMemcpy(t, s->d_ktimer.p, sizeof t, hipMemcpyDeviceToHost));
    for (int c = 0; c < kClasses; ++c) {
        s->kt_cls_ms[c] = (double)t[8 * c + 4] * s->tick_ns * 1e-6;
        s->kt_cls_n[c] = (int64_t)t[8 * c + 5];
    }
}

// One epoch (or part of one): the large-pack class on the second stream and
// the small-pack class on the main stream run concurrently, forked from and
// joined back into the main stream (also inside a captured graph).
void launch_range(sim_t *s, int64_t epoch, int t0, int t1, bool use_ptr) {
    const int pr = s->precision == SIM_FP64 ? 0 : 1;
    auto args = [&](const Launch &L, int c) {
        EpochArgs a = make_args(s);
        a.ktimer = s->d_ktimer.p + 8 * c;
        a.wg_off = s->d_wg_off.p + L.off0;
        a.wg_list = s->d_wg_list.p + L.list0;
        a.epoch = epoch;
        a.epoch_ptr = use_ptr ? s->d_epoch.p : nullptr;
        a.t0 = t0;
        a.t1 = t1;
        a.scratch_stride = s->scratch_bytes;
        return a;
    };
    bool forked = false;
    for (int c = kClasses - 1; c >= 1; --c) {  // largest packs first
        const Launch &L = s->launch[c];
        if (L.n_wg == 0) continue;
        if (!forked) {
            HIPCHK(hipEventRecord(s->ev_fork, s->stream));
            forked = true;
        }
        HIPCHK(hipStreamWaitEvent(s->side[c], s->ev_fork, 0));
        EpochArgs ac = args(L, c);
        HIPCHK(launch_stamp(ac.ktimer, s->side[c]));
        HIPCHK(launch_epoch(ac, pr, s->solver, L.n_wg, L.threads, L.lds, L.resident, s->side[c]));
        HIPCHK(hipEventRecord(s->ev_join[c], s->side[c]));
    }
    const Launch &S0 = s->launch[0];
    if (S0.n_wg > 0) {
        const EpochArgs a0 = args(S0, 0);
        HIPCHK(launch_stamp(a0.ktimer, s->stream));
        HIPCHK(launch_epoch(a0, pr, s->solver, S0.n_wg, S0.threads, S0.lds, S0.resident,
                                 s->stream));
    }
    for (int c = 1; c < kClasses; ++c)
        if (s->launch[c].n_wg > 0) HIPCHK(hipStreamWaitEvent(s->stream, s->ev_join[c], 0));
}

void capture(sim_t *s, int epochs, hipGraph_t &g, hipGraphExec_t &ex) {
    HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < epochs; ++k) {
        launch_range(s, 0, 0, s->E, true);
        hipError_t e = launch_advance(s->d_epoch.p, s->stream);
        if (e != hipSuccess) {
            hipGraph_t dummy;
            (void)hipStreamEndCapture(s->stream, &dummy);
            throw fail(SIM_EDEVICE, "capture failed: %s", hipGetErrorString(e));
        }
    }
    HIPCHK(hipStreamEndCapture(s->stream, &g));
    HIPCHK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
}

// Spikes of the steps (lo, hi] staged in `slot`, appended to the host list in
// (step, neuron) order once the copy has landed.
void scan_stage(sim_t *s, int slot) {
    sim_t::Drain &d = s->drain[slot];
    if (!d.pending) return;
    HIPCHK(hipEventSynchronize(s->ev_stage[slot]));
    const int E = s->E;
    if (s->sink) {
        // allocation-free form for sim_step_noalloc: step by step over the
        // staged words, into the caller's buffer (counting past its end)
        for (int32_t r = 0; r < d.rows; ++r) {
            const int64_t e = d.first_epoch + r;
            const uint64_t *w = s->h_stage[slot] + (size_t)r * s->N;
            for (int t = 0; t < E; ++t) {
                const int64_t step = e * E + t + 1;
                if (step <= d.lo || step > d.hi) continue;
                for (int32_t j = 0; j < s->N; ++j)
                    if ((w[j] >> t) & 1ull) {
                        if (s->sink_n < s->sink_cap)
                            s->sink[s->sink_n] = sim_spike_t{j, (int32_t)step};
                        s->sink_n++;
                    }
            }
        }
        d.pending = false;
        return;
    }
    s->by_t.resize(E);
    for (int32_t r = 0; r < d.rows; ++r) {
        const int64_t e = d.first_epoch + r;
        for (auto &v : s->by_t) v.clear();
        const uint64_t *w = s->h_stage[slot] + (size_t)r * s->N;
        for (int32_t j = 0; j < s->N; ++j)
            for (uint64_t m = w[j]; m; m &= m - 1) s->by_t[__builtin_ctzll(m)].push_back(j);
        for (int t = 0; t < E; ++t) {
            const int64_t step = e * E + t + 1;
            if (step <= d.lo || step > d.hi) continue;
            for (int32_t j : s->by_t[t]) s->spikes.push_back(sim_spike_t{j, (int32_t)step});
        }
    }
    d.pending = false;
}

// After the steps (lo, hi] are enqueued: copy their ring rows to the next
// staging slot behind them on the stream (the slot's previous contents are
// read first).
void enqueue_drain(sim_t *s, int64_t lo, int64_t hi) {
    if (hi <= lo) return;
    const int E = s->E, R = s->ring_rows;
    const int64_t e0 = lo / E, e1 = (hi - 1) / E;
    const int slot = s->drain_slot;
    scan_stage(s, slot);
    const int32_t rows = (int32_t)(e1 - e0 + 1);
    if (rows > R) throw fail(SIM_ESTATE, "drain of %d epochs exceeds the ring", rows);
    for (int32_t r = 0; r < rows;) {
        const int64_t row = (e0 + r) % R;
        const int32_t n = (int32_t)std::min<int64_t>(rows - r, R - row);
        HIPCHK(hipMemcpyAsync(s->h_stage[slot] + (size_t)r * s->N, s->d_ring.p + row * s->N,
                              sizeof(uint64_t) * (size_t)n * s->N, hipMemcpyDeviceToHost,
                              s->stream));
        r += n;
    }
    HIPCHK(hipEventRecord(s->ev_stage[slot], s->stream));
    s->drain[slot] = sim_t::Drain{e0, rows, lo, hi, true};
    s->drain_slot = slot ^ 1;
}

void advance(sim_t *s, int64_t n, bool graphs);

// Steps in stretches that never overwrite a ring row before it is staged: a
// stretch ends before the epoch ring_rows after its first one begins.
// graphs = false launches every epoch directly (no capture, no replay).
void run_steps(sim_t *s, int64_t n, bool graphs = true) {
    if (n <= 0) return;
    const int E = s->E;
    while (n > 0) {
        const int64_t lo = s->step;
        const int64_t room = (lo / E + s->ring_rows) * E - lo;
        const int64_t m = std::min(n, room);
        advance(s, m, graphs);
        enqueue_drain(s, lo, s->step);
        n -= m;
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    scan_stage(s, s->drain_slot);  // older first
    scan_stage(s, s->drain_slot ^ 1);
    if (s->kt_on) kt_collect(s);
}

void advance(sim_t *s, int64_t n, bool graphs) {
    const int E = s->E;
    while (n > 0) {
        const int64_t ep = s->step / E;
        const int t0 = (int)(s->step % E);
        const int64_t full = (t0 == 0) ? n / E : 0;
        if (full > 0 && s->P.use_graph && graphs) {
            if (!s->exec1) capture(s, 1, s->graph1, s->exec1);
            if (!s->execK) capture(s, s->graphK_epochs, s->graphK, s->execK);
            // stream-ordered: the replays of an earlier stretch may still be
            // running on this stream and advancing the counter
            HIPCHK(launch_fill_u64((uint64_t *)s->d_epoch.p, 1, (uint64_t)ep, s->stream));
            auto replay = [&](hipGraphExec_t ex, int epochs) {
                std::pair<hipEvent_t, hipEvent_t> ev{};
                if (s->kt_on) {
                    ev = kt_pair(s, epochs);
                    HIPCHK(hipEventRecord(ev.first, s->stream));
                }
                HIPCHK(hipGraphLaunch(ex, s->stream));
                if (s->kt_on) HIPCHK(hipEventRecord(ev.second, s->stream));
            };
            int64_t left = full;
            while (left >= s->graphK_epochs) {
                replay(s->execK, s->graphK_epochs);
                left -= s->graphK_epochs;
            }
            while (left > 0) {
                replay(s->exec1, 1);
                left -= 1;
            }
            if (s->kt_on)
                for (int c = 0; c < kClasses; ++c)
                    if (s->launch[c].n_wg > 0) s->kt_cls_upd[c] += s->cls_comps[c] * full * E;
            s->step += full * E;
            n -= full * E;
            continue;
        }
        const int t1 = (int)std::min<int64_t>(E, t0 + n);
        std::pair<hipEvent_t, hipEvent_t> ev{};
        if (s->kt_on) {
            ev = kt_pair(s, 1);
            HIPCHK(hipEventRecord(ev.first, s->stream));
        }
        launch_range(s, ep, t0, t1, false);
        if (s->kt_on) {
            HIPCHK(hipEventRecord(ev.second, s->stream));
            for (int c = 0; c < kClasses; ++c)
                if (s->launch[c].n_wg > 0) s->kt_cls_upd[c] += s->cls_comps[c] * (t1 - t0);
        }
        s->step += t1 - t0;
        n -= t1 - t0;
    }
}

std::string describe(const sim_t *s) {
    char buf[640];
    int nglob = 0;
    for (auto &d : s->packs) nglob += d.global_mem ? 1 : 0;
    snprintf(buf, sizeof buf,
             "threads=%d pack_comps=%d lds_limit=%d classes=%d sched=%s packs=%zu global_packs=%d "
             "wg=%d+%d+%d wg_threads=%d+%d+%d lds_bytes=%zu+%zu+%zu E=%d precision=%s solver=%s "
             "packing=%s",
             s->var.threads, s->var.pack_comps, s->var.lds_limit, s->var.nclass,
             (s->P.packing == SIM_PACK_PLAIN || s->var.sched == SIM_SCHED_DISPATCH) ? "dispatch"
                                                                                    : "persistent",
             s->packs.size(), nglob, s->launch[0].n_wg, s->launch[1].n_wg, s->launch[2].n_wg,
             s->launch[0].threads, s->launch[1].threads, s->launch[2].threads,
             s->launch[0].lds, s->launch[1].lds, s->launch[2].lds, s->E,
             s->precision == SIM_FP64 ? "fp64" : "fp32-gating",
             s->solver == SIM_SOLVE_FAST ? "fast"
             : s->solver == SIM_SOLVE_CONTRACT ? "contract" : "exact",
             s->P.packing == SIM_PACK_PLAIN ? "plain"
             : s->P.packing == SIM_PACK_COUNT ? "count"
             : !s->ncost.empty() ? "learned(given costs)"
             : s->cost_model.empty() ? "learned(fallback count)" : "learned");
    return buf;
}

void apply_variant(sim_t *s, const Variant &v) {
    destroy_graphs(s);
    build_layout(s, v);
    upload_layout(s);
    assign_scratch(s);
    init_state(s);
    s->config = describe(s);
}

// LDS budget of a pack class: the bytes of a pack of `comps` compartments
// with a typical synapse count.
int lds_for(const sim_t *s, int comps) {
    return (int)std::min<int64_t>(s->max_lds, state_bytes(s, comps, comps / 4 + 16, 64));
}

// Autotuning: time epochs of each candidate from the initial state, keep
// the fastest, then re-initialise. Candidates never change results: they only
// move neurons between workgroups or memory spaces.

constexpr int64_t kAutotuneShapesMaxComps = 50000000;

void autotune(sim_t *s, Variant base) {
    // (pack_comps, LDS budget in compartments): small packs keep more
    // workgroups resident per CU, which hides the latency of the sweeps
    static const int kShapes[][2] = {{300, 420},  {400, 550},   {500, 680},  {600, 800},
                                     {800, 1100}, {1000, 1300}, {1400, 1800}};
    // Every trial lays the network out again on the host, which takes seconds
    // at 1e8 compartments: there the pack-shape sweep (whose winner has been
    // the default shape on every multi-morphology workload measured) is left
    // out and only the class structure is tried.
    const bool large = s->C > kAutotuneShapesMaxComps;
    std::vector<Variant> cand;
    for (int thr : {128, 256, 320})
        for (const auto &sh : kShapes) {
            if (large) break;
            Variant v = base;
            v.threads = thr;
            v.pack_comps = sh[0];
            v.lds_limit = lds_for(s, sh[1]);
            v.sched = SIM_SCHED_DISPATCH;
            cand.push_back(v);
        }
    for (int nc : {1, 3}) {  // the largest packs in fewer or more launches
        Variant v = base;
        v.sched = SIM_SCHED_DISPATCH;
        v.nclass = nc;
        cand.push_back(v);
    }
    // the balance between the concurrent size classes: larger budgets for
    // the small-pack class, and more threads for the larger-pack classes
    for (int comps : {1500, 2000})
        for (int nc : {2, 3}) {
            Variant v = base;
            v.sched = SIM_SCHED_DISPATCH;
            v.lds_limit = lds_for(s, comps);
            v.nclass = nc;
            cand.push_back(v);
        }
    for (int nc : {2, 3}) {
        Variant v = base;
        v.sched = SIM_SCHED_DISPATCH;
        v.nclass = nc;
        v.cls_thr = 2;
        cand.push_back(v);
    }
    {
        Variant v = base;
        v.sched = SIM_SCHED_PERSISTENT;
        cand.push_back(v);
    }
    if (s->tsize == 4 && s->solver == SIM_SOLVE_CONTRACT) {
        // packs capped at the register slots of their class's threads, so
        // that every launch keeps all gates and constants in registers (on
        // the multi-morphology workloads the fuller uncapped packs have won)
        for (int thr : {192, 256})
            for (int nc2 : {2, 3}) {
                Variant v = base;
                v.sched = SIM_SCHED_DISPATCH;
                v.threads = thr;
                v.lds_limit = lds_for(s, kResident * thr);
                v.nclass = nc2;
                v.res_cap = true;
                cand.push_back(v);
            }
        Variant v = base;
        v.sched = SIM_SCHED_DISPATCH;
        v.res_cap = true;
        cand.push_back(v);
    }
    // each candidate: a warm-up epoch, then the fastest of `reps` timed
    // epochs; the three fastest candidates are then timed again and the
    // fastest of those is kept (one epoch of one layout varies by a few
    // percent from run to run, about as much as the layouts differ)
    auto time_variant = [&](const Variant &v, int reps) {
        apply_variant(s, v);
        launch_range(s, 0, 0, s->E, false);  // warm-up
        HIPCHK(hipStreamSynchronize(s->stream));
        double best_ms = 1e30;
        for (int r = 0; r < reps; ++r) {
            HIPCHK(hipEventRecord(s->ev0, s->stream));
            launch_range(s, 0, 0, s->E, false);
            HIPCHK(hipEventRecord(s->ev1, s->stream));
            HIPCHK(hipEventSynchronize(s->ev1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, s->ev0, s->ev1));
            best_ms = std::min(best_ms, (double)ms);
        }
        return best_ms;
    };
    // The requested layout is kept unless another is faster by more than
    // kKeep: epochs timed from the initial state rank layouts within a
    // percent or two of each other less reliably than that.
    constexpr double kKeep = 0.015;
    std::vector<std::pair<double, size_t>> t;
    for (size_t k = 0; k < cand.size(); ++k) t.emplace_back(time_variant(cand[k], 2), k);
    std::sort(t.begin(), t.end());
    double best = 1e30;
    Variant bestv = base;
    for (size_t r = 0; r < std::min<size_t>(3, t.size()); ++r) {
        const Variant &v = cand[t[r].second];
        const double ms = std::min(t[r].first, time_variant(v, 4));
        if (ms < best) {
            best = ms;
            bestv = v;
        }
    }
    if (time_variant(base, 4) <= best * (1.0 + kKeep)) bestv = base;
    apply_variant(s, bestv);
}

// The launch variant the parameters ask for (before autotuning).
Variant variant_from(const sim_t *s, const sim_params_t *params) {
    Variant v;
    v.threads = params->threads ? params->threads : 256;
    v.pack_comps = params->pack_comps ? params->pack_comps : 800;
    v.comp_cap = params->pack_comps;
    v.lds_limit = lds_for(s, params->lds_comps ? params->lds_comps : 1100);
    if (params->lds_classes) v.nclass = params->lds_classes;
    v.sched = params->sched == SIM_SCHED_PERSISTENT ? SIM_SCHED_PERSISTENT : SIM_SCHED_DISPATCH;
    return v;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void sim_default_params(sim_params_t *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->dt_ms = 0.025;
    p->theta = 0.5;
    p->tau_syn_ms = 2.0;
    p->e_syn_mV = 0.0;
    p->v_thresh_mV = 0.0;
    p->v_init_mV = -65.0;
    p->precision = SIM_FP32_GATING;
    p->solver = SIM_SOLVE_EXACT;
    p->packing = SIM_PACK_COUNT;
    p->sched = SIM_SCHED_AUTO;
    p->use_graph = 1;
}

int sim_create(const sim_params_t *params, const sim_morphology_t *morph,
               const sim_channels_t *channels, const sim_synapses_t *syn, sim_t **out) {
    if (!out) {
        g_create_error = "null output pointer";
        return SIM_EINVAL;
    }
    *out = nullptr;
    sim_t *s = nullptr;
    try {
        validate(params, morph, channels, syn);
        s = new sim_t();
        copy_inputs(s, params, morph, channels, syn);
        analyse_all(s);
        // device
        int dev = 0;
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
            throw fail(SIM_EDEVICE, "no HIP device available");
        HIPCHK(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, dev));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            throw fail(SIM_EDEVICE, "device %s is not gfx950", prop.gcnArchName);
        s->n_cu = prop.multiProcessorCount;
        s->max_lds = (int)std::min<size_t>(prop.maxSharedMemoryPerMultiProcessor, 160 * 1024);
        if (s->max_lds < (int)prop.sharedMemPerBlock) s->max_lds = (int)prop.sharedMemPerBlock;
        if (set_epoch_lds_limit(s->max_lds) != hipSuccess) {
            (void)hipGetLastError();
            s->max_lds = (int)prop.sharedMemPerBlock;
        }
        HIPCHK(noalloc_scratch(&s->na_scratch));
        int clk_khz = 0;
        if (hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess &&
            clk_khz > 0)
            s->tick_ns = 1e6 / (double)clk_khz;
        if (params->hip_stream) {
            s->stream = (hipStream_t)params->hip_stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
            s->own_stream = true;
        }
        HIPCHK(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
        for (int c = 1; c < kClasses; ++c) {
            HIPCHK(hipStreamCreateWithFlags(&s->side[c], hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&s->ev_join[c], hipEventDisableTiming));
        }
        HIPCHK(hipEventCreate(&s->ev0));
        HIPCHK(hipEventCreate(&s->ev1));
        s->d_epoch.alloc(1);
        s->d_ktimer.alloc(8 * kClasses);
        ktimer_reset(s);
        s->d_ring.alloc((int64_t)s->ring_rows * s->N);
        for (int k = 0; k < 2; ++k) {
            HIPCHK(hipHostMalloc((void **)&s->h_stage[k],
                                 sizeof(uint64_t) * (size_t)s->ring_rows * s->N, hipHostMallocDefault));
            HIPCHK(hipEventCreateWithFlags(&s->ev_stage[k], hipEventDisableTiming));
        }
        compute_cost(s);
        const Variant v = variant_from(s, params);
        if (params->autotune)
            autotune(s, v);
        else
            apply_variant(s, v);
        *out = s;
        return SIM_OK;
    } catch (const Error &e) {
        g_create_error = e.msg;
        if (s) sim_destroy(s);
        return e.code;
    } catch (const std::bad_alloc &) {
        g_create_error = "host allocation failed";
        if (s) sim_destroy(s);
        return SIM_ENOMEM;
    }
}

int sim_plan_create(const sim_params_t *params, const sim_morphology_t *morph,
                    const sim_channels_t *channels, const sim_synapses_t *syn,
                    int32_t lds_bytes_per_cu, int32_t n_cu, sim_t **out) {
    if (!out) {
        g_create_error = "null output pointer";
        return SIM_EINVAL;
    }
    *out = nullptr;
    sim_t *s = nullptr;
    try {
        validate(params, morph, channels, syn);
        if (lds_bytes_per_cu < 4096 || lds_bytes_per_cu > (1 << 20) || n_cu < 1)
            throw fail(SIM_EINVAL, "plan needs 4096 <= lds_bytes_per_cu <= 1 MiB and n_cu >= 1");
        if (params->packing == SIM_PACK_LEARNED && params->cost_model)
            throw fail(SIM_EINVAL, "a learned cost model needs the device (sim_create)");
        if (params->autotune) throw fail(SIM_EINVAL, "autotuning needs the device (sim_create)");
        s = new sim_t();
        s->planned_only = true;
        copy_inputs(s, params, morph, channels, syn);
        analyse_all(s);
        s->max_lds = lds_bytes_per_cu;
        s->n_cu = n_cu;
        compute_cost(s);
        build_layout(s, variant_from(s, params));
        {
            // a planned layout keeps its contraction items for introspection
            std::vector<uint64_t> cit = std::move(s->hl.cit);
            s->hl = sim_t::HostLayout{};
            s->hl.cit = std::move(cit);
        }
        s->config = describe(s);
        *out = s;
        return SIM_OK;
    } catch (const Error &e) {
        g_create_error = e.msg;
        if (s) sim_destroy(s);
        return e.code;
    } catch (const std::bad_alloc &) {
        g_create_error = "host allocation failed";
        if (s) sim_destroy(s);
        return SIM_ENOMEM;
    }
}

int32_t sim_pack_count(const sim_t *s) { return s ? (int32_t)s->packs.size() : -1; }

int sim_pack_info(const sim_t *s, int32_t pack, sim_pack_info_t *out) {
    if (!s || !out || pack < 0 || pack >= (int32_t)s->packs.size()) return SIM_EINVAL;
    const PackDesc &d = s->packs[pack];
    int cls = -1;
    for (int c = 0; c < kClasses && cls < 0; ++c) {
        const Launch &L = s->launch[c];
        for (int32_t w = 0; w < L.n_wg && cls < 0; ++w)
            for (int32_t q = s->wg_off[L.off0 + w]; q < s->wg_off[L.off0 + w + 1]; ++q)
                if (s->wg_list[L.list0 + q] == pack) {
                    cls = c;
                    break;
                }
    }
    out->first_position = d.neur0;
    out->n_neurons = d.nneur;
    out->n_comp = d.ncomp;
    out->n_syn = d.nsyn;
    out->n_branches = d.nbr;
    out->size_class = cls;
    out->in_global = d.global_mem ? 1 : 0;
    out->n_rounds = d.nrnd;
    out->n_levels = d.nbw + d.nfw + 2;
    out->n_child_entries = d.nch;
    out->table_bytes = d.tbytes;
    out->state_bytes = state_bytes(s, d.ncomp, d.nsyn, d.nneur);
    out->cost = s->pack_cost[pack];
    out->n_wide_rounds = d.nrw;
    out->n_staged_items = d.nst;
    return SIM_OK;
}

int sim_pack_neurons(const sim_t *s, int32_t pack, int32_t *ids, int64_t cap) {
    if (!s || !ids || pack < 0 || pack >= (int32_t)s->packs.size()) return SIM_EINVAL;
    const PackDesc &d = s->packs[pack];
    if (cap < d.nneur) return SIM_EINVAL;
    for (int32_t k = 0; k < d.nneur; ++k) ids[k] = s->order[d.neur0 + k];
    return SIM_OK;
}

int sim_class_launch(const sim_t *s, int32_t cls, int32_t *n_wg, int32_t *threads,
                     int64_t *lds_bytes) {
    if (!s || cls < 0 || cls >= kClasses) return SIM_EINVAL;
    if (n_wg) *n_wg = s->launch[cls].n_wg;
    if (threads) *threads = s->launch[cls].threads;
    if (lds_bytes) *lds_bytes = (int64_t)s->launch[cls].lds;
    return SIM_OK;
}

int sim_workgroup_packs(const sim_t *s, int32_t cls, int32_t wg, int32_t *packs, int64_t cap,
                        int32_t *n) {
    if (!s || cls < 0 || cls >= kClasses) return SIM_EINVAL;
    const Launch &L = s->launch[cls];
    if (wg < 0 || wg >= L.n_wg) return SIM_EINVAL;
    const int32_t q0 = s->wg_off[L.off0 + wg], q1 = s->wg_off[L.off0 + wg + 1];
    if (n) *n = q1 - q0;
    if (!packs) return SIM_OK;
    if (cap < q1 - q0) return SIM_EINVAL;
    for (int32_t q = q0; q < q1; ++q) packs[q - q0] = s->wg_list[L.list0 + q];
    return SIM_OK;
}

int sim_contraction_schedule(const sim_t *s, int32_t neuron, int32_t *items, int64_t cap,
                             int32_t *round_off, int64_t cap_rounds, int32_t *n_rounds) {
    if (!s || neuron < 0 || neuron >= s->N) return SIM_EINVAL;
    if (s->solver != SIM_SOLVE_CONTRACT) return SIM_ESTATE;
    const int32_t nr = contraction_rounds(s, neuron);
    const int64_t n = s->off[neuron + 1] - s->off[neuron];
    if (n_rounds) *n_rounds = nr;
    if (!items) return SIM_OK;
    if (cap < 4 * n || !round_off || cap_rounds < nr + 1) return SIM_EINVAL;
    for (int64_t q = 0; q < n; ++q) {
        const uint64_t it = s->citems[s->off[neuron] + q];
        const uint32_t n1 = (uint32_t)(it >> 16) & 0xFFFFu, n2 = (uint32_t)(it >> 32) & 0xFFFFu;
        items[4 * q + 0] = (int32_t)(it & 0x7FFFu);
        items[4 * q + 1] = n1 == kNoNb ? -1 : (int32_t)n1;
        items[4 * q + 2] = n2 == kNoNb ? -1 : (int32_t)n2;
        items[4 * q + 3] = (int32_t)((it >> 15) & 1u) | (int32_t)(((it >> 49) & 1u) << 1) |
                           (int32_t)(((it >> 50) & 1u) << 2);
    }
    const int32_t *ro = s->croff.data() + s->croff0[neuron];
    for (int32_t r = 0; r <= nr; ++r) round_off[r] = ro[r];
    return SIM_OK;
}

int sim_pack_contraction_items(const sim_t *s, int32_t pack, uint64_t *items, int64_t cap,
                               int64_t *n) {
    if (!s || pack < 0 || pack >= (int32_t)s->packs.size() || !n) return SIM_EINVAL;
    if (s->solver != SIM_SOLVE_CONTRACT || !s->planned_only) return SIM_ESTATE;
    const PackDesc &d = s->packs[pack];
    *n = d.ncomp;
    if (!items) return SIM_OK;
    if (cap < d.ncomp) return SIM_EINVAL;
    if ((int64_t)d.it0 + d.ncomp > (int64_t)s->hl.cit.size()) return SIM_ESTATE;
    std::copy(s->hl.cit.begin() + d.it0, s->hl.cit.begin() + d.it0 + d.ncomp, items);
    return SIM_OK;
}

int sim_step(sim_t *s, int64_t n_steps) {
    if (!s) return SIM_EINVAL;
    if (s->planned_only) {
        s->err = "a planned simulation has no device state";
        return SIM_ESTATE;
    }
    if (n_steps < 0) {
        s->err = "n_steps must be >= 0";
        return SIM_EINVAL;
    }
    try {
        run_steps(s, n_steps);
        return SIM_OK;
    } catch (const Error &e) {
        s->err = e.msg;
        return e.code;
    }
}

int sim_step_noalloc(sim_t *s, int64_t n_steps, sim_spike_t *out, int64_t cap,
                     int64_t *n_out) {
    if (!s) return SIM_EINVAL;
    if (s->planned_only) {
        s->err = "a planned simulation has no device state";
        return SIM_ESTATE;
    }
    if (n_steps < 0 || cap < 0 || (cap > 0 && !out)) {
        s->err = "n_steps and cap must be >= 0, out non-null when cap > 0";
        return SIM_EINVAL;
    }
    if (s->scratch_total > kNoAllocScratchBytes) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "packs kept in global memory need %lld bytes of scratch, more than the "
                 "%lld of the fixed array",
                 (long long)s->scratch_total, (long long)kNoAllocScratchBytes);
        s->err = buf;
        return SIM_ENOMEM;
    }
    if (s->kt_on) {
        s->err = "launch timing is on; sim_step_noalloc records no timing";
        return SIM_ESTATE;
    }
    s->sink = out;
    s->sink_cap = cap;
    s->sink_n = 0;
    s->scratch_override = (char *)s->na_scratch;
    int rc = SIM_OK;
    try {
        run_steps(s, n_steps, false);
    } catch (const Error &e) {
        s->err = e.msg;
        rc = e.code;
    }
    s->sink = nullptr;
    s->scratch_override = nullptr;
    if (n_out) *n_out = s->sink_n;
    if (rc == SIM_OK && s->sink_n > cap) {
        s->err = "spike buffer too small: the steps were taken, the spikes beyond cap are lost";
        rc = SIM_ENOMEM;
    }
    return rc;
}

int64_t sim_time_steps(const sim_t *s) { return s ? s->step : -1; }

// Calls that need device state refuse a simulation that was only planned.
static bool need_device(sim_t *s) {
    if (!s->planned_only) return true;
    s->err = "a planned simulation has no device state";
    return false;
}

static int read_comp(sim_t *s, const char *src, int64_t cap, int elem, double *out) {
    if (!s || !out) return SIM_EINVAL;
    if (!need_device(s)) return SIM_ESTATE;
    if (cap < s->C) {
        s->err = "capacity smaller than the compartment count";
        return SIM_EINVAL;
    }
    try {
        std::vector<char> host((size_t)s->C * elem);
        HIPCHK(hipMemcpy(host.data(), src, host.size(), hipMemcpyDeviceToHost));
        for (int64_t c = 0; c < s->C; ++c) {
            double v;
            if (elem == 8)
                std::memcpy(&v, host.data() + c * 8, 8);
            else {
                float f;
                std::memcpy(&f, host.data() + c * 4, 4);
                v = f;
            }
            out[s->comp_perm[c]] = v;
        }
        return SIM_OK;
    } catch (const Error &e) {
        s->err = e.msg;
        return e.code;
    }
}

int sim_read_voltages(sim_t *s, double *out, int64_t cap) {
    return s ? read_comp(s, (const char *)s->d_V.p, cap, 8, out) : SIM_EINVAL;
}

int sim_read_gates(sim_t *s, double *m, double *h, double *n, int64_t cap) {
    if (!s) return SIM_EINVAL;
    int rc = read_comp(s, s->d_gm.p, cap, s->tsize, m);
    if (rc == SIM_OK) rc = read_comp(s, s->d_gh.p, cap, s->tsize, h);
    if (rc == SIM_OK) rc = read_comp(s, s->d_gn.p, cap, s->tsize, n);
    return rc;
}

int sim_read_conductances(sim_t *s, double *out, int64_t cap) {
    if (!s || !out) return SIM_EINVAL;
    if (!need_device(s)) return SIM_ESTATE;
    if (cap < s->S) {
        s->err = "capacity smaller than the synapse count";
        return SIM_EINVAL;
    }
    try {
        std::vector<char> host((size_t)s->S * s->tsize);
        if (s->S) HIPCHK(hipMemcpy(host.data(), s->d_sg.p, host.size(), hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < s->S; ++k) {
            double v;
            if (s->tsize == 8)
                std::memcpy(&v, host.data() + k * 8, 8);
            else {
                float f;
                std::memcpy(&f, host.data() + k * 4, 4);
                v = f;
            }
            out[s->syn_perm[k]] = v;
        }
        return SIM_OK;
    } catch (const Error &e) {
        s->err = e.msg;
        return e.code;
    }
}

int sim_spikes(sim_t *s, sim_spike_t *out, int64_t cap, int64_t *n_total) {
    if (!s) return SIM_EINVAL;
    const int64_t total = (int64_t)s->spikes.size();
    if (n_total) *n_total = total;
    if (!out) return SIM_OK;  // count query
    if (cap < total) {
        s->err = "spike buffer too small";
        return SIM_EINVAL;
    }
    if (total) std::memcpy(out, s->spikes.data(), sizeof(sim_spike_t) * (size_t)total);
    return SIM_OK;
}

int sim_neuron_timings(sim_t *s, double *out, int64_t cap, int32_t reset) {
    if (!s || !out || cap < s->N) return SIM_EINVAL;
    if (!need_device(s)) return SIM_ESTATE;
    try {
        std::vector<uint64_t> t(s->packs.size());
        HIPCHK(hipMemcpy(t.data(), s->d_ptime.p, sizeof(uint64_t) * t.size(), hipMemcpyDeviceToHost));
        for (int32_t j = 0; j < s->N; ++j) {
            const int p = s->pack_of_neuron[j];
            const double share = (double)(s->off[j + 1] - s->off[j]) / (double)s->packs[p].ncomp;
            out[j] = (double)t[p] * s->tick_ns * share;
        }
        if (reset) HIPCHK(hipMemset(s->d_ptime.p, 0, sizeof(uint64_t) * t.size()));
        return SIM_OK;
    } catch (const Error &e) {
        s->err = e.msg;
        return e.code;
    }
}

int sim_features(sim_t *s, float *out, int64_t cap) {
    if (!s || !out || cap < (int64_t)s->N * kFeat) return SIM_EINVAL;
    std::memcpy(out, s->feat.data(), sizeof(float) * s->feat.size());
    return SIM_OK;
}

int sim_set_kernel_timing(sim_t *s, int32_t on) {
    if (!s) return SIM_EINVAL;
    if (!need_device(s)) return SIM_ESTATE;
    try {
        HIPCHK(hipStreamSynchronize(s->stream));
        ktimer_reset(s);
    } catch (const Error &e) {
        s->err = e.msg;
        return e.code;
    }
    s->kt_on = on != 0;
    s->kt_used = 0;
    s->kt_ms = 0;
    s->kt_launches = 0;
    for (int c = 0; c < kClasses; ++c) {
        s->kt_cls_ms[c] = 0;
        s->kt_cls_n[c] = 0;
        s->kt_cls_upd[c] = 0;
    }
    return SIM_OK;
}

int sim_class_time(sim_t *s, int32_t cls, double *ms, int64_t *launches, int64_t *comps,
                   int64_t *updates) {
    if (!s || cls < 0 || cls >= kClasses) return SIM_EINVAL;
    if (ms) *ms = s->kt_cls_ms[cls];
    if (launches) *launches = s->kt_cls_n[cls];
    if (comps) *comps = s->cls_comps[cls];
    if (updates) *updates = s->kt_cls_upd[cls];
    return SIM_OK;
}

int sim_kernel_time(sim_t *s, double *ms, int64_t *launches) {
    if (!s) return SIM_EINVAL;
    if (ms) *ms = s->kt_ms;
    if (launches) *launches = s->kt_launches;
    return SIM_OK;
}

const char *sim_config_string(const sim_t *s) { return s ? s->config.c_str() : ""; }

void sim_destroy(sim_t *s) {
    if (!s) return;
    destroy_graphs(s);
    auto fr = [](auto &b) { b.free_(); };
    fr(s->d_packs); fr(s->d_wg_off); fr(s->d_wg_list); fr(s->d_spre); fr(s->d_sdelay);
    fr(s->d_nid); fr(s->d_ndet); fr(s->d_lvl); fr(s->d_lparent); fr(s->d_V); fr(s->d_cdt);
    fr(s->d_e); fr(s->d_len); fr(s->d_diam); fr(s->d_w64);
    fr(s->d_iext64); fr(s->d_q); fr(s->d_gm); fr(s->d_gh); fr(s->d_gn); fr(s->d_af);
    fr(s->d_sg); fr(s->d_sw); fr(s->d_niext); fr(s->d_scratch); fr(s->d_topo); fr(s->d_cnb); fr(s->d_scomp);
    fr(s->d_sseg); fr(s->d_chl); fr(s->d_fw); fr(s->d_cit); fr(s->d_br); fr(s->d_ncomp0); fr(s->d_epoch);
    fr(s->d_ring); fr(s->d_ptime); fr(s->d_ktimer);
    for (int k = 0; k < 2; ++k) {
        if (s->h_stage[k]) (void)hipHostFree(s->h_stage[k]);
        if (s->ev_stage[k]) (void)hipEventDestroy(s->ev_stage[k]);
    }
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    for (int c = 1; c < kClasses; ++c) {
        if (s->ev_join[c]) (void)hipEventDestroy(s->ev_join[c]);
        if (s->side[c]) (void)hipStreamDestroy(s->side[c]);
    }
    for (hipEvent_t e : s->kt_pool) (void)hipEventDestroy(e);
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

const char *sim_last_error(const sim_t *s) { return s ? s->err.c_str() : g_create_error.c_str(); }

// ---- cost model -------------------------------------------------------------
int64_t sim_mlp_nparams(void) { return kMlpParams; }

int sim_mlp_init(float *p, const float *x, const float *y, int64_t n, uint64_t seed) {
    if (!p || !x || !y || n < 2) {
        g_create_error = "sim_mlp_init: need params, x, y and n >= 2";
        return SIM_EINVAL;
    }
    const int F = kFeat, H1 = kH1, H2 = kH2;
    std::memset(p, 0, sizeof(float) * kMlpParams);
    // standardisation of log(1+x) and of the targets
    for (int i = 0; i < F; ++i) {
        double m = 0, v = 0;
        for (int64_t s = 0; s < n; ++s) m += std::log1p((double)x[s * F + i]);
        m /= n;
        for (int64_t s = 0; s < n; ++s) {
            const double d = std::log1p((double)x[s * F + i]) - m;
            v += d * d;
        }
        v = std::sqrt(v / n);
        p[i] = (float)m;
        p[F + i] = (float)(v > 1e-6 ? v : 1.0);
    }
    double ym = 0, yv = 0;
    for (int64_t s = 0; s < n; ++s) ym += y[s];
    ym /= n;
    for (int64_t s = 0; s < n; ++s) yv += (y[s] - ym) * (y[s] - ym);
    yv = std::sqrt(yv / n);
    const int64_t OW1 = 2 * F, OB1 = OW1 + H1 * F, OW2 = OB1 + H1, OB2 = OW2 + H2 * H1,
                  OW3 = OB2 + H2, OB3 = OW3 + H2;
    p[OB3 + 1] = (float)ym;
    p[OB3 + 2] = (float)(yv > 1e-6 ? yv : 1.0);
    // He-uniform weights from a 64-bit linear congruential stream
    uint64_t st = seed * 6364136223846793005ull + 1442695040888963407ull;
    auto uni = [&]() {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(st >> 11) * (1.0 / 9007199254740992.0);
    };
    auto fill = [&](int64_t off, int64_t count, int fan_in) {
        const double a = std::sqrt(6.0 / fan_in);
        for (int64_t i = 0; i < count; ++i) p[off + i] = (float)((2 * uni() - 1) * a);
    };
    fill(OW1, (int64_t)H1 * F, F);
    fill(OW2, (int64_t)H2 * H1, H1);
    fill(OW3, H2, H2);
    return SIM_OK;
}

int sim_mlp_forward(const float *p, const float *x, int64_t n, float *out) {
    if (!p || (!x && n) || (!out && n) || n < 0) return SIM_EINVAL;
    hipError_t e = mlp_forward(p, x, n, out);
    if (e != hipSuccess) {
        g_create_error = hipGetErrorString(e);
        return SIM_EDEVICE;
    }
    return SIM_OK;
}

int sim_mlp_loss_grad(const float *p, const float *x, const float *y, int64_t n, float *loss,
                      float *grad) {
    if (!p || !x || !y || !loss || !grad || n < 1) return SIM_EINVAL;
    hipError_t e = mlp_loss_grad(p, x, y, n, loss, grad);
    if (e != hipSuccess) {
        g_create_error = hipGetErrorString(e);
        return SIM_EDEVICE;
    }
    return SIM_OK;
}

int sim_mlp_train(float *p, const float *x, const float *y, int64_t n, int32_t epochs, float lr,
                  float *final_loss) {
    if (!p || !x || !y || n < 1 || epochs < 0 || !(lr > 0)) return SIM_EINVAL;
    hipError_t e = mlp_train(p, x, y, n, epochs, lr, final_loss);
    if (e != hipSuccess) {
        g_create_error = hipGetErrorString(e);
        return SIM_EDEVICE;
    }
    return SIM_OK;
}

}  // extern "C"
