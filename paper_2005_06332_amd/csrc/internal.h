// Internal layout shared by the host side of the library and its kernels.
//
// Device memory holds every neuron in *packed* order: neurons are grouped
// into packs (one pack = the unit a workgroup advances through an epoch), and
// a pack's compartments are contiguous (structure-of-arrays, one array per
// quantity, so consecutive threads touch consecutive addresses). Inside a
// neuron the compartments keep their input (Hines) order, parent(i) < i.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmh {

// Topology word of a compartment (pack-local indices, < 32767):
//   bits  0..14  parent compartment, or the neuron's index within the pack
//                when the compartment is a root
//   bit   15     Hodgkin-Huxley channels (else passive)
//   bits 16..30  branch id when the compartment ends a branch (kNone when its
//                only child is the next compartment)
//   bit   31     root of a neuron
constexpr uint32_t kNone = 0x7FFF;
__host__ __device__ inline uint32_t topo_parent(uint32_t t) { return t & 0x7FFFu; }
__host__ __device__ inline bool topo_hh(uint32_t t) { return (t >> 15) & 1u; }
__host__ __device__ inline uint32_t topo_branch(uint32_t t) { return (t >> 16) & 0x7FFFu; }
__host__ __device__ inline bool topo_root(uint32_t t) { return (t >> 31) & 1u; }
__host__ __device__ inline uint32_t make_topo(uint32_t parent_or_neuron, bool hh,
                                              uint32_t branch, bool root) {
    return (parent_or_neuron & 0x7FFFu) | (hh ? 0x8000u : 0u) |
           ((branch & 0x7FFFu) << 16) | (root ? 0x80000000u : 0u);
}

// Children word of a compartment: its first two children (pack-local, in
// ascending order; kNoNb when absent) as c1 | c2 << 16, or kManyChildren
// when it has more than two (their bases are then read from the branch
// record the topology word names).
constexpr uint32_t kManyChildren = 0xFFFFFFFEu;
__host__ __device__ inline uint32_t make_children(uint32_t c1, uint32_t c2) {
    return (c1 & 0xFFFFu) | ((c2 & 0xFFFFu) << 16);
}

// A branch: a maximal run b0..b1 of consecutive compartments where each one
// is the only child of the previous. Branch records of a pack are stored in
// backward-sweep order (by height, longest chains first within a level), and
// a branch's id is its position there. Its children (branches whose base
// hangs off b1) occupy child-list entries child0 .. child0+nchild-1 in
// ascending order of their bases; the entries hold the children's base
// compartments, and cb[0], cb[1] repeat the first two. par is the parent
// compartment of b0, or kRootPar when b0 is the root of its neuron.
constexpr uint16_t kRootPar = 0xFFFF;
struct alignas(16) Branch {
    uint16_t b0, b1, child0, nchild, par, pad;
    uint16_t cb[2];
};

struct PackDesc {
    int64_t comp0;   // first compartment (packed index)
    int64_t syn0;    // first synapse (packed index)
    int32_t ncomp, nsyn;
    int32_t neur0, nneur;  // packed neuron range
    int32_t br0, nbr;      // branch table range (records and forward order)
    int32_t ch0;           // child list / child contribution offset
    int32_t lv0;           // level offsets: nbw+1 backward, nfw+1 forward, then
                           // nrnd+1 contraction round offsets
    int32_t nbw, nfw;      // number of height / depth levels
    int32_t global_mem;    // 0: state in LDS; k > 0: state in global scratch slice k-1
    int32_t nch;           // child list entries
    int32_t tbytes;        // bytes of staged tables (always in LDS)
    int32_t it0, nrnd;     // contraction solver: first item, rounds (0: other solvers)
    int32_t nrw;           // contraction rounds [0, nrw) run by the whole workgroup,
                           // rounds [nrw, nrnd) (at most kWave - 1 of them, at
                           // most kWave items each, all staged in LDS) by its
                           // first wavefront alone, with no workgroup barrier
    int32_t nst;           // contraction: the last nst items staged in LDS
};

// Lanes of a wavefront on gfx950.
constexpr int kWave = 64;

// Contraction solver item, one per compartment of a pack: bits 0..14 the
// eliminated compartment k, bit 15 set when n1 is k's current parent, bits
// 16..31 n1, bits 32..47 n2 (pack-local; kNoNb when absent), bit 49 (50) set
// when the coupling to n1 (n2) was made by an earlier elimination of the
// step (it is then in the working slot, else it is the off-diagonal). Items
// are stored by round; round r of a pack spans items rof[r] .. rof[r+1]-1.
constexpr uint32_t kNoNb = 0xFFFF;
// The same item as the epoch kernel reads it, in a pack of n compartments
// whose state arrays have m = n + 1 entries: entry n is a spare compartment
// that stands in for an absent neighbour (its off-diagonal entry is 0, so
// the coupling it is read with is 0 and every update it takes is void).
// Bits 0..14 k, 15..30 i1 (n1, or n when absent), 31..46 i2 (likewise),
// 47..62 u1: where the coupling to n1 is read, as an index into the working
// slot W followed by the off-diagonal (the two arrays are adjacent: u < m is
// W[u], u >= m the off-diagonal entry u - m); bit 63 set when the coupling
// to n2 is W[i2] (else the off-diagonal entry of i2).
__host__ __device__ inline uint64_t make_citem(uint32_t k, uint32_t i1, uint32_t i2, uint32_t u1,
                                               bool w2) {
    return (uint64_t)(k & 0x7FFFu) | ((uint64_t)(i1 & 0xFFFFu) << 15) |
           ((uint64_t)(i2 & 0xFFFFu) << 31) | ((uint64_t)(u1 & 0xFFFFu) << 47) |
           (w2 ? (1ull << 63) : 0ull);
}
__host__ __device__ inline uint64_t make_item(uint32_t k, bool n1_parent, uint32_t n1,
                                              uint32_t n2, bool f1 = false, bool f2 = false) {
    return (uint64_t)(k & 0x7FFFu) | (n1_parent ? 0x8000ull : 0ull) | ((uint64_t)n1 << 16) |
           ((uint64_t)n2 << 32) | (f1 ? (1ull << 49) : 0ull) | (f2 ? (1ull << 50) : 0ull);
}

// Everything the epoch kernel reads or writes. T is the gating precision.
struct EpochArgs {
    const PackDesc *packs;
    const int32_t *wg_off;   // [n_wg+1] ranges into wg_list
    const int32_t *wg_list;  // pack ids in execution order
    // per compartment (packed)
    double *V;
    void *gm, *gh, *gn;
    const uint32_t *topo;
    const uint32_t *cnb;  // children words
    const double *cdt;  // C/dt (uS)
    const double *e;    // off-diagonal -theta*G (G = coupling to parent, uS), 0 at roots
    const void *af;     // area factor (T)
    // per synapse (packed: by pack, target compartment, synapse id)
    void *sg;                 // conductance (T)
    const void *sw;           // weight (T)
    const int32_t *spre;      // presynaptic neuron (input id)
    const int32_t *sdelay;
    const uint16_t *scomp;    // pack-local target compartment
    const uint16_t *sseg;     // run length of equal targets at a run start, else 0
    // per neuron (packed)
    const int32_t *nid;       // input id
    const int32_t *ndet;      // pack-local detector compartment
    const void *niext;        // injected current (T)
    // per pack tables
    const Branch *br;
    const uint16_t *fw;  // forward-sweep order: record ids by depth, longest chains first
    const uint16_t *chl;
    const int32_t *lvl;
    const uint64_t *cit;   // contraction items (by pack, by round); the round
                           // offsets follow a pack's level offsets in lvl
    // spike history, a ring of ring_rows epochs: ring[(epoch mod ring_rows)
    // * n_neurons + input id] = bit t set when the neuron spiked at step
    // epoch*E + t + 1. ring_rows exceeds the epochs any delay looks back.
    uint64_t *ring;
    int32_t ring_rows;
    int32_t n_neurons;
    int32_t E;
    const int64_t *epoch_ptr;  // when non-null, the epoch index is read here
    int64_t epoch;
    int32_t t0, t1;            // steps [t0, t1) of the epoch
    // scratch for packs too large for LDS: slice k-1 of scratch_stride bytes
    char *scratch;
    int64_t scratch_stride;
    // constants
    double omt;        // 1 - theta
    double ginv;       // -1/theta (exact: theta is 1/2 or 1)
    double v_thresh;
    double gnabar, gkbar, gl, ena, ek, el, g_pas, e_pas, e_syn, dt, q;
    float fch[11];     // the same eleven, rounded to float (FP32 gating)
    // timing
    uint64_t *pack_time;  // accumulated ns per pack, or null
    // launch timer of this size class (device clock ticks): [0] start (set
    // by k_stamp just before the launch, or the earliest workgroup start),
    // [1] latest workgroup end, [2] finished workgroups of the running
    // launch, [4] summed launch spans, [5] launches
    uint64_t *ktimer;
};

// Bytes of per-pack state for a pack of n compartments, s synapses and k
// neurons in precision T (must match the carve-up in the kernel).
// (The contraction solver's packs pass n + 1: their arrays end with a spare
// compartment.)
template <typename T>
__host__ __device__ inline int64_t pack_state_bytes(int64_t n, int64_t s, int64_t k) {
    int64_t b = 4 * 8 * n;                 // V, off-diagonal, R, D
    b += 8 * s + 8 * k + 8 * k;            // synapse masks, spike masks, V_det
    b += 8 * k + 8 * k;                    // external current, detector index
    b += ((int64_t)sizeof(T) * s + 15) / 16 * 16;  // synaptic conductances
    b += 64;  // slack: the blocked sweeps read up to 3 doubles past a branch
    return b;
}
// Bytes of the pack's tables staged in LDS next to the state: branch records,
// synapse weights (T), level offsets, the forward order, child list, synapse
// targets and run lengths. Must match the carve-up in the kernel.
// The contraction solver adds its round offsets (nrnd + 1 ints) and the
// items staged in LDS (nst; the others stay in global memory), and stages no
// branch records, forward order, child list or level offsets (nbr = nch =
// nlev = 0); nrnd = 0 for the other solvers.
template <typename T>
__host__ __device__ inline int64_t pack_table_bytes(int64_t nbr, int64_t nch, int64_t nlev,
                                                    int64_t nsyn, int64_t ncomp = 0,
                                                    int64_t nrnd = 0, int64_t nst = 0) {
    int64_t b = (int64_t)sizeof(Branch) * nbr;
    b += (int64_t)sizeof(T) * nsyn;
    b = (b + 3) / 4 * 4 + 4 * nlev;
    b += 2 * nbr + 2 * nch + 2 * 2 * nsyn;
    if (nrnd > 0) b = (b + 3) / 4 * 4 + 4 * (nrnd + 1);
    if (nst > 0) b = (b + 7) / 8 * 8 + 8 * nst;
    (void)ncomp;
    return (b + 15) / 16 * 16;
}

struct SetupArgs {
    int32_t n_neurons;          // packed neuron count
    const int64_t *ncomp0;      // [n+1] packed compartment offsets per neuron
    const int32_t *lparent;     // neuron-local parent per compartment
    const double *length, *diam;
    double cm, ra, dt, theta, v_init;
    double *cdt, *e, *V;
    void *af, *gm, *gh, *gn;
    double *q_out;              // exp(-dt/tau)
    double tau;
};

// Launchers (kernels.hip).
hipError_t launch_setup(const SetupArgs &a, int precision, hipStream_t s);
// solver: 0 = exact operation order of the elimination, 1 = division-free
// homogeneous form, 2 = tree contraction
// resident: the launch's packs all keep their state in LDS and have at most
// kResident compartments per thread (FP32 gating, contraction solver only),
// which selects a kernel without the global-state and non-resident paths
hipError_t launch_epoch(const EpochArgs &a, int precision, int solver, int n_wg, int threads,
                        size_t lds_bytes, bool resident, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_advance(int64_t *epoch, hipStream_t s);
hipError_t launch_stamp(uint64_t *timer, hipStream_t s);
hipError_t launch_decay_weights_convert(const double *w, void *out, int64_t n,
                                        int precision, hipStream_t s);
hipError_t set_epoch_lds_limit(int bytes);
// Device address of the fixed scratch array of the current device (resolved
// once per device); kNoAllocScratchBytes long.
constexpr int64_t kNoAllocScratchBytes = (int64_t)64 << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(void **ptr);
// Compartments per thread whose gates and constants the epoch kernel keeps in
// registers for a whole epoch (FP32 gating, contraction solver).
constexpr int kResident = 4;
// Largest epoch-kernel workgroup (launch bounds): double precision needs
// more registers per lane.
constexpr int kMaxThreadsF32 = 1024;
constexpr int kMaxThreadsF64 = 512;

// MLP (mlp.hip).
constexpr int kFeat = 16, kH1 = 64, kH2 = 64;
constexpr int64_t kMlpParams = 16 + 16 + kH1 * kFeat + kH1 + kH2 * kH1 + kH2 + kH2 + 1 + 2;

}  // namespace mmh
