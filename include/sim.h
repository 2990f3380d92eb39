/*
 * mmhines — C ABI of the MI355X multi-morphology compartmental simulator.
 *
 * The library advances a network of branched neurons through time. Each step
 * it performs, per neuron and on the GPU (gfx950):
 *   1. synaptic delivery: a synapse whose presynaptic neuron spiked exactly
 *      `delay_steps` steps earlier adds its weight to its conductance
 *      (the paper's two-level stepping, Section 2: spikes travel with a
 *      network delay and are exchanged once per global step);
 *   2. Hodgkin-Huxley gating and membrane current per compartment (the
 *      current I of the cable equation, Eq. 1);
 *   3. assembly of the per-compartment system of Eq. 2 and its right-hand
 *      side on the neuron's parent vector p;
 *   4. the Hines elimination and back-substitution (Algorithm 1);
 *   5. spike detection by threshold crossing (Section 2, after Algorithm 1).
 * Neurons are independent inside an epoch of E <= min(delay) steps, so one
 * kernel launch advances every neuron by a whole epoch; the spike history is
 * exchanged through device memory between epochs.
 *
 * Conventions for every call:
 *  - return 0 on success or a negative SIM_E* code; sim_last_error() then
 *    describes the failure in a library-owned string;
 *  - input arrays are borrowed for the duration of the call and copied;
 *  - output buffers are caller-allocated host memory with an explicit
 *    capacity `cap` in elements;
 *  - neuron ids and compartment order are always the caller's input order,
 *    never the library's internal (packed) order;
 *  - calls on one sim_t are not thread-safe; distinct sim_t are independent;
 *  - the library uses the HIP runtime the process has loaded under the soname
 *    libamdhip64.so.7; a stream passed in (sim_params_t.hip_stream) must come
 *    from that same runtime, so a host that brings its own copy (as torch
 *    does) loads it before this library;
 *  - results (voltages, spikes) are bitwise independent of the packing mode,
 *    the autotuner and the cost model.
 */
#ifndef MMHINES_SIM_H
#define MMHINES_SIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_OK 0
#define SIM_EINVAL (-1)  /* bad argument, topology or size */
#define SIM_ENOMEM (-2)  /* host or device allocation failed / size cap */
#define SIM_EDEVICE (-3) /* HIP runtime error or no usable gfx950 device */
#define SIM_ESTATE (-4)  /* call made in the wrong state */

#define SIM_FP64 0          /* gates, rates and currents in double */
#define SIM_FP32_GATING 1   /* gates, rates, currents, synaptic g in float;
                               voltage, assembly and Hines solve in double */

#define SIM_SOLVE_EXACT 0   /* elimination in the operation order of the
                               paper's Algorithm 1 (a division per
                               compartment on the dependent chain) */
#define SIM_SOLVE_FAST 1    /* the same elimination in division-free
                               homogeneous form: one fused multiply-add per
                               compartment on each dependent chain; agrees
                               with the exact order to rounding */
#define SIM_SOLVE_CONTRACT 2 /* the same linear system (Eq. 2) eliminated by
                               parallel tree contraction: rounds of
                               compartments of degree <= 2, at least three
                               apart, then back substitution in reverse;
                               agrees with the exact order to rounding */

#define SIM_PACK_PLAIN 0    /* neurons in input order, one workgroup per pack,
                               hardware dispatch order */
#define SIM_PACK_COUNT 1    /* neurons by decreasing compartment count go
                               best-fit into packs that fill the LDS budget
                               of their size class; packs run in decreasing
                               summed compartment count (dispatch or LPT) */
#define SIM_PACK_LEARNED 2  /* the same packs, run in decreasing predicted
                               time (the MLP's largest prediction among a
                               pack's neurons); falls back to COUNT when no
                               model is given */

#define SIM_SCHED_AUTO 0       /* chosen by the autotuner, else DISPATCH */
#define SIM_SCHED_PERSISTENT 1 /* one resident workgroup per slot; static LPT
                                  lists of packs */
#define SIM_SCHED_DISPATCH 2   /* one workgroup per pack in cost order */

typedef struct sim sim_t; /* opaque, owned by the library */

/* Morphologies in compressed-row form (the paper's parent vector p per
 * neuron, "Hines matrix" paragraph of Section 2). For neuron j its
 * compartments are comp_offset[j] .. comp_offset[j+1]-1. */
typedef struct {
    int32_t n_neurons;           /* >= 1 */
    const int64_t *comp_offset;  /* [n_neurons+1], comp_offset[0] = 0, strictly
                                    increasing; at most 32767 compartments per
                                    neuron */
    const int32_t *parent;       /* [total] neuron-local parent index:
                                    parent[first] = -1, 0 <= parent[i] < i */
    const double *length_um;     /* [total] > 0, finite */
    const double *diam_um;       /* [total] > 0, finite */
    const uint8_t *mech;         /* [total] 0 passive leak, 1 Hodgkin-Huxley */
    const int32_t *detector;     /* [n_neurons] local compartment watched for
                                    spikes */
    const double *i_ext_nA;      /* [n_neurons] constant current into the
                                    neuron's compartment 0 */
} sim_morphology_t;

/* Membrane and channel constants (densities in S/cm^2, potentials in mV). */
typedef struct {
    double cm_uF_cm2, ra_ohm_cm;
    double gnabar, gkbar, gl, ena, ek, el; /* Hodgkin-Huxley compartments */
    double g_pas, e_pas;                   /* passive compartments */
} sim_channels_t;

/* Conductance-based exponential synapses, one record per synapse; the
 * record index is the synapse id used for the order of simultaneous events
 * (ascending id). */
typedef struct {
    int64_t n;
    const int32_t *pre;          /* [n] presynaptic neuron */
    const int32_t *post;         /* [n] postsynaptic neuron */
    const int32_t *post_comp;    /* [n] local compartment of `post` */
    const int32_t *delay_steps;  /* [n] >= 1 */
    const double *weight_uS;     /* [n] >= 0, finite */
} sim_synapses_t;

typedef struct {
    double dt_ms;        /* > 0 */
    double theta;        /* axial time weighting: 0.5 (Crank-Nicolson, the
                            factor 2 of Eq. 2) or 1.0 (backward Euler) */
    double tau_syn_ms;   /* > 0 */
    double e_syn_mV;
    double v_thresh_mV;  /* spike when V crosses it upward at the detector */
    double v_init_mV;    /* initial voltage; gates start at steady state */
    int32_t precision;   /* SIM_FP64 | SIM_FP32_GATING */
    int32_t solver;      /* SIM_SOLVE_EXACT | SIM_SOLVE_FAST | SIM_SOLVE_CONTRACT */
    int32_t packing;     /* SIM_PACK_* */
    int32_t sched;       /* SIM_SCHED_* */
    int32_t epoch_steps; /* 0: min(delay) capped at 64; else 1..min(delay),
                            <= 64 */
    int32_t autotune;    /* 1: time trial epochs over launch variants at
                            create and keep the fastest */
    int32_t threads;     /* workgroup size 64..1024 (multiple of 64; at most 512
                            in SIM_FP64), 0 = 256 */
    int32_t pack_comps;  /* plain packing: target compartments per pack,
                            0 = 800. Count and learned packing: cap on a
                            pack's compartments, 0 = none (packs are filled
                            best-fit to their LDS budget) */
    int32_t lds_comps;   /* LDS budget of the smallest pack class, in
                            compartments (the two larger classes get 2x and
                            4x, capped by the CU's LDS); packs beyond every
                            budget use global scratch. 0 = 1100 */
    int32_t lds_classes; /* size classes in use, 1..3 (0 = 2); packs beyond
                            the largest budget in use keep their state in
                            global scratch inside that class's launch */
    int32_t use_graph;   /* 1: replay whole epochs from a captured hipGraph */
    int32_t record_timings; /* 1: per-pack wall-clock time in the kernel */
    const float *cost_model;   /* MLP parameters (sim_mlp_nparams floats) for
                                  SIM_PACK_LEARNED, or NULL */
    void *hip_stream;    /* hipStream_t to launch on; NULL = the library's
                            own stream */
    const double *neuron_cost; /* SIM_PACK_LEARNED: per-neuron costs
                                  (n_neurons finite values > 0, input order)
                                  used in place of the cost model's
                                  predictions, e.g. measured times; NULL =
                                  the model */
} sim_params_t;

typedef struct {
    int32_t neuron; /* input order */
    int32_t step;   /* spike happened during the transition step-1 -> step */
} sim_spike_t;

/* Fill *p with defaults (FP32 gating, COUNT packing, autotune off).
 * Source: the numerical parameters of Eq. 2 (dt, theta) and of Section 2's
 * two-level stepping; the remaining fields are launch options of this library. */
void sim_default_params(sim_params_t *p);

/* Validate the network, lay it out on the device, compute the time-invariant
 * coefficients on the GPU and initialise the state (V = v_init, gates at
 * steady state, conductances 0). Every validation failure is reported before
 * any device allocation. On success *out owns the simulation.
 * Source: the problem as Section 2 states it: neurons with their parent
 * vectors p (Hines-matrix paragraph), the coefficients of Eq. 2 that do not
 * change in time (off-diagonals from the geometry), synapses with a network
 * delay (local/global steps). */
int sim_create(const sim_params_t *params, const sim_morphology_t *morph,
               const sim_channels_t *channels, const sim_synapses_t *syn,
               sim_t **out);

/* ---------------------------------------------------------------------------
 * Layout planning and introspection (host only). Source: the load-balancing
 * step of Section 4 (neurons sorted by size before they are scheduled) and
 * this library's packing of neurons into workgroups; the contraction
 * schedule is the elimination order of the solver SIM_SOLVE_CONTRACT for the
 * matrix of Eq. 2.
 * ------------------------------------------------------------------------- */

/* Validate and lay out the problem exactly as sim_create would for a device
 * with `lds_bytes_per_cu` bytes of LDS per compute unit and `n_cu` compute
 * units, without any device call: packing, size classes, workgroup lists
 * and (for SIM_SOLVE_CONTRACT) elimination schedules. The result answers
 * the introspection calls below and sim_config_string; calls that need
 * device state return SIM_ESTATE. Autotuning and learned packing with a
 * cost model need the device and are refused (SIM_EINVAL). */
int sim_plan_create(const sim_params_t *params, const sim_morphology_t *morph,
                    const sim_channels_t *channels, const sim_synapses_t *syn,
                    int32_t lds_bytes_per_cu, int32_t n_cu, sim_t **out);

typedef struct {
    int32_t first_position; /* position of the pack's first neuron in the
                               packed neuron order */
    int32_t n_neurons, n_comp, n_syn, n_branches;
    int32_t size_class;     /* 0..2: the launch that runs the pack */
    int32_t in_global;      /* 1: state in global scratch, tables in LDS */
    int32_t n_rounds;       /* contraction rounds (0 for the other solvers) */
    int32_t n_levels;       /* height levels + depth levels + 2 */
    int32_t n_child_entries; /* child-branch list entries */
    int64_t table_bytes;    /* LDS bytes of the pack's tables */
    int64_t state_bytes;    /* bytes of its state (LDS unless in_global) */
    double cost;            /* packing cost (compartments, or predicted time) */
    int32_t n_wide_rounds;  /* contraction: leading rounds run by the whole
                               workgroup; the later ones (at most 64 items
                               each, every item staged in LDS) by its first
                               wavefront alone */
    int32_t n_staged_items; /* contraction: the last items of the pack's
                               schedule (the single-wavefront tail) copied
                               to LDS, as many as the class's LDS budget
                               leaves room for; the rest stay in global
                               memory */
} sim_pack_info_t;

/* Number of packs (workgroup units of work). */
int32_t sim_pack_count(const sim_t *sim);
/* Description of pack `pack` (0 .. count-1). */
int sim_pack_info(const sim_t *sim, int32_t pack, sim_pack_info_t *out);
/* Input ids of the pack's neurons, in their order inside the pack. */
int sim_pack_neurons(const sim_t *sim, int32_t pack, int32_t *ids, int64_t cap);
/* Workgroups, threads per workgroup and dynamic LDS bytes of size class cls
 * (0..2); any output may be NULL. */
int sim_class_launch(const sim_t *sim, int32_t cls, int32_t *n_wg, int32_t *threads,
                     int64_t *lds_bytes);
/* Packs that workgroup `wg` of class `cls` runs, in order; *n receives the
 * count; packs == NULL only queries it. */
int sim_workgroup_packs(const sim_t *sim, int32_t cls, int32_t wg, int32_t *packs,
                        int64_t cap, int32_t *n);
/* Elimination schedule of neuron `neuron` (input id) under
 * SIM_SOLVE_CONTRACT (SIM_ESTATE otherwise): items[4q .. 4q+3] = (k, n1, n2,
 * flags) for the q-th eliminated compartment, neuron-local, -1 for an
 * absent neighbour; flags bit 0: n1 is k's current parent, bit 1 (bit 2):
 * k's coupling to n1 (n2) was made by an earlier elimination rather than
 * being the off-diagonal. Round r spans items round_off[r] .. round_off[r+1]-1.
 * cap >= 4 * compartments, cap_rounds >= rounds + 1; items == NULL only
 * queries *n_rounds. */
int sim_contraction_schedule(const sim_t *sim, int32_t neuron, int32_t *items, int64_t cap,
                             int32_t *round_off, int64_t cap_rounds, int32_t *n_rounds);
/* The contraction items of pack `pack` as the epoch kernel reads them, in
 * execution order (round by round), for a simulation laid out with
 * sim_plan_create under SIM_SOLVE_CONTRACT (SIM_ESTATE otherwise). One
 * 64-bit item per compartment, pack-local indices: bits 0..14 the
 * eliminated compartment k; bits 15..30 and 31..46 its two neighbours at
 * elimination time, where the pack's spare compartment n_comp stands for an
 * absent one; bits 47..62 where the coupling to the first neighbour is read,
 * as an index into the working couplings (below n_comp + 1) followed by the
 * off-diagonal (index - n_comp - 1); bit 63 set when the coupling to the
 * second neighbour is a working coupling (else its off-diagonal entry).
 * *n receives the count; items == NULL only queries it.
 * Host-only introspection of this library's layout (no passage of the
 * paper defines it). */
int sim_pack_contraction_items(const sim_t *sim, int32_t pack, uint64_t *items, int64_t cap,
                               int64_t *n);

/* Advance by n_steps (>= 0) time steps; returns when the work is complete
 * on the device, with the steps' spikes recorded (see sim_spikes).
 * Source: one local step of Section 2 per time step: delivery, the current
 * I of Eq. 1, assembly of Eq. 2, Algorithm 1, then spike detection (the
 * paragraph after Algorithm 1); spikes reach their targets after their
 * delay (the local and global buffers of Section 2.1). Device memory does
 * not grow with the number of steps. */
int sim_step(sim_t *sim, int64_t n_steps);

/* sim_step for callers that cannot allocate memory (code running under HIP
 * graph capture, tight serving loops, hosts that forbid allocation): the
 * same steps, kernels and results as sim_step, with no device, pinned or host
 * allocation and no hipMalloc/hipFree. Differences:
 *  - epochs are launched directly (never captured or replayed);
 *  - the state of packs too large for LDS lives in a fixed array of this
 *    library, 64 MiB per GPU (kNoAllocScratchBytes), held by every GPU the
 *    library runs on until the process ends; a simulation whose such packs
 *    need more returns SIM_ENOMEM before taking any step;
 *  - the spikes of this call are written to out[0 .. cap-1] in (step, neuron)
 *    order and *n_out receives their count; they are not added to the list
 *    sim_spikes returns. If the count exceeds cap the steps are still taken,
 *    the spikes beyond cap are lost and SIM_ENOMEM is returned (cap >=
 *    n_neurons * n_steps can never overflow);
 *  - launch timing must be off (SIM_ESTATE otherwise).
 * Every call on one GPU shares that GPU's array: calls on different
 * simulations that overlap in time on one GPU race and must be serialised by
 * the caller. Nothing in the array needs clearing between calls: each launch
 * loads a pack's state before it reads it. */
int sim_step_noalloc(sim_t *sim, int64_t n_steps, sim_spike_t *out, int64_t cap,
                     int64_t *n_out);

/* Steps simulated so far (local steps dt of Section 2). */
int64_t sim_time_steps(const sim_t *sim);

/* Membrane voltages (mV) of every compartment, input order; cap >= total.
 * Source: the unknowns V of Eq. 2 (the solution of Algorithm 1's forward
 * sweep) after the last step. */
int sim_read_voltages(sim_t *sim, double *out_mV, int64_t cap);

/* Gate states (m, h, n) of every compartment as double, input order.
 * Source: the state behind the membrane current I of Eq. 1 (the paper
 * names no channel model; the Hodgkin-Huxley reading is this library's). */
int sim_read_gates(sim_t *sim, double *m, double *h, double *n, int64_t cap);

/* Synaptic conductances (uS), synapse id order.
 * Source: the per-synapse work of Section 2 (the S term of the operation
 * count per global step). */
int sim_read_conductances(sim_t *sim, double *out_uS, int64_t cap);

/* All spikes so far, sorted by (step, neuron). *n_total always receives the
 * count; out == NULL only queries it; SIM_EINVAL if cap is too small
 * (nothing written then).
 * Source: Section 2, the paragraph after Algorithm 1 (a spike is a threshold
 * crossing of the voltage) and the spike events stored per global step. */
int sim_spikes(sim_t *sim, sim_spike_t *out, int64_t cap, int64_t *n_total);

/* Per-neuron kernel time in nanoseconds accumulated since create (or since
 * the last reset), when record_timings is on. A neuron sharing a pack with
 * others is charged the pack time split in proportion to compartments.
 * Source: not a call the paper defines; it feeds the learned cost model of
 * the benchmark specification (trained on per-neuron timings), the analogue
 * of the per-task traces of Section 3's performance analysis. */
int sim_neuron_timings(sim_t *sim, double *out_ns, int64_t cap, int32_t reset);

/* The 16 morphology features of every neuron (input order, row-major
 * [n_neurons][16], float) that the cost model consumes.
 * Source: the benchmark specification's cost model inputs (compartment
 * count, depth, branch count, longest branch, ...); the paper itself uses
 * only the size (Section 4, sorting by size). */
int sim_features(sim_t *sim, float *out, int64_t cap);

/* Launch timing, off by default. Source: measurement call of this library
 * (not defined by the paper). While on, sim_step records HIP events on
 * the simulator's stream around each graph replay (or directly launched
 * epoch), and sim_step reads them back before it returns. Each size-class
 * launch also times itself on the device: the span from a one-thread stamp
 * kernel run just before it on its stream (so a wait for resources held by
 * the concurrent launch counts) to its last workgroup's end, in the
 * device's constant clock. The epoch kernel keeps these totals always, and
 * graph replays carry them, where events inside a graph are not updated by
 * replays. Turning it on (again) waits for the stream and resets all
 * totals. */
int sim_set_kernel_timing(sim_t *sim, int32_t on);
/* Total device time (ms) of the epochs (fork to join of the concurrent
 * size-class launches) and their count.
 * Source: measurement call of this library (not defined by the paper). */
int sim_kernel_time(sim_t *sim, double *ms, int64_t *launches);
/* For size class cls (0..2, 0 = the smallest LDS budget, normally holding
 * most packs): total device time (ms) of its launches (stamp before the
 * launch to its last workgroup's end), their count, the compartments the class
 * advances per step, and the compartment-updates its timed launches performed
 * (compartments x the steps each launch ran). Any output may be NULL.
 * Source: measurement call of this library (not defined by the paper). */
int sim_class_time(sim_t *sim, int32_t cls, double *ms, int64_t *launches, int64_t *comps,
                   int64_t *updates);

/* Launch configuration actually used (after autotuning), as text.
 * Source: measurement call of this library (not defined by the paper). */
const char *sim_config_string(const sim_t *sim);

/* Release the simulation and its device memory. */
void sim_destroy(sim_t *sim);

/* Description of the last failure on `sim` (or, when sim is NULL, of the
 * calling thread's last failed call without a handle: sim_create or a cost
 * model call). Library-owned; valid until the next call.
 * Source: error reporting of this library (not defined by the paper). */
const char *sim_last_error(const sim_t *sim);

/* ---------------------------------------------------------------------------
 * Cost model: a 16-64-64-1 multilayer perceptron (ReLU) in float, trained on
 * the GPU with the library's own forward, backward and Adam kernels. Inputs
 * are the sim_features() rows; the model standardises them internally and
 * predicts log(kernel time). Parameter vector layout (sim_mlp_nparams floats):
 *   x_mean[16] x_std[16] W1[64][16] b1[64] W2[64][64] b2[64] W3[64] b3[1]
 *   y_mean y_std
 * ------------------------------------------------------------------------- */
int64_t sim_mlp_nparams(void);

/* Initialise parameters (He-uniform weights from `seed`, zero biases) and
 * the standardisation from the training set. */
int sim_mlp_init(float *params, const float *x, const float *y, int64_t n,
                 uint64_t seed);

/* Predictions (log time) for n feature rows. */
int sim_mlp_forward(const float *params, const float *x, int64_t n,
                    float *out);

/* Mean squared error on standardised targets and its gradient with respect
 * to the trainable parameters (the same layout; standardisation entries get
 * zero gradient). */
int sim_mlp_loss_grad(const float *params, const float *x, const float *y,
                      int64_t n, float *loss, float *grad);

/* Full-batch Adam training for `epochs` iterations; params updated in place;
 * final loss returned. */
int sim_mlp_train(float *params, const float *x, const float *y, int64_t n,
                  int32_t epochs, float lr, float *final_loss);

#ifdef __cplusplus
}
#endif
#endif
