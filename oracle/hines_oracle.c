/*
 * Serial CPU oracle of the compartmental network simulation.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
 * GPU library is checked against. Only the test suite, the package smoke
 * check and the benchmark's CPU-baseline leg may build, load or call it. It
 * shares no code, header, table or constant generator with the GPU library.
 *
 * What it computes, in the paper's terms (arXiv 2005.06332, Section 2):
 *   - the cable equation (Eq. 1) discretised per compartment into the
 *     three-point system of Eq. 2 with the coefficient definitions that
 *     follow it: off-diagonals constant in time, diagonal and right-hand side
 *     rebuilt every step, a factor 2 on the axial term (Crank-Nicolson,
 *     theta = 1/2);
 *   - branching morphologies numbered so that parent(i) < i, described by the
 *     parent vector p (the "Hines matrix" paragraph);
 *   - the Hines algorithm (Algorithm 1): backward sweep over i = n-1 .. 1,
 *     one division at the root, forward sweep over i = 1 .. n-1;
 *   - spike detection after the voltage solve (the paragraph after
 *     Algorithm 1): an upward threshold crossing at the detector compartment;
 *   - two-level time stepping (Section 2, "local" and "global" steps): spikes
 *     reach their targets after an integer synaptic delay.
 * Points the paper leaves open are fixed as follows (each a reading, not a
 * statement of the paper): Hodgkin-Huxley sodium/potassium/leak channels or a
 * passive leak per compartment; conductance-based exponential synapses; the
 * membrane current is linear in V once the gates of step n are fixed
 * (I = g V - J) and is taken at V^{n+1}, which puts the membrane conductance
 * g on the diagonal and is why the diagonal changes every step; per step the
 * order is
 *   deliver -> (g, J at gates^n) -> assemble -> solve -> gates(V^{n+1})
 *   -> synaptic decay -> detect;
 * gates by exponential Euler; finite-volume geometry (area pi*d*L, coupling
 * through two half-compartment resistances).
 *
 * Floating point: compiled without contraction; every multiply-add that is
 * meant to be fused is written as fma()/fmaf(). exp() is computed by the
 * method of Cody and Waite (argument reduction by ln 2 split into a high part
 * with trailing zero bits and a low part) followed by a Taylor polynomial of
 * e^r, so that results do not depend on the host's libm.
 *
 * Precision modes: ORC_FP64 (everything double) and ORC_FP32_GATING (gates,
 * rates, exponentials, ionic and synaptic currents and synaptic conductances
 * in float computed from (float)V; voltage, assembly and the Hines solve in
 * double).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_FP64 0
#define ORC_FP32_GATING 1

/* ---------------------------------------------------------------------- */
/* exp: Cody-Waite reduction x = k ln2 + r, |r| <= ln2/2, then Taylor.     */
/* ---------------------------------------------------------------------- */

/* ln 2 split (fdlibm values): the high part has >= 21 trailing zero bits in
 * double and 9 in float, so k*LN2_HI is exact for every k reached here. */
static const double LN2_HI_D = 0x1.62e42feep-1;
static const double LN2_LO_D = 0x1.a39ef35793c76p-33;
static const double INV_LN2_D = 0x1.71547652b82fep+0;
static const float LN2_HI_F = 0x1.62e4p-1f;
static const float LN2_LO_F = 0x1.7f7d1cp-20f;
static const float INV_LN2_F = 0x1.715476p+0f;

/* 1/k!, k = 0..13, rounded to nearest double. */
static const double INV_FACT_D[14] = {
    0x1p+0, 0x1p+0, 0x1p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5,
    0x1.1111111111111p-7, 0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13,
    0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22,
    0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};
/* 1/k!, k = 0..7, rounded to nearest float. */
static const float INV_FACT_F[8] = {
    0x1p+0f, 0x1p+0f, 0x1p-1f, 0x1.555556p-3f, 0x1.555556p-5f,
    0x1.111112p-7f, 0x1.6c16c2p-10f, 0x1.a01a02p-13f};

double orc_exp_d(double x)
{
    if (x != x) return x;
    if (x > 709.0) x = 709.0;
    if (x < -708.0) x = -708.0;
    double k = rint(x * INV_LN2_D);
    double r = fma(-k, LN2_HI_D, x);
    r = fma(-k, LN2_LO_D, r);
    double p = INV_FACT_D[13];
    for (int i = 12; i >= 0; --i) p = fma(p, r, INV_FACT_D[i]);
    int64_t e = (int64_t)k + 1023;
    uint64_t bits = (uint64_t)e << 52;
    double s;
    memcpy(&s, &bits, sizeof s);
    return p * s;
}

float orc_exp_f(float x)
{
    if (x != x) return x;
    if (x > 88.0f) x = 88.0f;
    if (x < -87.0f) x = -87.0f;
    float k = rintf(x * INV_LN2_F);
    float r = fmaf(-k, LN2_HI_F, x);
    r = fmaf(-k, LN2_LO_F, r);
    float p = INV_FACT_F[7];
    for (int i = 6; i >= 0; --i) p = fmaf(p, r, INV_FACT_F[i]);
    int32_t e = (int32_t)k + 127;
    uint32_t bits = (uint32_t)e << 23;
    float s;
    memcpy(&s, &bits, sizeof s);
    return p * s;
}

/* exprelr(u) = u / (e^u - 1), exprelr(0) = 1. For |u| < 1/2 the Bernoulli
 * series x/(e^x-1) = sum B_n x^n / n! is used (1 - u/2 + u^2/12 - ...);
 * elsewhere the quotient itself. */
static const double BERN_D[8] = {
    /* B_2k / (2k)!, k = 1..8 */
    0x1.5555555555555p-4,  -0x1.6c16c16c16c17p-10, 0x1.1566abc011567p-15,
    -0x1.bbd779334ef0bp-21, 0x1.66a8f2bf70ebep-26, -0x1.22805d644267fp-31,
    0x1.d6db2c4e09162p-37, -0x1.7da4e1f79955cp-42};
static const float BERN_F[4] = {
    0x1.555556p-4f, -0x1.6c16c2p-10f, 0x1.1566acp-15f, -0x1.bbd77ap-21f};

double orc_exprelr_d(double u)
{
    if (fabs(u) < 0.5) {
        double w = u * u;
        double c = BERN_D[7];
        for (int i = 6; i >= 0; --i) c = fma(c, w, BERN_D[i]);
        return fma(c, w, fma(-0.5, u, 1.0));
    }
    return u / (orc_exp_d(u) - 1.0);
}

float orc_exprelr_f(float u)
{
    if (fabsf(u) < 0.5f) {
        float w = u * u;
        float c = BERN_F[3];
        for (int i = 2; i >= 0; --i) c = fmaf(c, w, BERN_F[i]);
        return fmaf(c, w, fmaf(-0.5f, u, 1.0f));
    }
    return u / (orc_exp_f(u) - 1.0f);
}

/* ---------------------------------------------------------------------- */
/* Hodgkin-Huxley rates (ms^-1), V in mV, modern sign convention.          */
/* ---------------------------------------------------------------------- */

void orc_rates_d(double v, double *out6)
{
    out6[0] = orc_exprelr_d(-(v + 40.0) / 10.0);            /* alpha_m */
    out6[1] = 4.0 * orc_exp_d(-(v + 65.0) / 18.0);          /* beta_m  */
    out6[2] = 0.07 * orc_exp_d(-(v + 65.0) / 20.0);         /* alpha_h */
    out6[3] = 1.0 / (orc_exp_d(-(v + 35.0) / 10.0) + 1.0);  /* beta_h  */
    out6[4] = 0.1 * orc_exprelr_d(-(v + 55.0) / 10.0);      /* alpha_n */
    out6[5] = 0.125 * orc_exp_d(-(v + 65.0) / 80.0);        /* beta_n  */
}

void orc_rates_f(float v, float *out6)
{
    out6[0] = orc_exprelr_f(-(v + 40.0f) / 10.0f);
    out6[1] = 4.0f * orc_exp_f(-(v + 65.0f) / 18.0f);
    out6[2] = 0.07f * orc_exp_f(-(v + 65.0f) / 20.0f);
    out6[3] = 1.0f / (orc_exp_f(-(v + 35.0f) / 10.0f) + 1.0f);
    out6[4] = 0.1f * orc_exprelr_f(-(v + 55.0f) / 10.0f);
    out6[5] = 0.125f * orc_exp_f(-(v + 65.0f) / 80.0f);
}


/* Exponential-Euler update of the three HH gates at voltage v over dt:
 * x <- x_inf + (x - x_inf) exp(-dt (alpha + beta)), x_inf = alpha/(alpha+beta). */
void orc_gates_update_d(double v, double dt, double *m, double *h, double *n)
{
    double rt[6];
    orc_rates_d(v, rt);
    double *x[3] = {m, h, n};
    for (int g = 0; g < 3; ++g) {
        double s = rt[2 * g] + rt[2 * g + 1];
        double xinf = rt[2 * g] / s;
        double ex = orc_exp_d(-dt * s);
        *x[g] = xinf + (*x[g] - xinf) * ex;
    }
}

void orc_gates_update_f(float v, float dt, float *m, float *h, float *n)
{
    float rt[6];
    orc_rates_f(v, rt);
    float *x[3] = {m, h, n};
    for (int g = 0; g < 3; ++g) {
        float s = rt[2 * g] + rt[2 * g + 1];
        float xinf = rt[2 * g] / s;
        float ex = orc_exp_f(-dt * s);
        *x[g] = xinf + (*x[g] - xinf) * ex;
    }
}

/* ---------------------------------------------------------------------- */
/* Linear solve on a tree-structured matrix (the system of Eq. 2).         */
/* ---------------------------------------------------------------------- */

/* Solves A x = rhs where the only off-diagonal entries of A link each
 * compartment k >= 1 with its parent up = parent[k] < k:
 *   to_parent[k]   = A[up][k]  (the entry in the parent's row),
 *   from_parent[k] = A[k][up]  (the entry in row k).
 * Since every parent index is smaller than its child's, Gaussian elimination
 * of the rows in descending index order only modifies rows not yet
 * eliminated and creates no fill: eliminating row k subtracts
 * (A[up][k] / A[k][k]) times row k from row up, which changes A[up][up] and
 * rhs[up] only. Substitution then runs from the root outwards. This is the
 * method of Algorithm 1; several children of one parent reach the parent's
 * row in descending index order. diag and rhs are overwritten (the eliminated
 * diagonal, the reduced right-hand side); x receives the solution and may be
 * the same array as rhs. */
void orc_tree_solve(int32_t n, const int32_t *parent, const double *to_parent,
                    double *diag, const double *from_parent, double *rhs,
                    double *x)
{
    int32_t k = n;
    while (--k >= 1) {
        const int32_t up = parent[k];
        const double mult = to_parent[k] / diag[k];
        diag[up] = diag[up] - mult * from_parent[k];
        rhs[up] = rhs[up] - mult * rhs[k];
    }
    if (n < 1) return;
    x[0] = rhs[0] / diag[0];
    for (k = 1; k < n; ++k) {
        const double known = from_parent[k] * x[parent[k]];
        x[k] = (rhs[k] - known) / diag[k];
    }
}

/* ---------------------------------------------------------------------- */
/* Network simulator.                                                      */
/* ---------------------------------------------------------------------- */

typedef struct {
    double dt, theta, tau_syn, e_syn, v_thresh, v_init;
    double cm, ra, gnabar, gkbar, gl, ena, ek, el, g_pas, e_pas;
    int32_t precision;
} orc_params_t;

typedef struct {
    orc_params_t P;
    int32_t N;
    int64_t C, S;
    int64_t *off;        /* [N+1] compartment offsets */
    int32_t *parent;     /* [C] neuron-local */
    uint8_t *mech;       /* [C] */
    int32_t *detector;   /* [N] */
    double *iext;        /* [N] */
    /* per-compartment constants, computed once */
    double *cdt;         /* C_i / dt  (nF/ms = uS) */
    double *G;           /* coupling to parent (uS), G[root] = 0 */
    double *e;           /* off-diagonal A[i,p(i)] = A[p(i),i] = -theta*G[i] */
    double *af;          /* area factor: S/cm^2 -> uS */
    /* state */
    double *V;
    double *gm, *gh, *gn;     /* gates, double mode */
    float *fm, *fh, *fn;      /* gates, float mode */
    double *g_d;  float *g_f; /* synaptic conductance per synapse */
    /* synapses */
    int32_t *pre, *post, *pcomp, *delay;
    double *w;
    int64_t *syn_off;   /* [N+1] CSR of synapses by post neuron */
    int64_t *syn_idx;   /* [S] synapse ids, ascending within each post */
    double q;           /* exp(-dt/tau) */
    /* spikes */
    int64_t step;
    int64_t hist_cap;   /* steps stored in the bit history */
    uint8_t *hist;      /* [(hist_cap+1) * N] : spiked at step s (1-based) */
    uint8_t *spk_now;   /* [N] */
    int64_t nspk, spk_cap;
    int64_t *spk;       /* (neuron, step) pairs */
    /* replay: when set, presynaptic spikes come from this raster of another
     * run ([(ext_steps+1) * ext_N], 1 = neuron spiked at that step) instead
     * of this simulation's own history; pre ids then index that network */
    uint8_t *ext;
    int32_t ext_N;
    int64_t ext_steps;
    /* scratch, one set per thread */
    int nthreads;
    int32_t maxn;
    double *w_d, *w_r, *w_ax, *w_gs, *w_gm;
} orc_sim_t;

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s ? s : 1); }

void orc_destroy(orc_sim_t *o);

static double gate_inf_d(double a, double b) { return a / (a + b); }

orc_sim_t *orc_create(const orc_params_t *P, int32_t N, const int64_t *off,
                      const int32_t *parent, const double *length,
                      const double *diam, const uint8_t *mech,
                      const int32_t *detector, const double *iext, int64_t S,
                      const int32_t *pre, const int32_t *post,
                      const int32_t *pcomp, const int32_t *delay,
                      const double *w, int64_t max_steps)
{
    orc_sim_t *o = (orc_sim_t *)xcalloc(1, sizeof *o);
    o->P = *P;
    o->N = N;
    o->C = off[N];
    o->S = S;
    int64_t C = o->C;
    o->off = (int64_t *)xcalloc(N + 1, sizeof(int64_t));
    memcpy(o->off, off, (N + 1) * sizeof(int64_t));
    o->parent = (int32_t *)xcalloc(C, sizeof(int32_t));
    memcpy(o->parent, parent, C * sizeof(int32_t));
    o->mech = (uint8_t *)xcalloc(C, 1);
    memcpy(o->mech, mech, C);
    o->detector = (int32_t *)xcalloc(N, sizeof(int32_t));
    memcpy(o->detector, detector, N * sizeof(int32_t));
    o->iext = (double *)xcalloc(N, sizeof(double));
    memcpy(o->iext, iext, N * sizeof(double));

    /* geometry -> constants (finite volumes). Units: um, ms, mV, nA, nF, uS,
     * MOhm. area_um2 = pi*d*L. Capacitance C = cm[uF/cm2]*area*1e-8[cm2/um2]
     * *1e3[nF/uF] = cm*area*1e-5 nF. Half-compartment axial resistance
     * R/2 = 2*Ra[Ohm cm]*L/(pi d^2) with L/d^2 in 1/um = 1e4/cm, times
     * 1e-6 MOhm/Ohm: 2*Ra*L/(pi*d*d)*1e-2 MOhm. Area factor for a density in
     * S/cm2 to a conductance in uS: area*1e-8*1e6 = area*1e-2. */
    const double PI = 3.14159265358979323846;
    o->cdt = (double *)xcalloc(C, sizeof(double));
    o->G = (double *)xcalloc(C, sizeof(double));
    o->e = (double *)xcalloc(C, sizeof(double));
    o->af = (double *)xcalloc(C, sizeof(double));
    double *rhalf = (double *)xcalloc(C, sizeof(double));
    for (int64_t c = 0; c < C; ++c) {
        double area = PI * diam[c] * length[c];
        o->cdt[c] = P->cm * area * 1e-5 / P->dt;
        o->af[c] = area * 1e-2;
        rhalf[c] = 2.0 * P->ra * length[c] / (PI * diam[c] * diam[c]) * 1e-2;
    }
    o->maxn = 1;
    for (int32_t j = 0; j < N; ++j) {
        int64_t b = off[j];
        int32_t n = (int32_t)(off[j + 1] - off[j]);
        if (n > o->maxn) o->maxn = n;
        o->G[b] = 0.0;
        o->e[b] = 0.0;
        for (int32_t i = 1; i < n; ++i) {
            o->G[b + i] = 1.0 / (rhalf[b + i] + rhalf[b + parent[b + i]]);
            o->e[b + i] = -P->theta * o->G[b + i];
        }
    }
    free(rhalf);

    /* state: V = v_init, gates at steady state for v_init, g = 0 */
    o->V = (double *)xcalloc(C, sizeof(double));
    for (int64_t c = 0; c < C; ++c) o->V[c] = P->v_init;
    if (P->precision == ORC_FP64) {
        double r[6];
        orc_rates_d(P->v_init, r);
        o->gm = (double *)xcalloc(C, sizeof(double));
        o->gh = (double *)xcalloc(C, sizeof(double));
        o->gn = (double *)xcalloc(C, sizeof(double));
        for (int64_t c = 0; c < C; ++c) {
            o->gm[c] = gate_inf_d(r[0], r[1]);
            o->gh[c] = gate_inf_d(r[2], r[3]);
            o->gn[c] = gate_inf_d(r[4], r[5]);
        }
        o->g_d = (double *)xcalloc(S, sizeof(double));
    } else {
        float r[6];
        orc_rates_f((float)P->v_init, r);
        o->fm = (float *)xcalloc(C, sizeof(float));
        o->fh = (float *)xcalloc(C, sizeof(float));
        o->fn = (float *)xcalloc(C, sizeof(float));
        for (int64_t c = 0; c < C; ++c) {
            o->fm[c] = r[0] / (r[0] + r[1]);
            o->fh[c] = r[2] / (r[2] + r[3]);
            o->fn[c] = r[4] / (r[4] + r[5]);
        }
        o->g_f = (float *)xcalloc(S, sizeof(float));
    }

    /* synapses, and for each post neuron its synapses in ascending id */
    o->pre = (int32_t *)xcalloc(S, sizeof(int32_t));
    o->post = (int32_t *)xcalloc(S, sizeof(int32_t));
    o->pcomp = (int32_t *)xcalloc(S, sizeof(int32_t));
    o->delay = (int32_t *)xcalloc(S, sizeof(int32_t));
    o->w = (double *)xcalloc(S, sizeof(double));
    memcpy(o->pre, pre, S * sizeof(int32_t));
    memcpy(o->post, post, S * sizeof(int32_t));
    memcpy(o->pcomp, pcomp, S * sizeof(int32_t));
    memcpy(o->delay, delay, S * sizeof(int32_t));
    memcpy(o->w, w, S * sizeof(double));
    o->syn_off = (int64_t *)xcalloc(N + 1, sizeof(int64_t));
    o->syn_idx = (int64_t *)xcalloc(S, sizeof(int64_t));
    for (int64_t k = 0; k < S; ++k) o->syn_off[post[k] + 1]++;
    for (int32_t j = 0; j < N; ++j) o->syn_off[j + 1] += o->syn_off[j];
    {
        int64_t *fill = (int64_t *)xcalloc(N, sizeof(int64_t));
        for (int64_t k = 0; k < S; ++k) {
            int32_t j = post[k];
            o->syn_idx[o->syn_off[j] + fill[j]++] = k;
        }
        free(fill);
    }
    o->q = orc_exp_d(-P->dt / P->tau_syn);

    o->step = 0;
    o->hist_cap = max_steps;
    o->hist = (uint8_t *)xcalloc((size_t)(max_steps + 1) * N, 1);
    o->spk_now = (uint8_t *)xcalloc(N, 1);
    o->spk_cap = 1024;
    o->spk = (int64_t *)xcalloc(2 * o->spk_cap, sizeof(int64_t));

    o->nthreads = 1;
#ifdef _OPENMP
    o->nthreads = omp_get_max_threads();
#endif
    size_t ws = (size_t)o->nthreads * o->maxn;
    o->w_d = (double *)xcalloc(ws, sizeof(double));
    o->w_r = (double *)xcalloc(ws, sizeof(double));
    o->w_ax = (double *)xcalloc(ws, sizeof(double));
    o->w_gs = (double *)xcalloc(ws, sizeof(double));
    o->w_gm = (double *)xcalloc(ws, sizeof(double));
    if (!o->V || !o->hist || !o->w_d) { orc_destroy(o); return NULL; }
    return o;
}

void orc_destroy(orc_sim_t *o)
{
    if (!o) return;
    void *ptrs[] = {o->off, o->parent, o->mech, o->detector, o->iext, o->cdt,
                    o->G, o->e, o->af, o->V, o->gm, o->gh, o->gn, o->fm,
                    o->fh, o->fn, o->g_d, o->g_f, o->pre, o->post, o->pcomp,
                    o->delay, o->w, o->syn_off, o->syn_idx, o->hist,
                    o->spk_now, o->spk, o->w_d, o->w_r, o->w_ax, o->w_gs, o->w_gm,
                    o->ext};
    for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i) free(ptrs[i]);
    free(o);
}

static int spiked_at(const orc_sim_t *o, int32_t j, int64_t s)
{
    if (o->ext) {
        if (s < 1 || s > o->ext_steps) return 0;
        return o->ext[(size_t)s * o->ext_N + j];
    }
    if (s < 1 || s > o->hist_cap) return 0;
    return o->hist[(size_t)s * o->N + j];
}

/* Replay mode: deliver presynaptic spikes from a raster recorded elsewhere
 * (raster[s * ext_N + j] != 0: neuron j of that network spiked at step s,
 * s = 1 .. ext_steps). Every synapse's pre id must be < ext_N. The raster is
 * copied. Returns 0, or -1 on a bad argument or allocation failure. */
int orc_set_input_raster(orc_sim_t *o, int32_t ext_N, int64_t ext_steps, const uint8_t *raster)
{
    if (!o || ext_N < 1 || ext_steps < 0 || !raster) return -1;
    for (int64_t k = 0; k < o->S; ++k)
        if (o->pre[k] < 0 || o->pre[k] >= ext_N) return -1;
    size_t bytes = (size_t)(ext_steps + 1) * (size_t)ext_N;
    uint8_t *copy = (uint8_t *)malloc(bytes ? bytes : 1);
    if (!copy) return -1;
    memcpy(copy, raster, bytes);
    free(o->ext);
    o->ext = copy;
    o->ext_N = ext_N;
    o->ext_steps = ext_steps;
    return 0;
}

/* One step n -> n+1 of neuron j, double precision gating. */
static void neuron_step_d(orc_sim_t *o, int32_t j, int tid)
{
    const orc_params_t *P = &o->P;
    const int64_t b = o->off[j];
    const int32_t n = (int32_t)(o->off[j + 1] - b);
    const int32_t *p = o->parent + b;
    double *V = o->V + b;
    double *d = o->w_d + (size_t)tid * o->maxn;
    double *r = o->w_r + (size_t)tid * o->maxn;
    double *ax = o->w_ax + (size_t)tid * o->maxn;
    double *gs = o->w_gs + (size_t)tid * o->maxn;
    double *gmem = o->w_gm + (size_t)tid * o->maxn;
    const int64_t n_now = o->step;

    /* 1. deliver: g_k += w_k for each synapse whose presynaptic neuron
     *    spiked d_k steps ago; 2. per-compartment synaptic conductance,
     *    summed over the compartment's synapses in ascending synapse id. */
    for (int32_t i = 0; i < n; ++i) gs[i] = 0.0;
    for (int64_t t = o->syn_off[j]; t < o->syn_off[j + 1]; ++t) {
        int64_t k = o->syn_idx[t];
        if (spiked_at(o, o->pre[k], n_now - o->delay[k])) o->g_d[k] += o->w[k];
        gs[o->pcomp[k]] += o->g_d[k];
    }

    /* 3. membrane current, linear in V for the gates of step n:
     *    I(V) = g V - J with g the total membrane conductance (uS) and J the
     *    conductance-weighted reversal potentials plus the injected current
     *    (nA); evaluated implicitly at V^{n+1}. */
    for (int32_t i = 0; i < n; ++i) {
        double gion, jion;
        if (o->mech[b + i]) {
            double m = o->gm[b + i], h = o->gh[b + i], nn = o->gn[b + i];
            double gna = P->gnabar * (((m * m) * m) * h);
            double gk = P->gkbar * (((nn * nn) * nn) * nn);
            gion = (gna + gk) + P->gl;
            jion = (gna * P->ena + gk * P->ek) + P->gl * P->el;
        } else {
            gion = P->g_pas;
            jion = P->g_pas * P->e_pas;
        }
        double iext = (i == 0) ? o->iext[j] : 0.0;
        gmem[i] = o->af[b + i] * gion + gs[i];
        r[i] = (o->af[b + i] * jion + gs[i] * P->e_syn) + iext;   /* r holds J */
    }

    /* 4. assembly: d_i = C_i/dt + theta*(couplings) + g_i,
     *    rhs_i = C_i V_i/dt + J_i + (1-theta) * (axial current into i). */
    for (int32_t i = 0; i < n; ++i) { ax[i] = 0.0; d[i] = o->cdt[b + i]; }
    for (int32_t i = 1; i < n; ++i) {
        double flux = o->G[b + i] * (V[p[i]] - V[i]);
        ax[i] += flux;
        ax[p[i]] -= flux;
        d[i] -= o->e[b + i];
        d[p[i]] -= o->e[b + i];
    }
    const double omt = 1.0 - P->theta;
    for (int32_t i = 0; i < n; ++i) {
        d[i] += gmem[i];
        r[i] = (o->cdt[b + i] * V[i] + r[i]) + omt * ax[i];
    }

    /* 5. tree solve (Algorithm 1); the matrix is symmetric, both
     *    off-diagonals of a parent link are e */
    orc_tree_solve(n, p, o->e + b, d, o->e + b, r, r);

    /* 6. gates at V^{n+1} (exponential Euler); then commit V */
    const double dt = P->dt;
    const int32_t det = o->detector[j];
    const double vold = V[det];
    for (int32_t i = 0; i < n; ++i) {
        V[i] = r[i];
        if (!o->mech[b + i]) continue;
        orc_gates_update_d(V[i], dt, &o->gm[b + i], &o->gh[b + i], &o->gn[b + i]);
    }
    /* 7. synaptic decay */
    for (int64_t t = o->syn_off[j]; t < o->syn_off[j + 1]; ++t) {
        int64_t k = o->syn_idx[t];
        o->g_d[k] = o->q * o->g_d[k];
    }
    /* 8. detection: upward crossing of the threshold */
    o->spk_now[j] = (vold < P->v_thresh && V[det] >= P->v_thresh) ? 1 : 0;
}

/* Same step, float gating (rates, gates, currents and synaptic conductances
 * in float from (float)V; assembly and solve in double). */
static void neuron_step_f(orc_sim_t *o, int32_t j, int tid)
{
    const orc_params_t *P = &o->P;
    const int64_t b = o->off[j];
    const int32_t n = (int32_t)(o->off[j + 1] - b);
    const int32_t *p = o->parent + b;
    double *V = o->V + b;
    double *d = o->w_d + (size_t)tid * o->maxn;
    double *r = o->w_r + (size_t)tid * o->maxn;
    double *ax = o->w_ax + (size_t)tid * o->maxn;
    float *gs = (float *)(o->w_gs + (size_t)tid * o->maxn);
    double *gmem = o->w_gm + (size_t)tid * o->maxn;
    const int64_t n_now = o->step;
    const float wq = (float)o->q;

    for (int32_t i = 0; i < n; ++i) gs[i] = 0.0f;
    for (int64_t t = o->syn_off[j]; t < o->syn_off[j + 1]; ++t) {
        int64_t k = o->syn_idx[t];
        if (spiked_at(o, o->pre[k], n_now - o->delay[k]))
            o->g_f[k] += (float)o->w[k];
        gs[o->pcomp[k]] += o->g_f[k];
    }

    const float gnabar = (float)P->gnabar, gkbar = (float)P->gkbar;
    const float gl = (float)P->gl, g_pas = (float)P->g_pas;
    const float ena = (float)P->ena, ek = (float)P->ek, el = (float)P->el;
    const float e_pas = (float)P->e_pas, e_syn = (float)P->e_syn;
    for (int32_t i = 0; i < n; ++i) {
        float gion, jion;
        float af = (float)o->af[b + i];
        if (o->mech[b + i]) {
            float m = o->fm[b + i], h = o->fh[b + i], nn = o->fn[b + i];
            float gna = gnabar * (((m * m) * m) * h);
            float gk = gkbar * (((nn * nn) * nn) * nn);
            gion = (gna + gk) + gl;
            jion = (gna * ena + gk * ek) + gl * el;
        } else {
            gion = g_pas;
            jion = g_pas * e_pas;
        }
        float iext = (i == 0) ? (float)o->iext[j] : 0.0f;
        gmem[i] = (double)(af * gion + gs[i]);
        r[i] = (double)((af * jion + gs[i] * e_syn) + iext);
    }

    for (int32_t i = 0; i < n; ++i) { ax[i] = 0.0; d[i] = o->cdt[b + i]; }
    for (int32_t i = 1; i < n; ++i) {
        double flux = o->G[b + i] * (V[p[i]] - V[i]);
        ax[i] += flux;
        ax[p[i]] -= flux;
        d[i] -= o->e[b + i];
        d[p[i]] -= o->e[b + i];
    }
    const double omt = 1.0 - P->theta;
    for (int32_t i = 0; i < n; ++i) {
        d[i] += gmem[i];
        r[i] = (o->cdt[b + i] * V[i] + r[i]) + omt * ax[i];
    }

    orc_tree_solve(n, p, o->e + b, d, o->e + b, r, r);

    const float dt = (float)P->dt;
    const int32_t det = o->detector[j];
    const double vold = V[det];
    for (int32_t i = 0; i < n; ++i) {
        V[i] = r[i];
        if (!o->mech[b + i]) continue;
        orc_gates_update_f((float)V[i], dt, &o->fm[b + i], &o->fh[b + i], &o->fn[b + i]);
    }
    for (int64_t t = o->syn_off[j]; t < o->syn_off[j + 1]; ++t) {
        int64_t k = o->syn_idx[t];
        o->g_f[k] = wq * o->g_f[k];
    }
    o->spk_now[j] = (vold < P->v_thresh && V[det] >= P->v_thresh) ? 1 : 0;
}

/* Advance the whole network by nsteps. Neurons are independent within a
 * step (delivery only reads spikes of earlier steps), so the neuron loop may
 * run in parallel; the result does not depend on the thread count. */
int orc_step(orc_sim_t *o, int64_t nsteps)
{
    for (int64_t s = 0; s < nsteps; ++s) {
        if (o->step + 1 > o->hist_cap) return -1;
        if (o->P.precision == ORC_FP64) {
#pragma omp parallel for schedule(dynamic, 8) num_threads(o->nthreads)
            for (int32_t j = 0; j < o->N; ++j) {
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
                neuron_step_d(o, j, tid);
            }
        } else {
#pragma omp parallel for schedule(dynamic, 8) num_threads(o->nthreads)
            for (int32_t j = 0; j < o->N; ++j) {
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
                neuron_step_f(o, j, tid);
            }
        }
        o->step += 1;
        uint8_t *row = o->hist + (size_t)o->step * o->N;
        for (int32_t j = 0; j < o->N; ++j) {
            row[j] = o->spk_now[j];
            if (!o->spk_now[j]) continue;
            if (o->nspk == o->spk_cap) {
                int64_t *nb = (int64_t *)realloc(o->spk, 4 * o->spk_cap * sizeof(int64_t));
                if (!nb) return -2;
                o->spk = nb;
                o->spk_cap *= 2;
            }
            o->spk[2 * o->nspk] = j;
            o->spk[2 * o->nspk + 1] = o->step;
            o->nspk++;
        }
    }
    return 0;
}

/* ---- accessors ---- */
int64_t orc_n_comp(const orc_sim_t *o) { return o->C; }
int64_t orc_cur_step(const orc_sim_t *o) { return o->step; }
void orc_get_v(const orc_sim_t *o, double *out) { memcpy(out, o->V, o->C * sizeof(double)); }
void orc_set_v(orc_sim_t *o, const double *in) { memcpy(o->V, in, o->C * sizeof(double)); }
void orc_get_gates(const orc_sim_t *o, double *m, double *h, double *n)
{
    for (int64_t c = 0; c < o->C; ++c) {
        if (o->P.precision == ORC_FP64) { m[c] = o->gm[c]; h[c] = o->gh[c]; n[c] = o->gn[c]; }
        else { m[c] = o->fm[c]; h[c] = o->fh[c]; n[c] = o->fn[c]; }
    }
}
void orc_get_g(const orc_sim_t *o, double *out)
{
    for (int64_t k = 0; k < o->S; ++k)
        out[k] = (o->P.precision == ORC_FP64) ? o->g_d[k] : (double)o->g_f[k];
}
int64_t orc_n_spikes(const orc_sim_t *o) { return o->nspk; }
void orc_get_spikes(const orc_sim_t *o, int64_t *out) { memcpy(out, o->spk, 2 * o->nspk * sizeof(int64_t)); }
/* Constants as the oracle computed them: C/dt, G, e, area factor, and the
 * assembled diagonal (before elimination) of neuron j. */
void orc_get_consts(const orc_sim_t *o, double *cdt, double *G, double *e, double *af)
{
    memcpy(cdt, o->cdt, o->C * sizeof(double));
    memcpy(G, o->G, o->C * sizeof(double));
    memcpy(e, o->e, o->C * sizeof(double));
    memcpy(af, o->af, o->C * sizeof(double));
}
void orc_assemble_diag(const orc_sim_t *o, int32_t j, double *d)
{
    const int64_t b = o->off[j];
    const int32_t n = (int32_t)(o->off[j + 1] - b);
    for (int32_t i = 0; i < n; ++i) d[i] = o->cdt[b + i];
    for (int32_t i = 1; i < n; ++i) {
        d[i] -= o->e[b + i];
        d[o->parent[b + i]] -= o->e[b + i];
    }
}
double orc_q(const orc_sim_t *o) { return o->q; }
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
/* Threads of simulations created from now on (each keeps the count it was
 * created with, which sizes its per-thread work space). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
