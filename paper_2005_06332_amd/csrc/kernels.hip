// Epoch kernel and setup kernel of the multi-morphology simulator (gfx950).
//
// One workgroup advances one pack of neurons through the steps of an epoch
// (E <= the smallest synaptic delay, so no spike produced inside the epoch
// can reach a neuron before the epoch ends; Section 2 of the paper, two-level
// time stepping). While it does so the pack's voltages, off-diagonal,
// synaptic conductances and the per-step matrix (diagonal D and right-hand
// side R) stay in LDS (or, for packs too large for LDS, in a private slice
// of global scratch). With FP32 gating and the contraction solver the gates
// and time-invariant constants of each thread's first kResident compartments
// stay in registers for the epoch; the others' are read from global memory
// (mostly L2) every step.
//
// Per step and pack, in the order of the paper's update (Section 2):
//   A  synaptic delivery from the spike history, per-compartment conductance
//   B  membrane conductance g and source J per compartment (HH gates of step
//      n), assembly of Eq. 2: D_i = C_i/dt + theta*sum G + g_i,
//      R_i = C_i V_i/dt + J_i + (1-theta) * axial current
//   C  backward sweep of Algorithm 1, one lane per branch, branches grouped
//      by height so that every child is finished before its parent (or the
//      eliminations of a tree contraction, round by round)
//   D  forward sweep of Algorithm 1, branches grouped by depth (or the
//      contraction's back substitution, rounds in reverse)
//   E  gates at V^{n+1} (exponential Euler); threshold-crossing detection
// The exact solver performs every floating-point operation in the order of
// Algorithm 1 as written (children of a node eliminated in descending index
// order), with no contraction; the fast solver reassociates the elimination
// into a division-free homogeneous form, and the contraction solver performs
// the same Gaussian elimination in another order. In all three, a neuron's
// arithmetic does not depend on how neurons are packed or launched.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace mmh {

// Scratch for the entry point that allocates nothing (sim_step_noalloc): the
// state slices of packs too large for LDS live here instead of in memory the
// simulation allocated. Every device holds its own copy for the life of the
// process; its address is resolved once per device, at set-up, and only
// that address is handed to kernels (the array's name is a host-side stand-in).
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void **ptr) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

#ifdef MMH_PHASE_PROFILE
// Optional per-phase wall-clock accounting (workgroup time in each phase of
// the step loop), compiled only into profiling builds: thread 0 sums each
// phase's time in registers and adds the sums once per pack.
__device__ unsigned long long g_phase_ticks[8];
#define MMH_PHASE(k)                                                             \
    do {                                                                         \
        if (threadIdx.x == 0) {                                                  \
            const uint64_t now_ = wall_clock64();                                \
            ph_acc_[k] += now_ - ph_t_;                                          \
            ph_t_ = now_;                                                        \
        }                                                                        \
    } while (0)
#else
#define MMH_PHASE(k) \
    do {             \
    } while (0)
#endif

namespace {

// ---------------------------------------------------------------------------
// Elementary functions. exp: Cody & Waite argument reduction x = k ln2 + r
// with ln2 split into a high part with trailing zero bits (k*hi exact) and a
// low part, then the Taylor polynomial of e^r (degree 13 in double, 7 in
// float) by Horner with fused multiply-adds, then the scaling by 2^k
// (ldexp; exact, since the clamp keeps the result a normal number).
// ---------------------------------------------------------------------------
constexpr double kLn2HiD = 0x1.62e42feep-1;
constexpr double kLn2LoD = 0x1.a39ef35793c76p-33;
constexpr double kInvLn2D = 0x1.71547652b82fep+0;
constexpr float kLn2HiF = 0x1.62e4p-1f;
constexpr float kLn2LoF = 0x1.7f7d1cp-20f;
constexpr float kInvLn2F = 0x1.715476p+0f;

// The argument is clamped to [-708, 709] ([-87, 88] in float), where the
// result is a normal number; for every finite argument this is the same
// function as clamping with comparisons (only a NaN argument differs, which a
// valid state never produces).
__device__ __forceinline__ double dexp(double x) {
    x = __builtin_fmin(__builtin_fmax(x, -708.0), 709.0);
    const double k = __builtin_rint(x * kInvLn2D);
    double r = __builtin_fma(-k, kLn2HiD, x);
    r = __builtin_fma(-k, kLn2LoD, r);
    double p = 0x1.6124613a86d09p-33;            // 1/13!
    p = __builtin_fma(p, r, 0x1.1eed8eff8d898p-29);  // 1/12!
    p = __builtin_fma(p, r, 0x1.ae64567f544e4p-26);  // 1/11!
    p = __builtin_fma(p, r, 0x1.27e4fb7789f5cp-22);  // 1/10!
    p = __builtin_fma(p, r, 0x1.71de3a556c734p-19);  // 1/9!
    p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-16);  // 1/8!
    p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-13);  // 1/7!
    p = __builtin_fma(p, r, 0x1.6c16c16c16c17p-10);  // 1/6!
    p = __builtin_fma(p, r, 0x1.1111111111111p-7);   // 1/5!
    p = __builtin_fma(p, r, 0x1.5555555555555p-5);   // 1/4!
    p = __builtin_fma(p, r, 0x1.5555555555555p-3);   // 1/3!
    p = __builtin_fma(p, r, 0x1p-1);                 // 1/2!
    p = __builtin_fma(p, r, 1.0);                    // 1/1!
    p = __builtin_fma(p, r, 1.0);                    // 1/0!
    return __builtin_amdgcn_ldexp(p, (int)k);
}

__device__ __forceinline__ float fexp(float x) {
    x = __builtin_amdgcn_fmed3f(x, -87.0f, 88.0f);
    const float k = __builtin_rintf(x * kInvLn2F);
    float r = __builtin_fmaf(-k, kLn2HiF, x);
    r = __builtin_fmaf(-k, kLn2LoF, r);
    float p = 0x1.a01a02p-13f;                  // 1/7!
    p = __builtin_fmaf(p, r, 0x1.6c16c2p-10f);  // 1/6!
    p = __builtin_fmaf(p, r, 0x1.111112p-7f);   // 1/5!
    p = __builtin_fmaf(p, r, 0x1.555556p-5f);   // 1/4!
    p = __builtin_fmaf(p, r, 0x1.555556p-3f);   // 1/3!
    p = __builtin_fmaf(p, r, 0x1p-1f);          // 1/2!
    p = __builtin_fmaf(p, r, 1.0f);             // 1/1!
    p = __builtin_fmaf(p, r, 1.0f);             // 1/0!
    return __builtin_amdgcn_ldexpf(p, (int)k);
}

// Correctly rounded a / b for operands and quotients far from the overflow
// and underflow limits (the rate arguments and gate coefficients of the HH
// model, and the reciprocal pivots): hardware reciprocal, Newton steps, and
// Markstein's residual corrections. This is the sequence the compiler emits
// for IEEE division with its range-scaling and special-case steps left out,
// which are identities on such operands, so the quotient is bit for bit the
// IEEE one.
__device__ __forceinline__ float div_core(float a, float b) {
    float y = __builtin_amdgcn_rcpf(b);
    const float e = __builtin_fmaf(-b, y, 1.0f);
    y = __builtin_fmaf(e, y, y);
    float q = a * y;
    float r = __builtin_fmaf(-b, q, a);
    q = __builtin_fmaf(r, y, q);
    r = __builtin_fmaf(-b, q, a);
    return __builtin_fmaf(r, y, q);
}
__device__ __forceinline__ double div_core(double a, double b) {
    double y = __builtin_amdgcn_rcp(b);
    double e = __builtin_fma(-b, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-b, y, 1.0);
    y = __builtin_fma(y, e, y);
    const double q = a * y;
    const double r = __builtin_fma(-b, q, a);
    return __builtin_fma(r, y, q);
}

// u / (e^u - 1): Bernoulli series B_2k/(2k)! u^2k near 0, the quotient elsewhere.
__device__ __forceinline__ double dexprelr(double u) {
    if (__builtin_fabs(u) < 0.5) {
        const double w = u * u;
        double c = -0x1.7da4e1f79955cp-42;
        c = __builtin_fma(c, w, 0x1.d6db2c4e09162p-37);
        c = __builtin_fma(c, w, -0x1.22805d644267fp-31);
        c = __builtin_fma(c, w, 0x1.66a8f2bf70ebep-26);
        c = __builtin_fma(c, w, -0x1.bbd779334ef0bp-21);
        c = __builtin_fma(c, w, 0x1.1566abc011567p-15);
        c = __builtin_fma(c, w, -0x1.6c16c16c16c17p-10);
        c = __builtin_fma(c, w, 0x1.5555555555555p-4);
        return __builtin_fma(c, w, __builtin_fma(-0.5, u, 1.0));
    }
    return div_core(u, dexp(u) - 1.0);
}

__device__ __forceinline__ float fexprelr(float u) {
    if (__builtin_fabsf(u) < 0.5f) {
        const float w = u * u;
        float c = -0x1.bbd77ap-21f;
        c = __builtin_fmaf(c, w, 0x1.1566acp-15f);
        c = __builtin_fmaf(c, w, -0x1.6c16c2p-10f);
        c = __builtin_fmaf(c, w, 0x1.555556p-4f);
        return __builtin_fmaf(c, w, __builtin_fmaf(-0.5f, u, 1.0f));
    }
    return div_core(u, fexp(u) - 1.0f);
}

// x / c for the rate constants c. Float: q = RN(x RN(1/c)), then Markstein's
// correction with the exact residual x - q c. For c = 10, 18, 20 and 80 this
// equals the correctly rounded quotient for every float with
// 1e-30 <= |x| <= 1e30 (checked exhaustively), and for x = +0; x = -0 gives
// +0 where the quotient is -0, which changes nothing, since the quotient only
// enters exp and exprelr, and both give 1 at either zero. The rate arguments
// v + const are 0 or at least ulp(40) in magnitude. Double: the IEEE
// quotient.
__device__ __forceinline__ float div_const(float x, float c, float rc) {
    const float q = x * rc;
    const float r = __builtin_fmaf(-q, c, x);
    return __builtin_fmaf(r, rc, q);
}
__device__ __forceinline__ double div_const(double x, double c, double) { return x / c; }

template <typename T> struct Fn;
template <> struct Fn<double> {
    static __device__ __forceinline__ double ex(double x) { return dexp(x); }
    static __device__ __forceinline__ double exr(double x) { return dexprelr(x); }
};
template <> struct Fn<float> {
    static __device__ __forceinline__ float ex(float x) { return fexp(x); }
    static __device__ __forceinline__ float exr(float x) { return fexprelr(x); }
};

// Hodgkin-Huxley rates (1/ms) at v (mV), modern sign convention.
template <typename T>
__device__ __forceinline__ void hh_rates(T v, T &am, T &bm, T &ah, T &bh, T &an, T &bn) {
    am = Fn<T>::exr(div_const(-(v + T(40)), T(10), T(1) / T(10)));
    bm = T(4) * Fn<T>::ex(div_const(-(v + T(65)), T(18), T(1) / T(18)));
    ah = T(0.07) * Fn<T>::ex(div_const(-(v + T(65)), T(20), T(1) / T(20)));
    bh = div_core(T(1), Fn<T>::ex(div_const(-(v + T(35)), T(10), T(1) / T(10))) + T(1));
    an = T(0.1) * Fn<T>::exr(div_const(-(v + T(55)), T(10), T(1) / T(10)));
    bn = T(0.125) * Fn<T>::ex(div_const(-(v + T(65)), T(80), T(1) / T(80)));
}

// Exponential Euler: x <- x_inf + (x - x_inf) exp(-dt (a + b)).
template <typename T>
__device__ __forceinline__ T gate_step(T x, T a, T b, T dt) {
    const T s = a + b;
    const T xinf = div_core(a, s);
    const T ex = Fn<T>::ex(-dt * s);
    return xinf + (x - xinf) * ex;
}

// ---------------------------------------------------------------------------
// Setup: time-invariant coefficients of every neuron (capacitance over dt,
// area factor, off-diagonal -theta G with G the coupling through the two
// half-compartment resistances) and the initial state. One thread per neuron.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_setup(SetupArgs a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) *a.q_out = dexp(-a.dt / a.tau);
    if (j >= a.n_neurons) return;
    const double PI = 3.14159265358979323846;
    const int64_t c0 = a.ncomp0[j];
    const int32_t n = (int32_t)(a.ncomp0[j + 1] - c0);
    T am, bm, ah, bh, an, bn;
    hh_rates<T>(T(a.v_init), am, bm, ah, bh, an, bn);
    const T m0 = am / (am + bm), h0 = ah / (ah + bh), n0 = an / (an + bn);
    T *af = (T *)a.af, *gm = (T *)a.gm, *gh = (T *)a.gh, *gn = (T *)a.gn;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t c = c0 + i;
        const double area = PI * a.diam[c] * a.length[c];
        a.cdt[c] = a.cm * area * 1e-5 / a.dt;
        af[c] = (T)(area * 1e-2);
        a.V[c] = a.v_init;
        gm[c] = m0;
        gh[c] = h0;
        gn[c] = n0;
    }
    a.e[c0] = 0.0;
    for (int32_t i = 1; i < n; ++i) {
        const int64_t c = c0 + i;
        const int64_t pc = c0 + a.lparent[c];
        const double rh = 2.0 * a.ra * a.length[c] / (PI * a.diam[c] * a.diam[c]) * 1e-2;
        const double rp = 2.0 * a.ra * a.length[pc] / (PI * a.diam[pc] * a.diam[pc]) * 1e-2;
        const double G = 1.0 / (rh + rp);
        a.e[c] = -a.theta * G;
    }
}

// ---------------------------------------------------------------------------
// Epoch kernel.
// ---------------------------------------------------------------------------
template <typename T>
struct State {
    double *V, *R, *D, *Eo, *VO;
    uint64_t *SM, *SP;
    double *IX;    // per neuron: external current (a T in an 8-byte slot)
    int32_t *ND;   // per neuron: detector compartment (pack-local; 8-byte slots)
    T *SG;
};

template <typename T>
__device__ __forceinline__ State<T> carve(char *base, int n, int s, int k) {
    State<T> p;
    double *dp = (double *)base;
    // V, the off-diagonal, R, D: reads the blocked sweeps make a few
    // elements before an array (R, D, off-diagonal) or past its end stay
    // inside the pack's state or the slack after it
    p.V = dp;
    p.Eo = dp + n;
    p.R = dp + 2 * n;
    p.D = dp + 3 * n;
    uint64_t *up = (uint64_t *)(dp + 4 * n);
    p.SM = up;
    p.SP = up + s;
    p.VO = (double *)(up + s + k);
    p.IX = p.VO + k;
    p.ND = (int32_t *)(p.IX + k);
    p.SG = (T *)(p.ND + 2 * k);
    return p;
}

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}

// Events of synapse (pre, delay) in the steps epoch*E + t, t in [0, E): bit t
// set when `pre` spiked at step epoch*E + t - delay (>= 1). Reads only
// epochs before `epoch` because delay >= E, and at most
// ceil((delay + 1) / E) epochs back, which the ring still holds.
__device__ __forceinline__ uint64_t event_mask(const uint64_t *ring, int32_t R, int32_t N,
                                               int32_t E, int64_t epoch, int32_t pre,
                                               int32_t delay) {
    const int64_t g0 = epoch * E - delay - 1;  // history bit of t = 0
    if (g0 + E - 1 < 0) return 0;
    const int64_t w0 = floor_div(g0, E);
    const int off = (int)(g0 - w0 * E);
    const uint64_t lo = (w0 >= 0) ? ring[(w0 % R) * N + pre] : 0ull;
    uint64_t m = lo >> off;
    if (off > 0) {
        const uint64_t hi = (w0 + 1 >= 0) ? ring[((w0 + 1) % R) * N + pre] : 0ull;
        m |= hi << (E - off);
    }
    if (E < 64) m &= (1ull << E) - 1ull;
    return m;
}

// Correctly rounded t / d given y = RN(1/d): q = RN(t y) is within one ulp of
// t/d, the residual t - q d is exact in one fused multiply-add, and
// RN(q + r y) is then the correctly rounded quotient (Markstein's theorem;
// the operands here are far from the underflow and overflow ranges). This
// takes the division off the forward chain: y depends only on the finished
// diagonal and is computed one element ahead.
__device__ __forceinline__ double div_rn(double t, double d, double y) {
    const double q = t * y;
    const double r = __builtin_fma(-q, d, t);
    return __builtin_fma(r, y, q);
}

// Reciprocal to about one ulp: the hardware estimate y (relative error e,
// |e| < 2^-24), then one third-order step y (1 + e + e^2), which leaves a
// relative error of order e^3 before the final rounding (three dependent
// operations where two Newton steps take four).
__device__ __forceinline__ double rcp_nr(double b) {
    const double y = __builtin_amdgcn_rcp(b);
    const double e = __builtin_fma(-b, y, 1.0);
    return __builtin_fma(y, __builtin_fma(e, e, e), y);
}

// Fast solver, between the sweeps: from (P, Q, S) of compartment i form
// g_i = e_i / d'_i (into D) and h_i = r'_i / d'_i (into R), independently
// for every compartment.
__device__ __forceinline__ void pivots_h(double *__restrict__ D, double *__restrict__ R,
                                         const double *__restrict__ Q,
                                         const double *__restrict__ Eo, int i) {
    const double y = rcp_nr(D[i]);
    D[i] = (Eo[i] * Q[i]) * y;
    R[i] = R[i] * y;
}

// Both sweeps walk a branch in blocks of kBlk compartments. A block's
// coefficients are read from LDS together (constant offsets from one
// address, one round trip per block), then the dependent chain runs in
// registers. Every block but the last is full and stores unmasked; the last,
// partial block (at the base for the backward sweep, at the tip for the
// forward sweep) masks its stores and lets the chain run on past the branch
// in registers, which nothing reads afterwards (a parent branch takes its
// children's base states from LDS). A partial block reads up to kBlk-1
// doubles beyond the branch (inside the pack's arrays, or the slack after
// them) and discards them.
#ifndef MMH_SWEEP_BLOCK
#define MMH_SWEEP_BLOCK 5
#endif
constexpr int kBlk = MMH_SWEEP_BLOCK;

// One step of the elimination chain, compartment i+1 -> i (e = e_{i+1},
// dn = D_i, rn = R_i). Exact: (P, S) = (d', r'), the operation order of the
// elimination with a correctly rounded division. Fast: the division-free
// homogeneous form, (P, q, S) with d' = P/q and r' = S/q:
//   P_i = D_i P_{i+1} - e^2 q_{i+1},  S_i = R_i P_{i+1} - e S_{i+1},
//   q_i = P_{i+1}.
template <bool kFast>
__device__ __forceinline__ void chain_step(const double e, const double dn, const double rn,
                                           double &P, double &q, double &S) {
    if constexpr (kFast) {
        const double Pn = __builtin_fma(dn, P, -(e * e) * q);
        const double Sn = __builtin_fma(-e, S, rn * P);
        q = P;
        P = Pn;
        S = Sn;
    } else {
        const double f = div_core(e, P);
        P = dn - f * e;
        S = rn - f * S;
    }
}

// The elimination along one branch, tip b1 down to base b0 (the pivots and
// reduced right-hand sides of Algorithm 1 restricted to the branch; the fast
// form is rescaled by a power of two, exactly, after every full block and
// leaves (P, S, q) in D, R and Q). The base's state stays in D, R (and Q),
// where the parent branch's tip reads it at the next level.
template <bool kFast>
__device__ __forceinline__ void sweep_back_blk(double *__restrict__ D, double *__restrict__ R,
                                               double *__restrict__ Q,
                                               const double *__restrict__ Eo, const Branch b,
                                               const uint16_t *__restrict__ chl) {
    // the tip takes the contributions e^2/d' and e r'/d' of its child
    // branches, formed here from the base states the children left in D, R
    // (and Q). Exact: subtracted in descending base order. Fast: merged in
    // homogeneous form, d'/q - e^2 q_c/P_c over the common denominator
    // q P_c (likewise r'), so the tip needs no division either; the merged
    // state is rescaled by a power of two like the chain's.
    double P = D[b.b1], S = R[b.b1], q = 1.0;
    if constexpr (kFast) {
        auto merge = [&](const int j) {
            const double e0 = Eo[j], Pc = D[j], qc = Q[j], Sc = R[j];
            const double Pn = __builtin_fma(P, Pc, -((e0 * e0) * qc) * q);
            const double Sn = __builtin_fma(S, Pc, -(e0 * Sc) * q);
            q = q * Pc;
            P = Pn;
            S = Sn;
        };
        auto rescale = [&]() {
            const int x = -__builtin_amdgcn_frexp_exp(P);
            P = __builtin_amdgcn_ldexp(P, x);
            q = __builtin_amdgcn_ldexp(q, x);
            S = __builtin_amdgcn_ldexp(S, x);
        };
        if (b.nchild == 2) {
            merge(b.cb[1]);
            merge(b.cb[0]);
            rescale();
        } else {
            // any fan-out: rescaled after every child, so that a node with
            // many children cannot drive the products out of range
            for (int c = b.nchild - 1; c >= 0; --c) {
                merge(chl[b.child0 + c]);
                rescale();
            }
        }
    } else {
        auto contribution = [&](const int j, double &cd, double &cr) {
            const double f = div_core(Eo[j], D[j]);
            cd = f * Eo[j];
            cr = f * R[j];
        };
        if (b.nchild == 2) {
            double cd1, cr1, cd0, cr0;
            contribution(b.cb[1], cd1, cr1);
            contribution(b.cb[0], cd0, cr0);
            P = P - cd1;
            S = S - cr1;
            P = P - cd0;
            S = S - cr0;
        } else {
            for (int c = b.nchild - 1; c >= 0; --c) {
                double cd, cr;
                contribution(chl[b.child0 + c], cd, cr);
                P = P - cd;
                S = S - cr;
            }
        }
    }
    D[b.b1] = P;
    R[b.b1] = S;
    if constexpr (kFast) Q[b.b1] = q;
    int i = b.b1;  // the next compartment is i-1
    for (; i - kBlk >= b.b0; i -= kBlk) {  // full blocks from the tip
        const double *pe = Eo + i - (kBlk - 1);
        double *pd = D + i - kBlk, *pr = R + i - kBlk, *pq = Q + i - kBlk;
        double e[kBlk], dn[kBlk], rn[kBlk];
#pragma unroll
        for (int j = 0; j < kBlk; ++j) {
            e[j] = pe[kBlk - 1 - j];
            dn[j] = pd[kBlk - 1 - j];
            rn[j] = pr[kBlk - 1 - j];
        }
#pragma unroll
        for (int j = 0; j < kBlk; ++j) {
            chain_step<kFast>(e[j], dn[j], rn[j], P, q, S);
            pd[kBlk - 1 - j] = P;
            pr[kBlk - 1 - j] = S;
            if constexpr (kFast) pq[kBlk - 1 - j] = q;
        }
        if constexpr (kFast) {
            const int x = -__builtin_amdgcn_frexp_exp(P);
            P = __builtin_amdgcn_ldexp(P, x);
            q = __builtin_amdgcn_ldexp(q, x);
            S = __builtin_amdgcn_ldexp(S, x);
        }
    }
    if (i > b.b0) {  // partial block at the base: stores masked, state not needed
        const double *pe = Eo + i - (kBlk - 1);
        double *pd = D + i - kBlk, *pr = R + i - kBlk, *pq = Q + i - kBlk;
        double e[kBlk], dn[kBlk], rn[kBlk];
#pragma unroll
        for (int j = 0; j < kBlk - 1; ++j) {
            e[j] = pe[kBlk - 1 - j];
            dn[j] = pd[kBlk - 1 - j];
            rn[j] = pr[kBlk - 1 - j];
        }
        const int nv = i - b.b0;
#pragma unroll
        for (int j = 0; j < kBlk - 1; ++j) {
            chain_step<kFast>(e[j], dn[j], rn[j], P, q, S);
            if (j < nv) {
                pd[kBlk - 1 - j] = P;
                pr[kBlk - 1 - j] = S;
                if constexpr (kFast) pq[kBlk - 1 - j] = q;
            }
        }
    }
}

// One back-substitution step: exact x = (r' - e x_parent)/d' correctly
// rounded given y = RN(1/d'); fast x = h - g x_parent.
template <bool kFast>
__device__ __forceinline__ double subst_step(const double g, const double h, const double e,
                                             const double y, const double x) {
    if constexpr (kFast)
        return __builtin_fma(-g, x, h);
    else
        return div_rn(h - e * x, g, y);
}

// Back-substitution along one branch, base to tip. Exact: V holds RN(1/d')
// of the branch's own compartments on entry (D, R hold d', r'). Fast: D and R
// hold g = e/d' and h = r'/d'. V[par] is already the parent's new voltage.
template <bool kFast>
__device__ __forceinline__ void sweep_fwd_blk(double *__restrict__ V, const double *__restrict__ D,
                                              const double *__restrict__ R,
                                              const double *__restrict__ Eo, const Branch b) {
    // the base is the first element of the first block, against the parent's
    // new voltage (a root has none: its coupling e is +0, so 0 stands in)
    double x = b.par != kRootPar ? V[b.par] : 0.0;
    int i = b.b0;
    for (; i + kBlk - 1 <= b.b1; i += kBlk) {  // full blocks
        const double *pg = D + i, *ph = R + i, *pe = Eo + i;
        double *pv = V + i;
        double g[kBlk], h[kBlk], e[kBlk], y[kBlk];
#pragma unroll
        for (int j = 0; j < kBlk; ++j) {
            g[j] = pg[j];
            h[j] = ph[j];
            if constexpr (!kFast) {
                e[j] = pe[j];
                y[j] = pv[j];
            }
        }
#pragma unroll
        for (int j = 0; j < kBlk; ++j) {
            x = subst_step<kFast>(g[j], h[j], e[j], y[j], x);
            pv[j] = x;
        }
    }
    if (i <= b.b1) {  // partial block at the tip
        const double *pg = D + i, *ph = R + i, *pe = Eo + i;
        double *pv = V + i;
        double g[kBlk], h[kBlk], e[kBlk], y[kBlk];
#pragma unroll
        for (int j = 0; j < kBlk - 1; ++j) {
            g[j] = pg[j];
            h[j] = ph[j];
            if constexpr (!kFast) {
                e[j] = pe[j];
                y[j] = pv[j];
            }
        }
        const int nv = b.b1 - i + 1;
#pragma unroll
        for (int j = 0; j < kBlk - 1; ++j) {
            x = subst_step<kFast>(g[j], h[j], e[j], y[j], x);
            if (j < nv) pv[j] = x;
        }
    }
}

// Tree contraction (the third solver). Eliminating compartment k with its
// current neighbours n1, n2 (couplings a1, a2) is one step of Gaussian
// elimination: each neighbour's diagonal loses a^2/d_k and its right-hand
// side a r_k/d_k; when both exist, n2 is linked to n1 with the coupling
// -a1 a2/d_k. The V slot, free once the matrix is assembled, takes the
// couplings made by these fills (W, followed in memory by the off-diagonal:
// a coupling no elimination has made yet is still the off-diagonal entry,
// and the item gives the index of either, see make_citem). What k's back
// substitution needs replaces what k no longer needs: h = r_k/d_k into
// R[k], g1 = a1/d_k into W[k], g2 = a2/d_k into D[k]. A round's
// eliminations are at least three apart in the current tree, so each
// survivor is written by one lane at most.
// k, n1 and n2 are distinct, so every value is read before anything is
// written, with no branches and no selects: the reads go out together (one
// LDS round trip) rather than each waiting for the write before it, as they
// would if the compiler had to assume the slots may alias. An absent
// neighbour is the pack's spare compartment, read with a coupling of 0: the
// updates meant for it land in the spare's own slots, which stay finite and
// are only ever read multiplied by a zero coupling, and a fill made with it
// is never read (a compartment left without a parent is a root from then
// on).
__device__ __forceinline__ void contract_elim(double *__restrict__ D, double *__restrict__ R,
                                              double *__restrict__ W, const int m,
                                              const uint64_t it) {
    const int k = (int)(it & 0x7FFFu);
    const int i1 = (int)(it >> 15) & 0xFFFF, i2 = (int)(it >> 31) & 0xFFFF;
    const int u1 = (int)(it >> 47) & 0xFFFF;
    const int u2 = (it >> 63) ? i2 : i2 + m;
    const double dk = D[k], rk = R[k];
    const double a1 = W[u1], a2 = W[u2];
    const double d1 = D[i1], r1 = R[i1], d2 = D[i2], r2 = R[i2];
    const double y = rcp_nr(dk);
    const double h = rk * y, g1 = a1 * y, g2 = a2 * y;
    D[i1] = __builtin_fma(-a1, g1, d1);
    R[i1] = __builtin_fma(-a1, h, r1);
    D[i2] = __builtin_fma(-a2, g2, d2);
    R[i2] = __builtin_fma(-a2, h, r2);
    W[i2] = -(a1 * g2);
    R[k] = h;
    W[k] = g1;
    D[k] = g2;
}

// Back substitution of k, its neighbours at elimination time solved already
// (their solutions in the V slot): x_k = h - g1 x_n1 - g2 x_n2, into V[k]
// (an absent neighbour's g is 0).
__device__ __forceinline__ void contract_subst(const double *__restrict__ R,
                                               const double *__restrict__ D,
                                               double *__restrict__ V, const uint64_t it) {
    const int k = (int)(it & 0x7FFFu);
    const int i1 = (int)(it >> 15) & 0xFFFF, i2 = (int)(it >> 31) & 0xFFFF;
    const double rk = R[k], g1 = V[k], g2 = D[k];
    const double x1 = V[i1], x2 = V[i2];
    double x = rk;
    x = __builtin_fma(-g1, x1, x);
    x = __builtin_fma(-g2, x2, x);
    V[k] = x;
}

// Orders this wavefront's LDS accesses across lanes: LDS performs a
// wavefront's instructions in issue order, so a read issued after a write
// (by any lane of the same wavefront) sees it; only the compiler must be kept
// from moving accesses across (a wavefront-scope fence, which waits for
// nothing).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

struct Consts {
    double omt, vth, ginv;
};

// A copy of a wave-uniform value in a scalar register of its own (the
// compiler cannot see through the move).
__device__ __forceinline__ double sreg(double x) {
    double y;
    asm volatile("s_mov_b64 %0, %1" : "=s"(y) : "s"(x));
    return y;
}
__device__ __forceinline__ float sreg(float x) {
    float y;
    asm volatile("s_mov_b32 %0, %1" : "=s"(y) : "s"(x));
    return y;
}

// Channel constants of the membrane model, in the gating precision.
template <typename T>
struct Chan {
    T gnabar, gkbar, gl, ena, ek, el, g_pas, e_pas, e_syn, dt, q;
};
template <typename T>
__device__ __forceinline__ Chan<T> chan_consts(const EpochArgs &a) {
    if constexpr (sizeof(T) == 4) {
        const float *f = a.fch;
        return Chan<T>{sreg(f[0]), sreg(f[1]), sreg(f[2]), sreg(f[3]), sreg(f[4]),  sreg(f[5]),
                       sreg(f[6]), sreg(f[7]), sreg(f[8]), sreg(f[9]), sreg(f[10])};
    } else {
        return Chan<T>{sreg(a.gnabar), sreg(a.gkbar), sreg(a.gl),    sreg(a.ena),
                       sreg(a.ek),     sreg(a.el),    sreg(a.g_pas), sreg(a.e_pas),
                       sreg(a.e_syn),  sreg(a.dt),    sreg(a.q)};
    }
}

// Membrane conductance and source of one compartment from its gates, per
// unit of the compartment's own area factor: P = a*g_ion, Q = a*J_ion
// (HH: g = gNa m^3 h + gK n^4 + gL, J = gNa m^3 h ENa + gK n^4 EK + gL EL;
// passive: g_pas and g_pas e_pas). They are formed when the gates are
// advanced, so that the assembly of the next step needs no gates; the
// synaptic delivery then adds g_syn to P and g_syn E_syn to Q.
template <typename T>
__device__ __forceinline__ void membrane(const uint32_t tp, const T afv, const T m, const T h,
                                         const T x, const Chan<T> &c, T &P, T &Q) {
    T gion, jion;
    if (topo_hh(tp)) {
        const T gna = c.gnabar * (((m * m) * m) * h);
        const T gk = c.gkbar * (((x * x) * x) * x);
        gion = (gna + gk) + c.gl;
        jion = (gna * c.ena + gk * c.ek) + c.gl * c.el;
    } else {
        gion = c.g_pas;
        jion = c.g_pas * c.e_pas;
    }
    P = afv * gion;
    Q = afv * jion;
}

// Phase B for one compartment: the membrane terms (P, Q, synaptic part
// included) from the D and R slots, the external current of a root,
// axial current and diagonal from the couplings to the parent and the
// children (children in ascending order, as the time-invariant diagonal is
// defined), then D_i and R_i.
template <typename T>
__device__ __forceinline__ void assemble(const int i, const uint32_t tp, const double cdt,
                                         const double *__restrict__ V, double *__restrict__ R,
                                         double *__restrict__ D, const double *__restrict__ Eo,
                                         const Branch *__restrict__ br,
                                         const uint16_t *__restrict__ chl,
                                         const double *__restrict__ IX, const Consts c) {
    const double v = V[i];
    const T gmem = *(const T *)&D[i];
    const T jm = *(const T *)&R[i];
    const bool root = topo_root(tp);
    const T iext = root ? *(const T *)&IX[topo_parent(tp)] : T(0);
    const T J = jm + iext;
    double ax, d = cdt;
    if (root) {
        ax = 0.0;
    } else {
        const double ei = Eo[i];
        ax = (ei * c.ginv) * (V[topo_parent(tp)] - v);
        d = d - ei;
    }
    const uint32_t bid = topo_branch(tp);
    if (bid == kNone) {
        const double e1 = Eo[i + 1];
        ax = ax - (e1 * c.ginv) * (v - V[i + 1]);
        d = d - e1;
    } else {
        const Branch b = br[bid];
        for (int q = 0; q < b.nchild; ++q) {
            const int j = chl[b.child0 + q];
            const double ej = Eo[j];
            ax = ax - (ej * c.ginv) * (v - V[j]);
            d = d - ej;
        }
    }
    D[i] = d + (double)gmem;
    R[i] = (cdt * v + (double)J) + c.omt * ax;
}

// Phase B with the compartment's children word (chw, see make_children):
// the same operations in the same order as assemble(), but every operand is
// read at once, with no dependent read of a branch record or child list (an
// absent child reads the compartment's own slots, a root reads the slot its
// topology word names in place of a parent's, and neither term is applied).
// A compartment with more than two children takes assemble()'s path.
template <typename T>
__device__ __forceinline__ void assemble_cw(const int i, const uint32_t tp, const uint32_t chw,
                                            const double cdt, const double *__restrict__ V,
                                            double *__restrict__ R, double *__restrict__ D,
                                            const double *__restrict__ Eo,
                                            const Branch *__restrict__ br,
                                            const uint16_t *__restrict__ chl,
                                            const double *__restrict__ IX, const Consts c) {
    if (chw == kManyChildren) {
        assemble<T>(i, tp, cdt, V, R, D, Eo, br, chl, IX, c);
        return;
    }
    const bool root = topo_root(tp);
    const int pi = (int)topo_parent(tp);  // the neuron's index in the pack at a root
    const uint32_t u1 = chw & 0xFFFFu, u2 = chw >> 16;
    const bool h1 = u1 != kNoNb, h2 = u2 != kNoNb;
    const int c1 = h1 ? (int)u1 : i, c2 = h2 ? (int)u2 : i;
    const double v = V[i];
    const T gmem = *(const T *)&D[i];
    const T jm = *(const T *)&R[i];
    const T ix = *(const T *)&IX[root ? pi : 0];  // (IX holds one entry per neuron)
    const double ei = Eo[i], vp = V[pi];
    const double e1 = Eo[c1], v1 = V[c1], e2 = Eo[c2], v2 = V[c2];
    const T J = jm + (root ? ix : T(0));
    double ax = 0.0, d = cdt;
    if (!root) {
        ax = (ei * c.ginv) * (vp - v);
        d = d - ei;
    }
    if (h1) {
        ax = ax - (e1 * c.ginv) * (v - v1);
        d = d - e1;
    }
    if (h2) {
        ax = ax - (e2 * c.ginv) * (v - v2);
        d = d - e2;
    }
    D[i] = d + (double)gmem;
    R[i] = (cdt * v + (double)J) + c.omt * ax;
}

template <typename T>
__device__ __forceinline__ void gates_update(const double v64, T &m, T &h, T &x, const T dt) {
    const T v = (T)v64;
    T am, bm, ah, bh, an, bn;
    hh_rates<T>(v, am, bm, ah, bh, an, bn);
    m = gate_step<T>(m, am, bm, dt);
    h = gate_step<T>(h, ah, bh, dt);
    x = gate_step<T>(x, an, bn, dt);
}

// The pack's tables, staged in LDS for the whole epoch: branch records (in
// backward order), synapse weights, level offsets, the forward order (record
// ids), child list, synapse targets and run lengths; the contraction solver
// stages none of the branch tables (kNoBranch), but its round offsets and
// the items of its schedule's tail. The layout must match
// pack_table_bytes().
template <typename T>
struct Tables {
    Branch *br;
    uint16_t *fw;
    T *sw;
    int32_t *lvl;
    uint16_t *chl, *scomp, *sseg;
    int32_t *crof;  // contraction round offsets
    uint64_t *cst;  // contraction items staged in LDS (the schedule's last ones)
};

template <typename T, bool kNoBranch>
__device__ __forceinline__ Tables<T> carve_tables(char *smem, const PackDesc &pk) {
    const int nbr = kNoBranch ? 0 : pk.nbr, nch = kNoBranch ? 0 : pk.nch;
    const int nlev = kNoBranch ? 0 : pk.nbw + pk.nfw + 2;
    Tables<T> t;
    t.br = (Branch *)smem;
    t.sw = (T *)(t.br + nbr);
    char *p = (char *)(t.sw + pk.nsyn);
    p = smem + (((p - smem) + 3) / 4) * 4;
    t.lvl = (int32_t *)p;
    t.fw = (uint16_t *)(t.lvl + nlev);
    t.chl = t.fw + nbr;
    t.scomp = t.chl + nch;
    t.sseg = t.scomp + pk.nsyn;
    char *q = (char *)(t.sseg + pk.nsyn);
    t.crof = (int32_t *)(smem + (((q - smem) + 3) / 4) * 4);
    char *u = (char *)(t.crof + (pk.nrnd > 0 ? pk.nrnd + 1 : 0));
    t.cst = (uint64_t *)(smem + (((u - smem) + 7) / 8) * 8);
    return t;
}

// Compartments per thread whose gates and constants stay in registers for
// the whole epoch (FP32 gating, contraction solver): compartment tid + j*NT
// for j < kResident. The rest of a larger pack reads them from global memory
// each step, as do the level-sweep solvers (whose sweeps already hold most
// of the register budget) and FP64 gating (whose gates take twice the
// registers). A launch whose packs all fit the resident slots (kRes) leaves
// those paths out, which frees the scalar registers they held.

// One pack through steps [t0, t1) of an epoch. V, R, D and the off-diagonal
// live at `base` (LDS, or a global scratch slice for packs larger than any
// LDS budget). With FP32 gating each thread holds the gates, area factor,
// topology word and C/dt of its first kResident compartments in registers,
// loaded once per epoch; the gates go back to memory at the end.
// Between the gate update of one step and the assembly of the next, the D
// and R slots carry each compartment's membrane terms P and Q.
// In the sweeps the branches of a level go to consecutive lanes (sorted by
// length on the host), so one wave instruction advances as many chains as
// the level has branches.
template <typename T, int kSolve, bool kRes>
__device__ __forceinline__ void run_pack(const EpochArgs &a, const PackDesc &pk, char *smem,
                                         char *base, int64_t epoch) {
    constexpr bool kFast = kSolve == 1;
    constexpr bool kContract = kSolve == 2;
    const int tid = threadIdx.x;
    const int NT = blockDim.x;
    const int slot = tid;
    const int n = pk.ncomp, ns = pk.nsyn, nn = pk.nneur;
    const int64_t c0 = pk.comp0, s0 = pk.syn0;
    // (the contraction solver's arrays end with a spare compartment, n)
    const int m = kContract ? n + 1 : n;
    const State<T> st = carve<T>(base, m, ns, nn);
    const Tables<T> tb = carve_tables<T, kContract>(smem, pk);
#ifdef MMH_PHASE_PROFILE
    uint64_t ph_t_ = threadIdx.x == 0 ? wall_clock64() : 0;
    uint64_t ph_acc_[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#endif
    {
        if constexpr (!kContract) {
            const Branch *gbr = a.br + pk.br0;
            const uint16_t *gfw = a.fw + pk.br0;
            for (int k = tid; k < pk.nbr; k += NT) {
                tb.br[k] = gbr[k];
                tb.fw[k] = gfw[k];
            }
            const uint16_t *gch = a.chl + pk.ch0;
            for (int k = tid; k < pk.nch; k += NT) tb.chl[k] = gch[k];
            const int32_t *glv = a.lvl + pk.lv0;
            for (int k = tid; k < pk.nbw + pk.nfw + 2; k += NT) tb.lvl[k] = glv[k];
        }
        const T *gsw = (const T *)a.sw + s0;
        for (int k = tid; k < ns; k += NT) {
            tb.sw[k] = gsw[k];
            tb.scomp[k] = a.scomp[s0 + k];
            tb.sseg[k] = a.sseg[s0 + k];
        }
        if constexpr (kContract) {
            const int32_t *gro = a.lvl + pk.lv0 + pk.nbw + pk.nfw + 2;
            for (int k = tid; k <= pk.nrnd; k += NT) tb.crof[k] = gro[k];
            const uint64_t *gst = a.cit + pk.it0 + (pk.ncomp - pk.nst);
            for (int k = tid; k < pk.nst; k += NT) tb.cst[k] = gst[k];
        }
    }
    double *__restrict__ V = st.V;
    const int lane = tid & (kWave - 1);
    uint64_t spt = 0;  // lane t: this wave's crossings at step t (bit l: lane l's neuron)
    double *__restrict__ R = st.R;
    double *__restrict__ D = st.D;
    double *__restrict__ Eo = st.Eo;
    T *__restrict__ SG = st.SG;

    T *gm = (T *)a.gm + c0, *gh = (T *)a.gh + c0, *gn = (T *)a.gn + c0;
    const T *af = (const T *)a.af + c0;
    const double *cdtp = a.cdt + c0;
    const uint32_t *topo = a.topo + c0;
    const uint32_t *cnbp = a.cnb + c0;
    const T *niext = (const T *)a.niext;
    double *__restrict__ IX = st.IX;
    // (the contraction solver's assembly reads a branch record and child
    // list only for a compartment of more than two children: from global
    // memory)
    const Branch *br = kContract ? a.br + pk.br0 : tb.br;
    const uint16_t *chl = kContract ? a.chl + pk.ch0 : tb.chl;
    const int32_t *lvl = tb.lvl;

    // Each constant is copied into a scalar register of its own: otherwise
    // the compiler keeps the wide scalar loads they came from (eight doubles
    // in one register tuple) alive across the step loop, and when that tuple
    // spills it reloads all of it wherever one constant is used.
    const Chan<T> ch = chan_consts<T>(a);
    const Consts cs{sreg(a.omt), sreg(a.v_thresh), sreg(a.ginv)};
    const T e_syn = ch.e_syn, dt = ch.dt, q = ch.q;
    const int t0 = a.t0, t1 = a.t1;

    // resident compartments: tid + j*NT for j < KR; the others from i0 on
    constexpr int KR = (sizeof(T) == 4 && kContract) ? kResident : 0;
    static_assert(!kRes || KR > 0, "the resident-only kernel needs register slots");
    constexpr int KA = KR > 0 ? KR : 1;
    const int i0 = tid + KR * NT;
    T rm[KA], rh[KA], rx[KA], raf[KA];
    double rcdt[KA];
    uint32_t rtp[KA], rcw[KA];

    // ---- load state -------------------------------------------------------
    for (int i = tid; i < n; i += NT) {
        V[i] = a.V[c0 + i];
        Eo[i] = a.e[c0 + i];
    }
    if (kContract && tid == 0) {  // the spare compartment: a zero coupling, finite values
        V[n] = 0.0;
        Eo[n] = 0.0;
        D[n] = 0.0;
        R[n] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        const int i = tid + j * NT;
        if (i < n) {
            rm[j] = gm[i];
            rh[j] = gh[i];
            rx[j] = gn[i];
            raf[j] = af[i];
            rcdt[j] = cdtp[i];
            rtp[j] = topo[i];
            rcw[j] = cnbp[i];
            membrane<T>(rtp[j], raf[j], rm[j], rh[j], rx[j], ch, *(T *)&D[i], *(T *)&R[i]);
        }
    }
    if constexpr (!kRes)
        for (int i = i0; i < n; i += NT)
            membrane<T>(topo[i], af[i], gm[i], gh[i], gn[i], ch, *(T *)&D[i], *(T *)&R[i]);
    for (int k = tid; k < ns; k += NT) {
        SG[k] = ((const T *)a.sg)[s0 + k];
        st.SM[k] = event_mask(a.ring, a.ring_rows, a.n_neurons, a.E, epoch, a.spre[s0 + k],
                              a.sdelay[s0 + k]);
    }
    for (int k = tid; k < nn; k += NT) {
        const int32_t det = a.ndet[pk.neur0 + k];
        st.VO[k] = a.V[c0 + det];
        st.ND[2 * k] = det;
        *(T *)&IX[k] = niext[pk.neur0 + k];
        st.SP[k] = 0ull;
    }
    __syncthreads();
    MMH_PHASE(0);

    for (int t = t0; t < t1; ++t) {
        // the resident slots' thread index and topology words pass through
        // an empty asm once per step: otherwise the compiler hoists their
        // loop-invariant LDS addresses and loads out of the step loop and
        // holds them in registers for every slot
        int tl = tid;
        asm volatile("" : "+v"(tl));
#pragma unroll
        for (int j = 0; j < KR; ++j) asm volatile("" : "+v"(rtp[j]), "+v"(rcw[j]));
        // ---- A: delivery; each compartment's synaptic conductance joins its
        // membrane terms (P += g, Q += g E_syn) ------------------------------
        for (int k = tid; k < ns; k += NT) {
            const int L = tb.sseg[k];
            if (L == 0) continue;
            T sum = T(0);
            for (int j = k; j < k + L; ++j) {
                T g = SG[j];
                if (t > t0) g = q * g;
                if ((st.SM[j] >> t) & 1ull) g = g + tb.sw[j];
                SG[j] = g;
                sum = sum + g;
            }
            const int c = tb.scomp[k];
            T *P = (T *)&D[c];
            T *Q = (T *)&R[c];
            *P = *P + sum;
            *Q = *Q + sum * e_syn;
        }
        __syncthreads();
        MMH_PHASE(1);

        // ---- B: assembly ------------------------------------------------------
#pragma unroll
        for (int j = 0; j < KR; ++j) {
            const int i = tl + j * NT;
            if (i < n) assemble_cw<T>(i, rtp[j], rcw[j], rcdt[j], V, R, D, Eo, br, chl, IX, cs);
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (kContract && !kRes) {
#pragma unroll 2
            for (int i = i0; i < n; i += NT)
                assemble_cw<T>(i, topo[i], cnbp[i], cdtp[i], V, R, D, Eo, br, chl, IX, cs);
        } else if constexpr (!kRes) {
#pragma unroll 2
            for (int i = i0; i < n; i += NT)
                assemble<T>(i, topo[i], cdtp[i], V, R, D, Eo, br, chl, IX, cs);
        }
        __syncthreads();
        MMH_PHASE(2);

        if constexpr (kContract) {
            // ---- C': contraction rounds, then back substitution ------------
            // (V^n is no longer needed: detection keeps its own copy, so the
            // V slot takes the couplings the eliminations make)
            // every thread takes items of each round, a workgroup barrier
            // between rounds; the items stay in global memory (L2), and each
            // thread reads its first item of the next round before working on
            // the current one, so the read overlaps the round and its barrier.
            // The tail of small rounds (at most one wavefront's worth of
            // items each) runs on the first wavefront alone, which needs no
            // workgroup barrier between rounds: its lanes run in lockstep, so
            // waiting for its own LDS writes to complete is enough.
            const uint64_t *__restrict__ cit = a.cit + pk.it0;
            const int32_t *rof = tb.crof;
            const int nr = pk.nrnd, nw = pk.nrw, qs = n - pk.nst;
            const uint64_t *cst = tb.cst;  // item q >= qs staged at cst[q - qs]
            auto item = [&](int q, int end) -> uint64_t {
                return q < end ? (q >= qs ? cst[q - qs] : cit[q]) : 0ull;
            };
            {
                int lo = rof[0], hi = rof[nr > 0 ? 1 : 0];
                uint64_t cur = item(lo + tid, hi);
                for (int r = 0; r < nw; ++r) {
                    // the next round's end and first item, read before this
                    // round's work and barrier
                    const int hi2 = (r + 1 < nr) ? rof[r + 2] : hi;
                    const uint64_t nxt = item(hi + tid, hi2);
                    if (lo + tid < hi) contract_elim(D, R, V, m, cur);
                    for (int q2 = lo + tid + NT; q2 < hi; q2 += NT)
                        contract_elim(D, R, V, m, cit[q2]);
                    __syncthreads();
                    lo = hi;
                    hi = hi2;
                    cur = nxt;
                }
                if (tid < kWave) {
                    // the tail's items are all staged in LDS (the host moves
                    // the tail's start past any round that is not), and lane
                    // l holds the round offset rof[nw + l]: the next round's
                    // bounds come from a register, not a dependent LDS read
                    const int rl = (nw + tid <= nr) ? rof[nw + tid] : 0;
                    auto rofw = [&](int r) { return __builtin_amdgcn_readlane(rl, r - nw); };
                    // (reads clamped into the staged range rather than
                    // branched around, so that no wait is needed before the
                    // current round's own reads)
                    const int qmax = pk.nst - 1;
                    auto tail_item = [&](int q) { return cst[max(0, min(q - qs, qmax))]; };
                    if (nw < nr) cur = tail_item(lo + tid);
                    for (int r = nw; r < nr; ++r) {
                        const int hi2 = (r + 1 < nr) ? rofw(r + 2) : hi;
                        const uint64_t nxt = tail_item(hi + tid);
                        if (lo + tid < hi) contract_elim(D, R, V, m, cur);
                        wave_lds_sync();
                        lo = hi;
                        hi = hi2;
                        cur = nxt;
                    }
                    MMH_PHASE(3);
                    // back substitution of the tail, in reverse round order
                    if (nw < nr) {
                        hi = rofw(nr);
                        lo = rofw(nr - 1);
                        cur = tail_item(lo + tid);
                    }
                    for (int r = nr - 1; r >= nw; --r) {
                        const int lo2 = (r - 1 >= nw) ? rofw(r - 1) : lo;
                        const uint64_t nxt = tail_item(lo2 + tid);
                        if (lo + tid < hi) contract_subst(R, D, V, cur);
                        wave_lds_sync();
                        hi = lo;
                        lo = lo2;
                        cur = nxt;
                    }
                }
                __syncthreads();
            }
            {
                int hi = rof[nw], lo = rof[nw > 0 ? nw - 1 : 0];
                uint64_t cur = item(lo + tid, hi);
                for (int r = nw - 1; r >= 0; --r) {
                    const int lo2 = (r > 0) ? rof[r - 1] : lo;
                    const uint64_t nxt = item(lo2 + tid, lo);
                    if (lo + tid < hi) contract_subst(R, D, V, cur);
                    for (int q2 = lo + tid + NT; q2 < hi; q2 += NT)
                        contract_subst(R, D, V, cit[q2]);
                    __syncthreads();
                    hi = lo;
                    lo = lo2;
                    cur = nxt;
                }
            }
            MMH_PHASE(4);
        } else {

        // ---- C: backward sweep by height -----------------------------------
        // (V^n is no longer needed: detection keeps its own copy, so the V
        // slot holds the reciprocal pivots, or Q of the fast solver). Each
        // lane takes entry `slot` of a level; the next level's bounds and
        // record are read before the current level's chains run, so their
        // latency is hidden (the tables are constant).
        {
            int lo = lvl[0], hi = lvl[1];
            Branch cur = br[min(lo + slot, pk.nbr - 1)];
            for (int h = 0; h < pk.nbw; ++h) {
                const int hi2 = lvl[min(h + 2, pk.nbw)];
                const Branch nxt = br[min(hi + slot, pk.nbr - 1)];
                if (lo + slot < hi) sweep_back_blk<kFast>(D, R, V, Eo, cur, chl);
                for (int q2 = lo + slot + NT; q2 < hi; q2 += NT)
                    sweep_back_blk<kFast>(D, R, V, Eo, br[q2], chl);
                __syncthreads();
                cur = nxt;
                lo = hi;
                hi = hi2;
            }
        }
        for (int i = tid; i < n; i += NT) {
            if constexpr (kFast)
                pivots_h(D, R, V, Eo, i);
            else
                V[i] = div_core(1.0, D[i]);
        }
        __syncthreads();
        MMH_PHASE(3);

        // ---- D: forward sweep by depth -------------------------------------
        {
            const int32_t *flv = lvl + pk.nbw + 1;
            const uint16_t *fw = tb.fw;
            int lo = flv[0], hi = flv[1];
            Branch cur = br[fw[min(lo + slot, pk.nbr - 1)]];
            for (int h = 0; h < pk.nfw; ++h) {
                const int hi2 = flv[min(h + 2, pk.nfw)];
                const Branch nxt = br[fw[min(hi + slot, pk.nbr - 1)]];
                if (lo + slot < hi) sweep_fwd_blk<kFast>(V, D, R, Eo, cur);
                for (int q2 = lo + slot + NT; q2 < hi; q2 += NT)
                    sweep_fwd_blk<kFast>(V, D, R, Eo, br[fw[q2]]);
                __syncthreads();
                cur = nxt;
                lo = hi;
                hi = hi2;
            }
        }
        MMH_PHASE(4);
        }  // level-synchronous solvers

        // ---- E: gates at V^{n+1}, the next step's membrane terms; detection
        const bool more = t + 1 < t1;
#pragma unroll
        for (int j = 0; j < KR; ++j) {
            const int i = tl + j * NT;
            if (i < n) {
                if (topo_hh(rtp[j])) gates_update<T>(V[i], rm[j], rh[j], rx[j], dt);
                if (more)
                    membrane<T>(rtp[j], raf[j], rm[j], rh[j], rx[j], ch, *(T *)&D[i],
                                *(T *)&R[i]);
            }
            // one compartment's gate update at a time: interleaving them
            // would hold several sets of rate temporaries live at once
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (!kRes) {
#pragma unroll 1
            for (int i = i0; i < n; i += NT) {
                const uint32_t tp = topo[i];
                T m = gm[i], h = gh[i], x = gn[i];
                if (topo_hh(tp)) {
                    gates_update<T>(V[i], m, h, x, dt);
                    gm[i] = m;
                    gh[i] = h;
                    gn[i] = x;
                }
                if (more) membrane<T>(tp, af[i], m, h, x, ch, *(T *)&D[i], *(T *)&R[i]);
            }
        }
        // detection: lane l of wave w watches neuron 64 w + l; a ballot
        // gathers the step's threshold crossings of the wave's neurons into
        // one mask, which lane t keeps (the masks are turned into per-neuron
        // step masks once, at the end of the launch)
        if (tid - lane < nn) {
            bool cross = false;
            if (tid < nn) {
                const double vn = V[st.ND[2 * tid]];
                cross = st.VO[tid] < cs.vth && vn >= cs.vth;
                st.VO[tid] = vn;
            }
            const uint64_t m = __ballot(cross);
            if (lane == t) spt = m;
        }
        for (int k = tid + NT; k < nn; k += NT) {  // packs of more neurons than threads
            const double vn = V[st.ND[2 * k]];
            if (st.VO[k] < cs.vth && vn >= cs.vth) st.SP[k] |= 1ull << t;
            st.VO[k] = vn;
        }
        __syncthreads();
        MMH_PHASE(5);
    }

    // ---- write back -----------------------------------------------------------
    // the wave's step masks, transposed by ballots: bit t of neuron l's mask
    // is bit l of lane t's step mask
    if (tid - lane < nn) {
        const int nb = min(kWave, nn - (tid - lane));
        uint64_t mine = 0;
        for (int b = 0; b < nb; ++b) {
            const uint64_t w = __ballot((spt >> b) & 1ull);
            if (lane == b) mine = w;
        }
        if (lane < nb) st.SP[tid] = mine;
    }
    __syncthreads();
    for (int i = tid; i < n; i += NT) a.V[c0 + i] = V[i];
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        const int i = tid + j * NT;
        if (i < n && topo_hh(rtp[j])) {
            gm[i] = rm[j];
            gh[i] = rh[j];
            gn[i] = rx[j];
        }
    }
    if (t1 > t0) {
        T *osg = (T *)a.sg;
        for (int k = tid; k < ns; k += NT) osg[s0 + k] = q * SG[k];
    }
    // the epoch's ring row: a launch that starts the epoch replaces the row's
    // previous contents (an epoch ring_rows earlier); a launch that continues
    // it adds its steps' bits
    for (int k = tid; k < nn; k += NT) {
        uint64_t *w = a.ring + (epoch % a.ring_rows) * a.n_neurons + a.nid[pk.neur0 + k];
        if (t0 == 0)
            *w = st.SP[k];
        else if (st.SP[k])
            *w = *w | st.SP[k];
    }
    MMH_PHASE(6);
#ifdef MMH_PHASE_PROFILE
    if (threadIdx.x == 0)
        for (int k = 0; k < 7; ++k) atomicAdd(&g_phase_ticks[k], (unsigned long long)ph_acc_[k]);
#endif
}

template <typename T, int kSolve, bool kRes = false>
__global__ void __launch_bounds__(sizeof(T) == 8 ? kMaxThreadsF64 : kMaxThreadsF32)
    k_epoch(EpochArgs a) {
    extern __shared__ __align__(16) char smem[];
    const int64_t epoch = a.epoch_ptr ? *a.epoch_ptr : a.epoch;
    if (a.ktimer && threadIdx.x == 0)
        atomicMin((unsigned long long *)&a.ktimer[0], (unsigned long long)wall_clock64());
    const int q0 = a.wg_off[blockIdx.x], q1 = a.wg_off[blockIdx.x + 1];
    for (int q = q0; q < q1; ++q) {
        const int pid = a.wg_list[q];
        const PackDesc pk = a.packs[pid];
        uint64_t tstart = 0;
        if (a.pack_time && threadIdx.x == 0) tstart = wall_clock64();
        // two call sites, so that in the common one the state pointer is
        // visibly derived from the shared array and its accesses compile to
        // LDS instructions rather than generic (flat) ones
        if (!kRes && pk.global_mem)
            run_pack<T, kSolve, kRes>(a, pk, smem,
                                      a.scratch + (int64_t)(pk.global_mem - 1) * a.scratch_stride,
                                      epoch);
        else
            run_pack<T, kSolve, kRes>(a, pk, smem, smem + pk.tbytes, epoch);
        __syncthreads();
        if (a.pack_time && threadIdx.x == 0)
            atomicAdd((unsigned long long *)&a.pack_time[pid],
                      (unsigned long long)(wall_clock64() - tstart));
    }
    // The launch's span, from the first workgroup's start to the last one's
    // end: every workgroup raises the end mark before it counts itself
    // done, so the last to count sees the final marks, adds the span to the
    // class total and re-arms the timer for the next launch (which the
    // stream orders after this one).
    if (a.ktimer && threadIdx.x == 0) {
        unsigned long long *kt = (unsigned long long *)a.ktimer;
        atomicMax(&kt[1], (unsigned long long)wall_clock64());
        __threadfence();
        if (atomicAdd(&kt[2], 1ull) == (unsigned long long)gridDim.x - 1) {
            __threadfence();
            const unsigned long long t0 = atomicAdd(&kt[0], 0ull), t1 = atomicAdd(&kt[1], 0ull);
            atomicAdd(&kt[4], t1 - t0);
            atomicAdd(&kt[5], 1ull);
            atomicExch(&kt[0], ~0ull);
            atomicExch(&kt[1], 0ull);
            atomicExch(&kt[2], 0ull);
        }
    }
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Marks the start of a size-class launch in its timer: runs just before the
// launch on the same stream, so the launch's span also covers any wait for
// resources held by a concurrent launch (as a dispatch-level trace counts it).
__global__ void k_stamp(uint64_t *timer) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        atomicMin((unsigned long long *)&timer[0], (unsigned long long)wall_clock64());
}

__global__ void k_advance(int64_t *epoch) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *epoch = *epoch + 1;
}

template <typename T>
__global__ void k_convert(const double *w, T *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (T)w[i];
}

}  // namespace

hipError_t launch_setup(const SetupArgs &a, int precision, hipStream_t s) {
    const int nt = 128;
    const int nb = (a.n_neurons + nt - 1) / nt;
    if (precision == 0)
        hipLaunchKernelGGL(k_setup<double>, dim3(nb > 0 ? nb : 1), dim3(nt), 0, s, a);
    else
        hipLaunchKernelGGL(k_setup<float>, dim3(nb > 0 ? nb : 1), dim3(nt), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_epoch(const EpochArgs &a, int precision, int solver, int n_wg, int threads,
                        size_t lds_bytes, bool resident, hipStream_t s) {
    const dim3 g(n_wg), b(threads);
    if (precision == 0) {
        if (solver == 0)
            hipLaunchKernelGGL((k_epoch<double, 0>), g, b, lds_bytes, s, a);
        else if (solver == 1)
            hipLaunchKernelGGL((k_epoch<double, 1>), g, b, lds_bytes, s, a);
        else
            hipLaunchKernelGGL((k_epoch<double, 2>), g, b, lds_bytes, s, a);
    } else {
        if (solver == 0)
            hipLaunchKernelGGL((k_epoch<float, 0>), g, b, lds_bytes, s, a);
        else if (solver == 1)
            hipLaunchKernelGGL((k_epoch<float, 1>), g, b, lds_bytes, s, a);
        else if (resident)
            hipLaunchKernelGGL((k_epoch<float, 2, true>), g, b, lds_bytes, s, a);
        else
            hipLaunchKernelGGL((k_epoch<float, 2>), g, b, lds_bytes, s, a);
    }
    return hipGetLastError();
}

hipError_t set_epoch_lds_limit(int bytes) {
    const void *fns[] = {(const void *)k_epoch<double, 0>, (const void *)k_epoch<double, 1>,
                         (const void *)k_epoch<double, 2>, (const void *)k_epoch<float, 0>,
                         (const void *)k_epoch<float, 1>, (const void *)k_epoch<float, 2>,
                         (const void *)k_epoch<float, 2, true>};
    for (const void *f : fns) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

#ifdef MMH_PHASE_PROFILE
extern "C" int mmh_phase_ticks(unsigned long long *out, int reset) {
    if (hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase_ticks), sizeof(unsigned long long) * 8) !=
        hipSuccess)
        return -1;
    if (reset) {
        unsigned long long z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_phase_ticks), z, sizeof z) != hipSuccess) return -1;
    }
    return 0;
}
#endif

hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_stamp(uint64_t *timer, hipStream_t s) {
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, timer);
    return hipGetLastError();
}

hipError_t launch_advance(int64_t *epoch, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, epoch);
    return hipGetLastError();
}

hipError_t launch_decay_weights_convert(const double *w, void *out, int64_t n, int precision,
                                        hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (precision == 0)
        hipLaunchKernelGGL(k_convert<double>, dim3((unsigned)nb), dim3(256), 0, s, w,
                           (double *)out, n);
    else
        hipLaunchKernelGGL(k_convert<float>, dim3((unsigned)nb), dim3(256), 0, s, w,
                           (float *)out, n);
    return hipGetLastError();
}

}  // namespace mmh
