"""Pins of the CPU oracle against what mathematics and the paper fix.

Every test here checks the oracle against something other than itself: a
dense LU solve, closed-form solutions of the discrete and continuum cable,
an exact conservation law, closed forms of the gate dynamics, special values
of the rate functions, libm, and textbook constants. Each is chosen so that a
plausible slip (a dropped term, a wrong sign, a swapped operand, a wrong unit
factor) fails at least one of them.
"""
import itertools
import math
import os

import numpy as np
import pytest

from paper_2005_06332_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ulp_diff64(a, b):
    a = np.asarray(a, np.float64).view(np.int64)
    b = np.asarray(b, np.float64).view(np.int64)
    return np.abs(a - b)


def ulp_diff32(a, b):
    a = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(a - b)


def chain_problem(n, diam=1.0, length=10.0, iext=0.0, mech=0, dt=0.025,
                  parent=None, lengths=None, diams=None, precision=0):
    """One neuron, no synapses. parent defaults to an unbranched chain."""
    if parent is None:
        parent = np.arange(-1, n - 1, dtype=np.int32)
    prob = dict(
        name="test", seed=0, n_steps=0,
        n_comp=np.array([n], np.int32), comp_off=np.array([0, n], np.int64),
        parent=np.asarray(parent, np.int32),
        length_um=np.full(n, length) if lengths is None else np.asarray(lengths, float),
        diam_um=np.full(n, diam) if diams is None else np.asarray(diams, float),
        mech=np.full(n, mech, np.uint8), detector=np.zeros(1, np.int32),
        iext_nA=np.array([iext]),
        syn_pre=np.zeros(0, np.int32), syn_post=np.zeros(0, np.int32),
        syn_comp=np.zeros(0, np.int32), syn_delay=np.zeros(0, np.int32),
        syn_w=np.zeros(0),
        params=W.default_params(precision), channels=dict(W.CHANNELS))
    prob["params"]["dt"] = dt
    return prob


# ---------------------------------------------------------------------------
# exp / exprelr against libm
# ---------------------------------------------------------------------------

def test_exp_double_within_two_ulp_of_libm(orc):
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(-700, 700, 2000), rng.uniform(-30, 30, 3000),
                         [0.0, 1.0, -1.0, 0.5 * math.log(2), -0.5 * math.log(2)]])
    got = np.array([orc.exp_d(x) for x in xs])
    ref = np.exp(xs)
    assert ulp_diff64(got, ref).max() <= 2
    assert orc.exp_d(0.0) == 1.0


def test_exp_float_within_two_ulp_of_correctly_rounded(orc):
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-87, 88, 2000), rng.uniform(-20, 20, 3000)]).astype(np.float32)
    got = np.array([orc.exp_f(x) for x in xs], np.float32)
    ref = np.exp(xs.astype(np.float64)).astype(np.float32)
    assert ulp_diff32(got, ref).max() <= 2


def test_exprelr_against_expm1(orc):
    rng = np.random.default_rng(2)
    us = np.concatenate([rng.uniform(-1, 1, 2000), rng.uniform(-30, 30, 2000),
                         [1e-12, -1e-12, 0.4999, 0.5, -0.5, 0.5001]])
    got = np.array([orc.exprelr_d(u) for u in us])
    ref = np.array([u / math.expm1(u) for u in us])
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 2e-15
    assert orc.exprelr_d(0.0) == 1.0
    gotf = np.array([orc.exprelr_f(u) for u in us.astype(np.float32)], np.float32)
    reff = np.array([float(np.float32(u)) / math.expm1(float(np.float32(u)))
                     for u in us], np.float64)
    assert np.max(np.abs(gotf - reff) / np.abs(reff)) < 4e-7


# ---------------------------------------------------------------------------
# Hodgkin-Huxley rates and gates
# ---------------------------------------------------------------------------

def hh_rates_libm(v):
    am = 0.1 * (v + 40) / (1 - math.exp(-(v + 40) / 10)) if v != -40 else 1.0
    bm = 4 * math.exp(-(v + 65) / 18)
    ah = 0.07 * math.exp(-(v + 65) / 20)
    bh = 1 / (1 + math.exp(-(v + 35) / 10))
    an = 0.01 * (v + 55) / (1 - math.exp(-(v + 55) / 10)) if v != -55 else 0.1
    bn = 0.125 * math.exp(-(v + 65) / 80)
    return np.array([am, bm, ah, bh, an, bn])


@pytest.mark.parametrize("v", [-90.0, -65.0, -54.3, -40.5, -20.0, 0.0, 35.0])
def test_rates_match_hh_closed_forms(orc, v):
    assert np.allclose(orc.rates(v, 0), hh_rates_libm(v), rtol=1e-13, atol=0)
    assert np.allclose(orc.rates(v, 1), hh_rates_libm(float(np.float32(v))), rtol=2e-6, atol=0)


def test_rates_removable_singularities(orc):
    # alpha_m -> 1 at -40 mV and alpha_n -> 0.1 at -55 mV (limits of x/(1-e^-x))
    assert orc.rates(-40.0, 0)[0] == 1.0
    assert orc.rates(-55.0, 0)[4] == pytest.approx(0.1, rel=1e-15)
    assert orc.rates(-40.0, 1)[0] == np.float32(1.0)
    eps = 1e-7
    assert orc.rates(-40.0 + eps, 0)[0] == pytest.approx(1.0 + eps / 20, rel=1e-12)


def test_resting_gates_match_textbook_values(orc):
    r = orc.rates(-65.0, 0)
    inf = dict(m_inf=r[0] / (r[0] + r[1]), h_inf=r[2] / (r[2] + r[3]),
               n_inf=r[4] / (r[4] + r[5]))
    for line in open(os.path.join(GOLDEN, "hh_resting_gates.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, val, tol = line.split()
        assert abs(inf[name] - float(val)) <= float(tol), name


@pytest.mark.parametrize("v", [-70.0, -65.0, -40.0, -10.0, 20.0])
def test_gates_under_voltage_clamp_follow_closed_form(orc, v):
    dt, nsteps = 0.025, 200
    a = hh_rates_libm(v)
    x0 = (0.1, 0.7, 0.25)
    x = x0
    for _ in range(nsteps):
        x = orc.gates_update(v, dt, *x)
    for g in range(3):
        s = a[2 * g] + a[2 * g + 1]
        xinf = a[2 * g] / s
        ref = xinf + (x0[g] - xinf) * math.exp(-nsteps * dt * s)
        assert x[g] == pytest.approx(ref, rel=1e-12, abs=1e-14)
    xf = tuple(np.float32(c) for c in x0)
    for _ in range(nsteps):
        xf = orc.gates_update(v, dt, *xf, precision=1)
    for g in range(3):
        s = a[2 * g] + a[2 * g + 1]
        xinf = a[2 * g] / s
        ref = xinf + (x0[g] - xinf) * math.exp(-nsteps * dt * s)
        assert float(xf[g]) == pytest.approx(ref, rel=2e-5, abs=2e-6)


def test_isolated_hh_compartment_rests_near_minus_65(orc):
    prob = chain_problem(1, diam=20.0, length=20.0, mech=1)
    s = orc.Sim(prob, max_steps=20000)
    s.step(20000)
    v = s.voltages()[0]
    assert -65.2 < v < -64.8
    assert len(s.spikes()) == 0


def hh_space_clamped_spike_times(j_uA_cm2, t_end):
    """Upward 0 mV crossings of the space-clamped HH membrane (Eq. 1 with no
    axial term) under a constant current density, integrated by scipy's LSODA
    at tight tolerance. Conductances in S/cm^2 times mV give mA/cm^2, hence
    the factor 1e3 against uA/cm^2 and uF/cm^2."""
    from scipy.integrate import solve_ivp
    ch = W.CHANNELS

    def rhs(t, y):
        v, m, h, n = y
        a = hh_rates_libm(v)
        i_ion = (ch["gnabar"] * m ** 3 * h * (v - ch["ena"]) + ch["gkbar"] * n ** 4 * (v - ch["ek"])
                 + ch["gl"] * (v - ch["el"]))
        return [(j_uA_cm2 - 1e3 * i_ion) / ch["cm"],
                a[0] * (1 - m) - a[1] * m, a[2] * (1 - h) - a[3] * h, a[4] * (1 - n) - a[5] * n]

    def crossing(t, y):
        return y[0]
    crossing.direction = 1
    a = hh_rates_libm(-65.0)
    y0 = [-65.0, a[0] / (a[0] + a[1]), a[2] / (a[2] + a[3]), a[4] / (a[4] + a[5])]
    sol = solve_ivp(rhs, (0.0, t_end), y0, method="LSODA", rtol=1e-10, atol=1e-12,
                    events=crossing)
    return sol.t_events[0]


def test_driven_hh_compartment_converges_to_the_hh_ode(orc):
    """A single HH compartment driven by 10 uA/cm^2 fires repetitively (about
    68 Hz, the classic HH result). The oracle's spike times converge at first
    order in dt to an independent high-accuracy ODE solution: this pins the
    current assembly (signs, reversal potentials, units, area scaling of the
    injected current) and the gate update order inside the time loop."""
    j, t_end, d = 10.0, 50.0, 20.0
    area_cm2 = math.pi * d * d * 1e-8
    ref = hh_space_clamped_spike_times(j, t_end)
    assert len(ref) == 4
    isi = np.diff(ref)
    assert np.all((isi > 14.0) & (isi < 15.2))
    errs = []
    for dt in (0.025, 0.0125, 0.00625):
        prob = chain_problem(1, diam=d, length=d, mech=1, iext=j * area_cm2 * 1e3, dt=dt)
        n = int(round(t_end / dt))
        s = orc.Sim(prob, max_steps=n)
        s.step(n)
        t_sp = s.spikes()[:, 1] * dt
        s.close()
        assert len(t_sp) == len(ref)
        err = t_sp - ref
        # detection reports the step that crosses, so each time lies at most
        # one step late on top of the scheme's O(dt) error
        assert np.all(np.abs(err) <= 10 * dt)
        errs.append(np.abs(err).max())
    for coarse, fine in zip(errs, errs[1:]):
        assert 1.6 < coarse / fine < 2.6
    # the FP32-gating mode crosses at the same steps, give or take one
    prob = chain_problem(1, diam=d, length=d, mech=1, iext=j * area_cm2 * 1e3, dt=0.025,
                         precision=1)
    s = orc.Sim(prob, max_steps=2000)
    s.step(2000)
    steps32 = s.spikes()[:, 1]
    s.close()
    prob = chain_problem(1, diam=d, length=d, mech=1, iext=j * area_cm2 * 1e3, dt=0.025)
    s = orc.Sim(prob, max_steps=2000)
    s.step(2000)
    steps64 = s.spikes()[:, 1]
    s.close()
    assert len(steps32) == len(steps64) == 4
    assert np.all(np.abs(steps32 - steps64) <= 1)


@pytest.mark.parametrize("precision", [0, 1])
def test_active_cable_converges_to_its_method_of_lines_ode(orc, precision):
    """An unbranched HH cable (40 compartments of 20 um x 2 um, sealed ends,
    0.2 nA into compartment 0) launches an action potential that propagates to
    the far end. The semi-discrete equations (Eq. 1 per compartment: capacitive
    current = axial currents to the neighbours through pi d^2 / (4 Ra L) +
    injected - ionic current, with the gate ODEs) are integrated by scipy's
    LSODA. The oracle's crossing times at both ends converge to them at first
    order in dt, which pins the axial coupling together with the active
    membrane."""
    from scipy.integrate import solve_ivp
    ch = W.CHANNELS
    n_c, d, L, i0, t_end = 40, 2.0, 20.0, 0.2, 12.0
    area = math.pi * d * L * 1e-8                                   # cm^2
    g_ax = math.pi * (d * 1e-4) ** 2 / (4 * ch["ra"] * L * 1e-4) * 1e6  # uS
    c_n = ch["cm"] * area * 1e3                                     # nF

    def rates(v):
        um, un = -(v + 40) / 10, -(v + 55) / 10
        with np.errstate(invalid="ignore", divide="ignore"):
            am = np.where(um == 0, 1.0, 0.1 * (v + 40) / (1 - np.exp(um)))
            an = np.where(un == 0, 0.1, 0.01 * (v + 55) / (1 - np.exp(un)))
        return (am, 4 * np.exp(-(v + 65) / 18), 0.07 * np.exp(-(v + 65) / 20),
                1 / (1 + np.exp(-(v + 35) / 10)), an, 0.125 * np.exp(-(v + 65) / 80))

    def rhs(t, y):
        v, m, h, n = y.reshape(4, n_c)
        am, bm, ah, bh, an, bn = rates(v)
        # S/cm^2 * mV * cm^2 = mA, times 1e6 for nA
        i_ion = 1e6 * area * (ch["gnabar"] * m ** 3 * h * (v - ch["ena"])
                              + ch["gkbar"] * n ** 4 * (v - ch["ek"]) + ch["gl"] * (v - ch["el"]))
        i_ax = np.zeros(n_c)
        i_ax[:-1] += g_ax * (v[1:] - v[:-1])
        i_ax[1:] += g_ax * (v[:-1] - v[1:])
        i_ax[0] += i0
        return np.concatenate([(i_ax - i_ion) / c_n, am * (1 - m) - bm * m,
                               ah * (1 - h) - bh * h, an * (1 - n) - bn * n])

    def near(t, y):
        return y[0]

    def far(t, y):
        return y[n_c - 1]
    near.direction = far.direction = 1
    r = rates(np.array(-65.0))
    y0 = np.concatenate([np.full(n_c, -65.0)] + [np.full(n_c, r[k] / (r[k] + r[k + 1]))
                                                 for k in (0, 2, 4)])
    sol = solve_ivp(rhs, (0.0, t_end), y0, method="LSODA", rtol=1e-9, atol=1e-10,
                    events=[near, far])
    assert len(sol.t_events[0]) == len(sol.t_events[1]) == 1
    ref = np.array([sol.t_events[0][0], sol.t_events[1][0]])
    assert 1.0 < ref[1] - ref[0] < 1.6   # about 0.6 m/s over 780 um

    errs = []
    for dt in (0.025, 0.0125, 0.00625):
        prob = chain_problem(n_c, diam=d, length=L, mech=1, iext=i0, dt=dt, precision=precision)
        steps = int(round(t_end / dt))
        s = orc.Sim(prob, max_steps=steps)
        prev, t_far = s.voltages()[-1], []
        for k in range(steps):
            s.step(1)
            v = s.voltages()[-1]
            if prev < 0.0 <= v:
                t_far.append((k + 1) * dt)
            prev = v
        t_near = s.spikes()[:, 1] * dt
        s.close()
        assert len(t_near) == len(t_far) == 1
        err = np.abs(np.array([t_near[0], t_far[0]]) - ref)
        assert np.all(err <= 3 * dt)
        errs.append(err[1])
    for coarse, fine in zip(errs, errs[1:]):
        assert 1.6 < coarse / fine < 2.6


# ---------------------------------------------------------------------------
# Algorithm 1 against dense Gaussian elimination
# ---------------------------------------------------------------------------

def all_hines_parents(n):
    """Every parent vector with p[0] = -1 and 0 <= p[i] < i."""
    return itertools.product(*[range(i) for i in range(1, n)])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_hines_solve_equals_dense_lu_on_every_tree(orc, n):
    rng = np.random.default_rng(n)
    worst = 0.0
    for tail in all_hines_parents(n):
        p = np.array((-1,) + tail, np.int32)
        a = rng.uniform(-1, 0, n)       # upper: A[p(i), i]
        c = rng.uniform(-1, 0, n)       # lower: A[i, p(i)]  (unsymmetric on purpose)
        b = rng.uniform(0.5, 1.5, n) + 3.0
        rhs = rng.normal(size=n)
        A = np.diag(b.copy())
        for i in range(1, n):
            A[p[i], i] = a[i]
            A[i, p[i]] = c[i]
        x = orc.hines_solve(p, a, b, c, rhs)
        ref = np.linalg.solve(A, rhs)
        worst = max(worst, np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
    assert worst < 1e-13


def test_hines_solve_random_large_trees(orc):
    rng = np.random.default_rng(7)
    for n in (40, 200):
        p = np.array([-1] + [rng.integers(0, i) for i in range(1, n)], np.int32)
        a, c = rng.uniform(-1, 0, n), rng.uniform(-1, 0, n)
        deg = np.zeros(n)
        for i in range(1, n):
            deg[i] += 1
            deg[p[i]] += 1
        b = deg + rng.uniform(0.1, 1.0, n)
        rhs = rng.normal(size=n)
        A = np.diag(b.copy())
        for i in range(1, n):
            A[p[i], i], A[i, p[i]] = a[i], c[i]
        x = orc.hines_solve(p, a, b, c, rhs)
        assert np.allclose(x, np.linalg.solve(A, rhs), rtol=0, atol=1e-12 * np.abs(x).max())


def test_assembled_matrix_is_a_hines_matrix(orc):
    """Symmetric, nonzero diagonal, one off-diagonal pair per parent link,
    strictly diagonally dominant (so Algorithm 1 needs no pivoting)."""
    for prob in (W.config1(), W.mini()):
        s = orc.Sim(prob, max_steps=1)
        cst = s.consts()
        off = prob["comp_off"]
        for j in range(0, prob["n_comp"].shape[0], 7):
            b0, n = off[j], off[j + 1] - off[j]
            p = prob["parent"][b0:b0 + n]
            e = cst["e"][b0:b0 + n]
            d = s.assembled_diag(j)
            A = np.diag(d)
            for i in range(1, n):
                A[p[i], i] = e[i]
                A[i, p[i]] = e[i]
            assert np.array_equal(A, A.T)
            assert np.all(d != 0)
            assert np.all(e[1:] < 0)
            off_sum = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
            assert np.all(np.diag(A) > off_sum)
            # exactly one nonzero per parent link in each triangle
            assert np.count_nonzero(np.triu(A, 1)) == n - 1
        s.close()


# ---------------------------------------------------------------------------
# Cable closed forms
# ---------------------------------------------------------------------------

def test_sealed_cable_steady_state_matches_discrete_closed_form(orc):
    """Uniform passive sealed cable, current I0 into compartment 0. The
    fixed point of the scheme solves G(V_{k-1}-2V_k+V_{k+1}) = g_m (V_k - E)
    with sealed ends, whose solution is V_k - E = A cosh(kappa (k - N + 1/2)),
    cosh(kappa) = 1 + g_m/(2G)."""
    N, d, L, I0 = 20, 1.0, 10.0, 0.05
    ch = W.CHANNELS
    prob = chain_problem(N, diam=d, length=L, iext=I0, mech=0)
    s = orc.Sim(prob, max_steps=14000)
    s.step(14000)
    v = s.voltages()
    # physical units: membrane conductance of a compartment (uS) and the
    # coupling of two equal compartments through two half-resistances (uS)
    area_cm2 = math.pi * d * L * 1e-8
    g_m = ch["g_pas"] * area_cm2 * 1e6
    R_ohm = ch["ra"] * (L * 1e-4) / (math.pi * (d * 1e-4) ** 2 / 4)
    G = 1e6 / R_ohm
    kappa = math.acosh(1 + g_m / (2 * G))
    A = I0 / ((g_m + G) * math.cosh(kappa * (N - 0.5)) - G * math.cosh(kappa * (N - 1.5)))
    k = np.arange(N)
    ref = ch["e_pas"] + A * np.cosh(kappa * (k - N + 0.5))
    assert np.max(np.abs(v - ref)) < 1e-10


def continuum_error(orc, N):
    ell, d, I0 = 1000.0, 2.0, 0.02
    ch = W.CHANNELS
    dx = ell / N
    prob = chain_problem(N, diam=d, length=dx, iext=I0, mech=0)
    s = orc.Sim(prob, max_steps=16000)
    s.step(16000)
    v = s.voltages()
    Rm = 1.0 / ch["g_pas"]                       # Ohm cm^2
    lam = math.sqrt((d * 1e-4) * Rm / (4 * ch["ra"]))  # cm
    r_a = 4 * ch["ra"] / (math.pi * (d * 1e-4) ** 2)   # Ohm/cm
    x = (np.arange(N) + 0.5) * dx * 1e-4          # cm
    ref_mV = I0 * 1e-9 * r_a * lam * np.cosh((ell * 1e-4 - x) / lam) / math.sinh(ell * 1e-4 / lam) * 1e3
    return np.max(np.abs((v - ch["e_pas"]) - ref_mV))


def test_cable_converges_to_continuum_at_second_order(orc):
    """Sealed finite cable with point injection at x=0:
    V(x) - E = I0 r_a lambda cosh((l-x)/lambda) / sinh(l/lambda)."""
    errs = [continuum_error(orc, N) for N in (25, 50, 100)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-2
    for o in orders:
        assert 1.9 < o < 2.1, (errs, orders)


@pytest.mark.parametrize("theta,order", [(0.5, 2.0), (1.0, 1.0)])
def test_axial_time_stepping_order(orc, theta, order):
    """With no membrane conductance the step is the theta-method on the
    cable's linear axial system C dV/dt = -K V: Crank-Nicolson (theta = 1/2,
    the factor 2 of Eq. 2) is second order in dt, backward Euler (theta = 1)
    first order. The reference is the exact solution exp(-C^-1 K t) V0 of the
    semi-discrete system, with K built from the geometry."""
    from scipy.linalg import expm
    ch = W.CHANNELS
    n, d, L, t_end = 30, 2.0, 20.0, 2.0
    g_ax = math.pi * (d * 1e-4) ** 2 / (4 * ch["ra"] * L * 1e-4) * 1e6   # uS
    c_n = ch["cm"] * math.pi * d * L * 1e-8 * 1e3                        # nF
    K = np.zeros((n, n))
    for i in range(1, n):
        K[i, i] += g_ax
        K[i - 1, i - 1] += g_ax
        K[i, i - 1] -= g_ax
        K[i - 1, i] -= g_ax
    x = (np.arange(n) + 0.5) / n
    v0 = ch["e_pas"] + 10.0 * np.cos(math.pi * x) + 5.0 * np.cos(2 * math.pi * x)
    ref = ch["e_pas"] + expm(-K / c_n * t_end) @ (v0 - ch["e_pas"])
    errs = []
    for dt in (0.05, 0.025, 0.0125):
        prob = chain_problem(n, diam=d, length=L, mech=0, dt=dt)
        prob["channels"]["g_pas"] = 0.0
        prob["params"]["theta"] = theta
        s = orc.Sim(prob, max_steps=200)
        s.set_voltages(v0)
        s.step(int(round(t_end / dt)))
        errs.append(np.max(np.abs(s.voltages() - ref)))
        s.close()
    for coarse, fine in zip(errs, errs[1:]):
        assert abs(math.log2(coarse / fine) - order) < 0.05, errs


def diameter_step_error(orc, k):
    """Passive sealed cable of 600 um at 2 um, then 400 um at 1 um, current
    into the first compartment. Max deviation (mV) of the steady state from
    the continuum solution with V and axial current continuous at the step."""
    ch = W.CHANNELS
    l0, l1, d0, d1, i0 = 600.0, 400.0, 2.0, 1.0, 0.02
    n0, n1 = 12 * k, 8 * k
    prob = chain_problem(n0 + n1, mech=0, iext=i0,
                         lengths=np.concatenate([np.full(n0, l0 / n0), np.full(n1, l1 / n1)]),
                         diams=np.concatenate([np.full(n0, d0), np.full(n1, d1)]))
    s = orc.Sim(prob, max_steps=16000)
    s.step(16000)
    v = s.voltages() - ch["e_pas"]
    s.close()
    rm = 1.0 / ch["g_pas"]

    def lam(d):
        return math.sqrt(d * 1e-4 * rm / (4 * ch["ra"]))

    def r_a(d):
        return 4 * ch["ra"] / (math.pi * (d * 1e-4) ** 2)
    x_0, x_1 = l0 * 1e-4 / lam(d0), l1 * 1e-4 / lam(d1)
    # daughter: B cosh(x_1 - y); parent: P cosh(x_0 - x) + Q sinh(x_0 - x), with
    # P = B cosh(x_1) (V continuous), Q = B sinh(x_1) r_a0 lam0 / (r_a1 lam1)
    # (current continuous) and the injected current fixing the scale at x = 0
    k1 = math.sinh(x_1) * r_a(d0) * lam(d0) / (r_a(d1) * lam(d1))
    b = i0 * 1e-9 * r_a(d0) * lam(d0) * 1e3 / (math.cosh(x_1) * math.sinh(x_0)
                                                + k1 * math.cosh(x_0))
    xs = (np.arange(n0) + 0.5) * (l0 / n0) * 1e-4 / lam(d0)
    ys = (np.arange(n1) + 0.5) * (l1 / n1) * 1e-4 / lam(d1)
    ref = np.concatenate([b * math.cosh(x_1) * np.cosh(x_0 - xs) + b * k1 * np.sinh(x_0 - xs),
                          b * np.cosh(x_1 - ys)])
    return np.max(np.abs(v - ref))


def test_diameter_step_converges_at_second_order(orc):
    """Across a change of diameter the two half-compartment resistances in
    series carry the axial current exactly, so the scheme keeps its second
    order: a wrong diameter or length in either half would not."""
    errs = [diameter_step_error(orc, k) for k in (2, 4, 8)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-4
    for o in orders:
        assert 1.9 < o < 2.1, (errs, orders)


def rall_tree_error(orc, k):
    """Passive parent cylinder (600 um, d0 = 2 um) forking into two identical
    daughters (400 um) whose diameters obey Rall's 3/2 power rule, current
    into the parent's first compartment. Max deviation (mV) of the oracle's
    steady state from the equivalent-cylinder solution at compartment
    centres."""
    ch = W.CHANNELS
    l0, l1, d0, i0 = 600.0, 400.0, 2.0, 0.02
    d1 = d0 * 2 ** (-2 / 3)                     # d0^(3/2) = 2 d1^(3/2)
    n0, n1 = 12 * k, 8 * k
    n = n0 + 2 * n1
    parent = np.empty(n, np.int32)
    parent[0] = -1
    parent[1:n0] = np.arange(n0 - 1)
    for b in range(2):
        s0 = n0 + b * n1
        parent[s0] = n0 - 1
        parent[s0 + 1:s0 + n1] = np.arange(s0, s0 + n1 - 1)
    prob = chain_problem(n, parent=parent, mech=0, iext=i0,
                         lengths=np.concatenate([np.full(n0, l0 / n0), np.full(2 * n1, l1 / n1)]),
                         diams=np.concatenate([np.full(n0, d0), np.full(2 * n1, d1)]))
    s = orc.Sim(prob, max_steps=16000)
    s.step(16000)
    v = s.voltages() - ch["e_pas"]
    s.close()
    rm = 1.0 / ch["g_pas"]
    lam0 = math.sqrt(d0 * 1e-4 * rm / (4 * ch["ra"]))
    lam1 = math.sqrt(d1 * 1e-4 * rm / (4 * ch["ra"]))
    r_a0 = 4 * ch["ra"] / (math.pi * (d0 * 1e-4) ** 2)
    big_x = l0 * 1e-4 / lam0 + l1 * 1e-4 / lam1    # electrotonic length of the equivalent cylinder
    x0 = (np.arange(n0) + 0.5) * (l0 / n0) * 1e-4 / lam0
    x1 = l0 * 1e-4 / lam0 + (np.arange(n1) + 0.5) * (l1 / n1) * 1e-4 / lam1
    amp = i0 * 1e-9 * r_a0 * lam0 / math.sinh(big_x) * 1e3
    ref = amp * np.cosh(big_x - np.concatenate([x0, x1, x1]))
    assert np.array_equal(v[n0:n0 + n1], v[n0 + n1:])   # the two daughters are one solution
    return np.max(np.abs(v - ref)), ref[0]


def test_branched_tree_converges_to_rall_equivalent_cylinder(orc):
    """A fork whose daughters obey the 3/2 power rule behaves, in the
    continuum, like one cylinder of the parent's diameter (Rall). The
    discrete steady state converges to it as the compartments shrink. The
    convergence is first order: each daughter couples to the parent's centre
    through its own half-resistance plus the parent's, so the parent's last
    half-compartment is counted once per daughter, an O(h) junction error
    (unbranched cables converge at second order)."""
    errs, v0 = zip(*[rall_tree_error(orc, k) for k in (2, 4, 8)])
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-3 * v0[-1]
    for o in orders:
        assert 0.9 < o < 1.2, (errs, orders)


def test_leak_decay_invariant_on_random_tree(orc):
    """Leak only, uniform g/cm: the axial terms cancel in the row sums, so
    sum_i C_i (V_i^{n+1} - E) = sum_i C_i (V_i^n - E) / (1 + dt g/cm)."""
    base = W.mini(n_neurons=3)
    rng = np.random.default_rng(3)
    for j in range(3):
        off = base["comp_off"]
        n = int(off[j + 1] - off[j])
        sl = slice(off[j], off[j + 1])
        prob = chain_problem(n, parent=base["parent"][sl], lengths=base["length_um"][sl],
                             diams=base["diam_um"][sl], mech=0)
        s = orc.Sim(prob, max_steps=3)
        E = W.CHANNELS["e_pas"]
        v0 = E + rng.normal(scale=10.0, size=n)
        s.set_voltages(v0)
        s.step(1)
        v1 = s.voltages()
        w = math.pi * prob["diam_um"] * prob["length_um"]   # C_i is proportional to area
        mu = prob["params"]["dt"] * W.CHANNELS["g_pas"] / (W.CHANNELS["cm"] * 1e-3)
        lhs = np.sum(w * (v1 - E))
        rhs = np.sum(w * (v0 - E)) / (1 + mu)
        assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(w * (v0 - E)))
        # a uniform voltage stays uniform
        s.set_voltages(np.full(n, -30.0))
        s.step(1)
        v2 = s.voltages()
        assert np.ptp(v2) < 1e-12
        assert v2[0] == pytest.approx(E + (-30.0 - E) / (1 + mu), rel=1e-13)
        s.close()


def test_single_compartment_is_implicit_euler_of_rc(orc):
    """n = 1: the solve is one division; with a leak and a constant current
    V_{n} - V_inf = (V_0 - V_inf) (1 + dt g/C)^-n, V_inf = E + I/g."""
    d, L, I0, dt = 5.0, 7.0, 0.003, 0.025
    prob = chain_problem(1, diam=d, length=L, iext=I0, mech=0, dt=dt)
    s = orc.Sim(prob, max_steps=500)
    area_cm2 = math.pi * d * L * 1e-8
    g = W.CHANNELS["g_pas"] * area_cm2 * 1e6          # uS
    Cn = W.CHANNELS["cm"] * area_cm2 * 1e3            # nF
    vinf = W.CHANNELS["e_pas"] + I0 / g
    v0 = W.CHANNELS["e_pas"]
    for n in (1, 10, 500):
        s.step(n - s.step_count)
        ref = vinf + (v0 - vinf) * (1 + dt * g / Cn) ** (-n)
        assert s.voltages()[0] == pytest.approx(ref, rel=1e-13)


# ---------------------------------------------------------------------------
# Synapses, delays and detection
# ---------------------------------------------------------------------------

def two_neuron_chain(delay, w, iext0=2.0):
    prob = chain_problem(1, diam=20.0, length=20.0, mech=1, iext=iext0)
    one = {k: prob[k] for k in prob}
    two = dict(prob)
    two.update(n_comp=np.array([1, 1], np.int32), comp_off=np.array([0, 1, 2], np.int64),
               parent=np.array([-1, -1], np.int32), length_um=np.array([20.0, 20.0]),
               diam_um=np.array([20.0, 20.0]), mech=np.array([1, 1], np.uint8),
               detector=np.zeros(2, np.int32), iext_nA=np.array([iext0, 0.0]),
               syn_pre=np.array([0], np.int32), syn_post=np.array([1], np.int32),
               syn_comp=np.array([0], np.int32), syn_delay=np.array([delay], np.int32),
               syn_w=np.array([w]))
    del one
    return two


def test_single_event_conductance_is_w_q_power_k(orc):
    delay, w = 40, 0.004
    prob = two_neuron_chain(delay, w)
    s = orc.Sim(prob, max_steps=2000)
    gs = []
    for _ in range(1000):
        s.step(1)
        gs.append(s.g()[0])
    gs = np.array(gs)
    spk = s.spikes()
    s0 = int(spk[spk[:, 0] == 0][0, 1])          # first spike of neuron 0
    q = math.exp(-prob["params"]["dt"] / prob["params"]["tau_syn"])
    assert s.q == pytest.approx(q, rel=1e-15)
    # gs[k] is g after k+1 completed steps. The event arrives in the step
    # that starts at step count s0 + delay and is decayed at its end.
    first = s0 + delay
    assert np.all(gs[:first] == 0.0)
    nxt = spk[spk[:, 0] == 0]
    stop = int(nxt[1, 1]) + delay if len(nxt) > 1 else len(gs)
    for k in range(0, min(200, stop - first)):
        assert gs[first + k] == pytest.approx(w * q ** (k + 1), rel=(k + 2) * 2.3e-16)


def test_conductances_superpose_events_across_delays(orc):
    """Several synapses onto one passive compartment, fed from a replay
    raster: two of them share a presynaptic neuron with different delays,
    one receives two events, and two events land in the same step. Each
    synapse's conductance must equal the superposition of w q^(k+1) over its
    events (linear first-order decay, Section 2), and nothing may arrive
    before its delay."""
    prob = chain_problem(1, diam=10.0, length=10.0, mech=0)
    pre = np.array([0, 1, 0, 2], np.int32)
    delay = np.array([40, 45, 100, 41], np.int32)
    w = np.array([0.003, 0.002, 0.001, 0.0025])
    prob.update(syn_pre=pre, syn_post=np.zeros(4, np.int32), syn_comp=np.zeros(4, np.int32),
                syn_delay=delay, syn_w=w)
    steps = 300
    raster = np.zeros((steps + 1, 3), np.uint8)
    fired = {0: [5, 9], 1: [4], 2: [8]}   # synapses 0, 1 and 3 all deliver at step 49
    for j, ts in fired.items():
        raster[ts, j] = 1
    s = orc.Sim(prob, max_steps=steps)
    s.set_input_raster(raster)
    q = s.q
    gs = []
    for _ in range(steps):
        s.step(1)
        gs.append(s.g())
    s.close()
    gs = np.array(gs)
    for k in range(4):
        arrivals = [t + int(delay[k]) for t in fired[int(pre[k])]]
        for m in range(steps):
            want = sum(w[k] * q ** (m - a + 1) for a in arrivals if m >= a)
            if want == 0.0:
                assert gs[m, k] == 0.0, (k, m)
            else:
                assert gs[m, k] == pytest.approx(want, rel=1e-13), (k, m)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("e_syn", [0.0, -80.0])
def test_postsynaptic_potential_converges_to_the_conductance_ode(orc, e_syn, precision):
    """One event onto a passive compartment (replay raster, spike at 1 ms,
    delay 2 ms). The membrane sees the conductance-based synaptic current
    g(t) (V - E_syn) with g(t) = w exp(-(t - t_a)/tau) from the arrival t_a on
    (Section 2): an EPSP of about 12 mV for E_syn = 0, an IPSP for -80 mV.
    The oracle's voltage converges at first order in dt to scipy's LSODA
    solution of C dV/dt = -g_pas A (V - E_pas) - g(t) (V - E_syn)."""
    from scipy.integrate import solve_ivp
    ch = W.CHANNELS
    d, w, t_spk, t_del, t_end = 10.0, 0.0005, 1.0, 2.0, 30.0
    tau = W.default_params()["tau_syn"]
    area_cm2 = math.pi * d * d * 1e-8
    g_m = ch["g_pas"] * area_cm2 * 1e6     # uS
    c_n = ch["cm"] * area_cm2 * 1e3        # nF
    t_a = t_spk + t_del

    def rhs(t, y):
        g = w * math.exp(-(t - t_a) / tau)
        return [(-g_m * (y[0] - ch["e_pas"]) - g * (y[0] - e_syn)) / c_n]
    ts = np.arange(4.0, t_end + 1e-9, 1.0)
    ref = solve_ivp(rhs, (t_a, t_end), [ch["e_pas"]], method="LSODA", rtol=1e-11, atol=1e-12,
                    t_eval=ts, first_step=1e-6).y[0]
    if e_syn == 0.0:
        assert 11.0 < ref.max() - ch["e_pas"] < 13.5
    else:
        assert -3.5 < ref.min() - ch["e_pas"] < -2.0
    errs = []
    for dt in (0.025, 0.0125, 0.00625):
        prob = chain_problem(1, diam=d, length=d, mech=0, dt=dt, precision=precision)
        prob["params"]["e_syn"] = e_syn
        prob.update(syn_pre=np.array([0], np.int32), syn_post=np.zeros(1, np.int32),
                    syn_comp=np.zeros(1, np.int32),
                    syn_delay=np.array([round(t_del / dt)], np.int32), syn_w=np.array([w]))
        steps = int(round(t_end / dt))
        raster = np.zeros((steps + 1, 1), np.uint8)
        raster[round(t_spk / dt), 0] = 1
        s = orc.Sim(prob, max_steps=steps)
        s.set_input_raster(raster)
        v = []
        for t in ts:
            s.step(int(round(t / dt)) - s.step_count)
            v.append(s.voltages()[0])
        s.close()
        errs.append(np.max(np.abs(np.array(v) - ref)))
        assert errs[-1] < 2.0 * dt
    for coarse, fine in zip(errs, errs[1:]):
        assert 1.8 < coarse / fine < 2.2


def test_spike_is_an_upward_threshold_crossing(orc):
    prob = two_neuron_chain(40, 0.0, iext0=0.25)   # ~20 uA/cm2: repetitive firing
    s = orc.Sim(prob, max_steps=3000)
    v = [s.voltages()[0]]
    for _ in range(2000):
        s.step(1)
        v.append(s.voltages()[0])
    v = np.array(v)
    th = prob["params"]["v_thresh"]
    crossings = np.where((v[:-1] < th) & (v[1:] >= th))[0] + 1
    spk = s.spikes()
    assert len(crossings) >= 2
    assert np.array_equal(spk[spk[:, 0] == 0][:, 1], crossings)


def test_threads_do_not_change_results(orc, monkeypatch):
    """Neurons are independent within a step: the parallel neuron loop of the
    oracle gives bitwise the same network trajectory with one thread as with
    several, and as in any other neuron order."""
    prob = W.mini(n_steps=120)
    n0 = orc.num_threads()
    try:
        orc.set_num_threads(1)
        v_one, s_one = orc.run(prob)
        orc.set_num_threads(8)
        v1, s1 = orc.run(prob)
    finally:
        orc.set_num_threads(n0)
    assert np.array_equal(v_one, v1) and np.array_equal(s_one, s1)
    # permuting neurons must give the same per-neuron results
    perm = np.random.default_rng(5).permutation(prob["n_comp"].shape[0])
    sub = W.subset(prob, perm)
    v2, s2 = orc.run(sub)
    off1, off2 = prob["comp_off"], sub["comp_off"]
    for new, old in enumerate(perm):
        assert np.array_equal(v2[off2[new]:off2[new + 1]], v1[off1[old]:off1[old + 1]])
    inv = np.argsort(perm)
    assert sorted(map(tuple, s1.tolist())) == sorted((int(perm[a]), int(b)) for a, b in s2.tolist())
    assert len(s1) > 0 and inv.shape == perm.shape


def test_replay_of_recorded_spikes_reproduces_the_network(orc):
    """Per-neuron replay: the oracle runs a few neurons of a network, fed
    with the network's recorded spikes instead of its own; their voltages
    and spikes must equal those of the full run exactly (the mechanism the
    full-length GPU check relies on)."""
    from paper_2005_06332_amd import workload as W
    prob = W.mini(seed=41, n_neurons=40, n_steps=240)
    steps = 240
    full = orc.Sim(prob, max_steps=steps)
    full.step(steps)
    v_full, s_full = full.voltages(), full.spikes()
    full.close()
    assert len(s_full) > 0
    targets = np.array([3, 17, 0, 29, 38])
    sub = W.replay_subset(prob, targets)
    rep = orc.Sim(sub, max_steps=steps)
    rep.set_input_raster(W.spike_raster(s_full, prob["n_comp"].shape[0], steps))
    rep.step(steps)
    v_rep, s_rep = rep.voltages(), rep.spikes()
    rep.close()
    off = prob["comp_off"]
    want = np.concatenate([v_full[off[j]:off[j + 1]] for j in targets])
    assert np.array_equal(v_rep, want)
    want_sp = sorted((int(np.where(targets == n)[0][0]), int(t))
                     for n, t in s_full if n in set(targets.tolist()))
    assert sorted(map(tuple, s_rep.tolist())) == want_sp
