"""ctypes wrapper of the CPU oracle (hines_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg are the only callers. Nothing in the GPU library
imports or links this module, and this module imports nothing from the
library; both receive their inputs as plain arrays from the workload
generator.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hines_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math", "-fno-builtin-rint"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "dt", "theta", "tau_syn", "e_syn", "v_thresh", "v_init", "cm", "ra",
        "gnabar", "gkbar", "gl", "ena", "ek", "el", "g_pas", "e_pas")] + [
        ("precision", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_exp_d.restype = C.c_double
        L.orc_exp_d.argtypes = [C.c_double]
        L.orc_exp_f.restype = C.c_float
        L.orc_exp_f.argtypes = [C.c_float]
        L.orc_exprelr_d.restype = C.c_double
        L.orc_exprelr_d.argtypes = [C.c_double]
        L.orc_exprelr_f.restype = C.c_float
        L.orc_exprelr_f.argtypes = [C.c_float]
        L.orc_rates_d.argtypes = [C.c_double, P]
        L.orc_rates_f.argtypes = [C.c_float, P]
        L.orc_tree_solve.argtypes = [C.c_int32, P, P, P, P, P, P]
        L.orc_gates_update_d.argtypes = [C.c_double, C.c_double, P, P, P]
        L.orc_gates_update_f.argtypes = [C.c_float, C.c_float, P, P, P]
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Params), C.c_int32, P, P, P, P, P,
                                 P, P, C.c_int64, P, P, P, P, P, C.c_int64]
        L.orc_destroy.argtypes = [P]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [P, C.c_int64]
        L.orc_n_comp.restype = C.c_int64
        L.orc_n_comp.argtypes = [P]
        L.orc_cur_step.restype = C.c_int64
        L.orc_cur_step.argtypes = [P]
        for f in ("orc_get_v", "orc_set_v", "orc_get_g", "orc_get_spikes"):
            getattr(L, f).argtypes = [P, P]
        L.orc_get_gates.argtypes = [P, P, P, P]
        L.orc_get_consts.argtypes = [P, P, P, P, P]
        L.orc_assemble_diag.argtypes = [P, C.c_int32, P]
        L.orc_n_spikes.restype = C.c_int64
        L.orc_n_spikes.argtypes = [P]
        L.orc_q.restype = C.c_double
        L.orc_q.argtypes = [P]
        L.orc_set_input_raster.restype = C.c_int
        L.orc_set_input_raster.argtypes = [P, C.c_int32, C.c_int64, P]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---- scalar functions -------------------------------------------------------

def exp_d(x: float) -> float:
    return lib().orc_exp_d(float(x))


def exp_f(x) -> np.float32:
    return np.float32(lib().orc_exp_f(float(np.float32(x))))


def exprelr_d(u: float) -> float:
    return lib().orc_exprelr_d(float(u))


def exprelr_f(u) -> np.float32:
    return np.float32(lib().orc_exprelr_f(float(np.float32(u))))


def rates(v: float, precision: int = 0) -> np.ndarray:
    """(alpha_m, beta_m, alpha_h, beta_h, alpha_n, beta_n) at v."""
    if precision == 0:
        out = np.zeros(6, np.float64)
        lib().orc_rates_d(float(v), _ptr(out))
    else:
        out = np.zeros(6, np.float32)
        lib().orc_rates_f(float(np.float32(v)), _ptr(out))
    return out


def gates_update(v, dt, m, h, n, precision: int = 0):
    """One exponential-Euler step of (m, h, n) at voltage v."""
    if precision == 0:
        x = [np.array([m], np.float64), np.array([h], np.float64), np.array([n], np.float64)]
        lib().orc_gates_update_d(float(v), float(dt), *(_ptr(a) for a in x))
    else:
        x = [np.array([m], np.float32), np.array([h], np.float32), np.array([n], np.float32)]
        lib().orc_gates_update_f(float(np.float32(v)), float(np.float32(dt)), *(_ptr(a) for a in x))
    return tuple(a[0] for a in x)


def hines_solve(p, a, b, c, rhs) -> np.ndarray:
    """Tree solve (the method of Algorithm 1) of the matrix with diagonal b,
    a[i] = A[p[i], i] and c[i] = A[i, p[i]]; returns x."""
    p = np.ascontiguousarray(p, np.int32)
    a = np.ascontiguousarray(a, np.float64)
    b = np.array(b, np.float64)
    c = np.ascontiguousarray(c, np.float64)
    r = np.array(rhs, np.float64)
    lib().orc_tree_solve(len(r), _ptr(p), _ptr(a), _ptr(b), _ptr(c), _ptr(r), _ptr(r))
    return r


# ---- network ------------------------------------------------------------------

class Sim:
    """The reference simulation of a workload problem dictionary."""

    def __init__(self, prob: dict, max_steps: int | None = None,
                 precision: int | None = None):
        L = lib()
        pr = dict(prob["params"])
        ch = prob["channels"]
        if precision is not None:
            pr["precision"] = precision
        self.precision = int(pr["precision"])
        P = _Params(dt=pr["dt"], theta=pr["theta"], tau_syn=pr["tau_syn"],
                    e_syn=pr["e_syn"], v_thresh=pr["v_thresh"],
                    v_init=pr["v_init"], cm=ch["cm"], ra=ch["ra"],
                    gnabar=ch["gnabar"], gkbar=ch["gkbar"], gl=ch["gl"],
                    ena=ch["ena"], ek=ch["ek"], el=ch["el"], g_pas=ch["g_pas"],
                    e_pas=ch["e_pas"], precision=self.precision)
        self._keep = {k: np.ascontiguousarray(prob[k]) for k in (
            "comp_off", "parent", "length_um", "diam_um", "mech", "detector",
            "iext_nA", "syn_pre", "syn_post", "syn_comp", "syn_delay", "syn_w")}
        k = self._keep
        assert k["comp_off"].dtype == np.int64 and k["parent"].dtype == np.int32
        self.N = int(prob["n_comp"].shape[0])
        self.C = int(k["comp_off"][-1])
        self.S = int(k["syn_pre"].shape[0])
        if max_steps is None:
            max_steps = int(prob.get("n_steps", 1000))
        self.max_steps = int(max_steps)
        self._h = L.orc_create(C.byref(P), self.N, _ptr(k["comp_off"]),
                               _ptr(k["parent"]), _ptr(k["length_um"]),
                               _ptr(k["diam_um"]), _ptr(k["mech"]),
                               _ptr(k["detector"]), _ptr(k["iext_nA"]),
                               self.S, _ptr(k["syn_pre"]), _ptr(k["syn_post"]),
                               _ptr(k["syn_comp"]), _ptr(k["syn_delay"]),
                               _ptr(k["syn_w"]), self.max_steps)
        if not self._h:
            raise MemoryError("oracle allocation failed")

    def set_input_raster(self, raster: np.ndarray):
        """Replay mode: presynaptic spikes come from ``raster`` (uint8
        [(steps+1), N_network], raster[s, j] = 1 when neuron j spiked at step
        s) instead of this simulation's own spikes; synapse pre ids index
        that network."""
        r = np.ascontiguousarray(raster, np.uint8)
        self._raster = r
        if lib().orc_set_input_raster(self._h, r.shape[1], r.shape[0] - 1, _ptr(r)) != 0:
            raise ValueError("bad replay raster")

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def step_count(self) -> int:
        return lib().orc_cur_step(self._h)

    def step(self, n: int = 1) -> None:
        rc = lib().orc_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError(f"orc_step failed ({rc}); history capacity {self.max_steps}")

    def voltages(self) -> np.ndarray:
        out = np.empty(self.C, np.float64)
        lib().orc_get_v(self._h, _ptr(out))
        return out

    def set_voltages(self, v: np.ndarray) -> None:
        v = np.ascontiguousarray(v, np.float64)
        lib().orc_set_v(self._h, _ptr(v))

    def gates(self):
        m, h, n = (np.empty(self.C, np.float64) for _ in range(3))
        lib().orc_get_gates(self._h, _ptr(m), _ptr(h), _ptr(n))
        return m, h, n

    def g(self) -> np.ndarray:
        out = np.empty(self.S, np.float64)
        lib().orc_get_g(self._h, _ptr(out))
        return out

    def spikes(self) -> np.ndarray:
        """(neuron, step) pairs sorted by step, then neuron."""
        n = lib().orc_n_spikes(self._h)
        out = np.empty((n, 2), np.int64)
        if n:
            lib().orc_get_spikes(self._h, _ptr(out))
        return out

    def consts(self):
        cdt, G, e, af = (np.empty(self.C, np.float64) for _ in range(4))
        lib().orc_get_consts(self._h, _ptr(cdt), _ptr(G), _ptr(e), _ptr(af))
        return dict(cdt=cdt, G=G, e=e, af=af)

    def assembled_diag(self, j: int) -> np.ndarray:
        n = int(self._keep["comp_off"][j + 1] - self._keep["comp_off"][j])
        out = np.empty(n, np.float64)
        lib().orc_assemble_diag(self._h, int(j), _ptr(out))
        return out

    @property
    def q(self) -> float:
        return lib().orc_q(self._h)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of the simulations created from now on."""
    lib().orc_set_num_threads(int(n))


def run(prob: dict, n_steps: int | None = None, precision: int | None = None):
    """Run a problem for n_steps; returns (V, spikes)."""
    n = int(prob["n_steps"] if n_steps is None else n_steps)
    s = Sim(prob, max_steps=n, precision=precision)
    s.step(n)
    v, spk = s.voltages(), s.spikes()
    s.close()
    return v, spk
