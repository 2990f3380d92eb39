"""ctypes binding of libmmhines.so (the C ABI in include/sim.h).

Argument marshalling only: every step of the simulation runs in the HIP
library. Importing this module loads the library; it raises if the library
has not been built, and the library itself refuses to run without a gfx950
GPU. There is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MMHINES_LIB") or os.path.join(HERE, "libmmhines.so")

SIM_OK, SIM_EINVAL, SIM_ENOMEM, SIM_EDEVICE, SIM_ESTATE = 0, -1, -2, -3, -4
FP64, FP32_GATING = 0, 1
SOLVE_EXACT, SOLVE_FAST, SOLVE_CONTRACT = 0, 1, 2
PACK_PLAIN, PACK_COUNT, PACK_LEARNED = 0, 1, 2
SCHED_AUTO, SCHED_PERSISTENT, SCHED_DISPATCH = 0, 1, 2
N_FEATURES = 16

EXPORTS = (
    "sim_default_params", "sim_create", "sim_step", "sim_time_steps",
    "sim_read_voltages", "sim_read_gates", "sim_read_conductances",
    "sim_spikes", "sim_neuron_timings", "sim_features",
    "sim_set_kernel_timing", "sim_kernel_time", "sim_class_time", "sim_config_string",
    "sim_destroy", "sim_last_error", "sim_mlp_nparams", "sim_mlp_init",
    "sim_mlp_forward", "sim_mlp_loss_grad", "sim_mlp_train",
    "sim_plan_create", "sim_pack_count", "sim_pack_info", "sim_pack_neurons",
    "sim_class_launch", "sim_workgroup_packs", "sim_contraction_schedule",
    "sim_pack_contraction_items", "sim_step_noalloc",
)


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("dt_ms", C.c_double), ("theta", C.c_double), ("tau_syn_ms", C.c_double),
        ("e_syn_mV", C.c_double), ("v_thresh_mV", C.c_double), ("v_init_mV", C.c_double),
        ("precision", C.c_int32), ("solver", C.c_int32), ("packing", C.c_int32),
        ("sched", C.c_int32),
        ("epoch_steps", C.c_int32), ("autotune", C.c_int32), ("threads", C.c_int32),
        ("pack_comps", C.c_int32), ("lds_comps", C.c_int32), ("lds_classes", C.c_int32),
        ("use_graph", C.c_int32),
        ("record_timings", C.c_int32), ("cost_model", C.c_void_p), ("hip_stream", C.c_void_p),
        ("neuron_cost", C.c_void_p),
    ]


class Morphology(C.Structure):
    _fields_ = [
        ("n_neurons", C.c_int32), ("comp_offset", C.c_void_p), ("parent", C.c_void_p),
        ("length_um", C.c_void_p), ("diam_um", C.c_void_p), ("mech", C.c_void_p),
        ("detector", C.c_void_p), ("i_ext_nA", C.c_void_p),
    ]


class Channels(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "cm_uF_cm2", "ra_ohm_cm", "gnabar", "gkbar", "gl", "ena", "ek", "el",
        "g_pas", "e_pas")]


class Synapses(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("pre", C.c_void_p), ("post", C.c_void_p),
        ("post_comp", C.c_void_p), ("delay_steps", C.c_void_p), ("weight_uS", C.c_void_p),
    ]


class PackInfo(C.Structure):
    _fields_ = [
        ("first_position", C.c_int32), ("n_neurons", C.c_int32), ("n_comp", C.c_int32),
        ("n_syn", C.c_int32), ("n_branches", C.c_int32), ("size_class", C.c_int32),
        ("in_global", C.c_int32), ("n_rounds", C.c_int32), ("n_levels", C.c_int32),
        ("n_child_entries", C.c_int32), ("table_bytes", C.c_int64),
        ("state_bytes", C.c_int64), ("cost", C.c_double),
        ("n_wide_rounds", C.c_int32), ("n_staged_items", C.c_int32),
    ]


class Spike(C.Structure):
    _fields_ = [("neuron", C.c_int32), ("step", C.c_int32)]


_lib = None


def lib():
    """Load libmmhines.so (built by paper_2005_06332_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2005_06332_amd/build.py "
                              "(or __graft_entry__.build()) first")
        # One HIP runtime per process. torch ships its own copy of the HIP
        # and ROCr runtimes under the same sonames the library depends on;
        # loaded after torch, the library binds to torch's copy, so streams
        # and device pointers from torch are valid in it. Loaded before
        # torch, the process would end up with two runtimes, and whichever
        # initialises second can find no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.sim_default_params.argtypes = [C.POINTER(Params)]
        L.sim_create.argtypes = [C.POINTER(Params), C.POINTER(Morphology), C.POINTER(Channels),
                                 C.POINTER(Synapses), C.POINTER(C.c_void_p)]
        L.sim_create.restype = C.c_int
        L.sim_step.argtypes = [P, C.c_int64]
        L.sim_step.restype = C.c_int
        L.sim_time_steps.argtypes = [P]
        L.sim_time_steps.restype = C.c_int64
        L.sim_read_voltages.argtypes = [P, P, C.c_int64]
        L.sim_read_gates.argtypes = [P, P, P, P, C.c_int64]
        L.sim_read_conductances.argtypes = [P, P, C.c_int64]
        L.sim_spikes.argtypes = [P, P, C.c_int64, C.POINTER(C.c_int64)]
        L.sim_neuron_timings.argtypes = [P, P, C.c_int64, C.c_int32]
        L.sim_features.argtypes = [P, P, C.c_int64]
        L.sim_set_kernel_timing.argtypes = [P, C.c_int32]
        L.sim_kernel_time.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.sim_class_time.argtypes = [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.sim_config_string.argtypes = [P]
        L.sim_config_string.restype = C.c_char_p
        L.sim_destroy.argtypes = [P]
        L.sim_destroy.restype = None
        L.sim_last_error.argtypes = [P]
        L.sim_last_error.restype = C.c_char_p
        L.sim_plan_create.argtypes = [C.POINTER(Params), C.POINTER(Morphology),
                                      C.POINTER(Channels), C.POINTER(Synapses), C.c_int32,
                                      C.c_int32, C.POINTER(C.c_void_p)]
        L.sim_pack_count.argtypes = [P]
        L.sim_pack_count.restype = C.c_int32
        L.sim_pack_info.argtypes = [P, C.c_int32, C.POINTER(PackInfo)]
        L.sim_pack_neurons.argtypes = [P, C.c_int32, P, C.c_int64]
        L.sim_class_launch.argtypes = [P, C.c_int32, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.sim_workgroup_packs.argtypes = [P, C.c_int32, C.c_int32, P, C.c_int64,
                                          C.POINTER(C.c_int32)]
        L.sim_contraction_schedule.argtypes = [P, C.c_int32, P, C.c_int64, P, C.c_int64,
                                               C.POINTER(C.c_int32)]
        L.sim_pack_contraction_items.argtypes = [P, C.c_int32, P, C.c_int64,
                                                 C.POINTER(C.c_int64)]
        L.sim_step_noalloc.argtypes = [P, C.c_int64, P, C.c_int64, C.POINTER(C.c_int64)]
        L.sim_step_noalloc.restype = C.c_int
        L.sim_mlp_nparams.restype = C.c_int64
        L.sim_mlp_init.argtypes = [P, P, P, C.c_int64, C.c_uint64]
        L.sim_mlp_forward.argtypes = [P, P, C.c_int64, P]
        L.sim_mlp_loss_grad.argtypes = [P, P, P, C.c_int64, P, P]
        L.sim_mlp_train.argtypes = [P, P, P, C.c_int64, C.c_int32, C.c_float, P]
        for f in ("sim_read_voltages", "sim_read_gates", "sim_read_conductances", "sim_spikes",
                  "sim_neuron_timings", "sim_features", "sim_set_kernel_timing",
                  "sim_kernel_time", "sim_class_time", "sim_mlp_init", "sim_mlp_forward",
                  "sim_mlp_loss_grad", "sim_mlp_train", "sim_plan_create", "sim_pack_info",
                  "sim_pack_neurons", "sim_class_launch", "sim_workgroup_packs",
                  "sim_contraction_schedule", "sim_pack_contraction_items"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, handle=None):
    if rc != SIM_OK:
        msg = lib().sim_last_error(handle)
        raise SimError(rc, msg.decode() if msg else "")


def default_params() -> Params:
    p = Params()
    lib().sim_default_params(C.byref(p))
    return p


class Simulation:
    """One network on the GPU. ``prob`` is a workload problem dictionary."""

    def __init__(self, prob: dict, precision: int | None = None, packing: int = PACK_COUNT,
                 sched: int = SCHED_AUTO, autotune: bool = False, threads: int = 0,
                 pack_comps: int = 0, lds_comps: int = 0, use_graph: bool = True,
                 record_timings: bool = False, cost_model: np.ndarray | None = None,
                 epoch_steps: int = 0, stream: int | None = None, solver: int | None = None,
                 lds_classes: int = 0, plan: tuple | None = None,
                 neuron_cost: np.ndarray | None = None):
        """plan = (lds_bytes_per_cu, n_cu): lay the problem out on the host
        only (sim_plan_create), for the introspection calls. neuron_cost:
        per-neuron costs that learned packing uses in place of a model's
        predictions."""
        L = lib()
        pr = prob["params"]
        ch = prob["channels"]
        P = default_params()
        P.dt_ms, P.theta, P.tau_syn_ms = pr["dt"], pr["theta"], pr["tau_syn"]
        P.e_syn_mV, P.v_thresh_mV, P.v_init_mV = pr["e_syn"], pr["v_thresh"], pr["v_init"]
        P.precision = int(pr["precision"] if precision is None else precision)
        if solver is not None:
            P.solver = int(solver)
        P.packing, P.sched, P.autotune = packing, sched, int(autotune)
        P.threads, P.pack_comps, P.lds_comps = threads, pack_comps, lds_comps
        P.lds_classes = lds_classes
        P.use_graph, P.record_timings, P.epoch_steps = int(use_graph), int(record_timings), epoch_steps
        self._cm = None
        if cost_model is not None:
            self._cm = np.ascontiguousarray(cost_model, np.float32)
            P.cost_model = self._cm.ctypes.data
        P.hip_stream = stream
        self._nc = None
        if neuron_cost is not None:
            self._nc = np.ascontiguousarray(neuron_cost, np.float64)
            P.neuron_cost = self._nc.ctypes.data
        self.precision = P.precision
        keep = {k: np.ascontiguousarray(prob[k]) for k in (
            "comp_off", "parent", "length_um", "diam_um", "mech", "detector", "iext_nA",
            "syn_pre", "syn_post", "syn_comp", "syn_delay", "syn_w")}
        assert keep["comp_off"].dtype == np.int64 and keep["parent"].dtype == np.int32
        assert keep["length_um"].dtype == np.float64 and keep["mech"].dtype == np.uint8
        for k in ("syn_pre", "syn_post", "syn_comp", "syn_delay", "detector"):
            keep[k] = keep[k].astype(np.int32, copy=False)
        self.N = int(prob["n_comp"].shape[0])
        self.C = int(keep["comp_off"][-1])
        self.S = int(keep["syn_pre"].shape[0])
        M = Morphology(self.N, _p(keep["comp_off"]), _p(keep["parent"]), _p(keep["length_um"]),
                       _p(keep["diam_um"]), _p(keep["mech"]), _p(keep["detector"]),
                       _p(keep["iext_nA"]))
        CH = Channels(ch["cm"], ch["ra"], ch["gnabar"], ch["gkbar"], ch["gl"], ch["ena"],
                      ch["ek"], ch["el"], ch["g_pas"], ch["e_pas"])
        SY = Synapses(self.S, _p(keep["syn_pre"]), _p(keep["syn_post"]), _p(keep["syn_comp"]),
                      _p(keep["syn_delay"]), _p(keep["syn_w"]))
        h = C.c_void_p()
        if plan is None:
            rc = L.sim_create(C.byref(P), C.byref(M), C.byref(CH), C.byref(SY), C.byref(h))
        else:
            rc = L.sim_plan_create(C.byref(P), C.byref(M), C.byref(CH), C.byref(SY),
                                   int(plan[0]), int(plan[1]), C.byref(h))
        _check(rc, None)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def config(self) -> str:
        return lib().sim_config_string(self._h).decode()

    @property
    def step_count(self) -> int:
        return lib().sim_time_steps(self._h)

    def step(self, n: int) -> None:
        _check(lib().sim_step(self._h, int(n)), self._h)

    def step_noalloc(self, n: int, cap: int | None = None) -> np.ndarray:
        """sim_step_noalloc: n steps without any allocation by the library;
        returns this call's spikes (neuron, step) as int64 [k, 2]. The buffer
        is allocated here, by the caller, before the call."""
        if cap is None:
            cap = self.N * max(int(n), 1)
        buf = (Spike * max(cap, 1))()
        cnt = C.c_int64(0)
        _check(lib().sim_step_noalloc(self._h, int(n), C.cast(buf, C.c_void_p), int(cap),
                                      C.byref(cnt)), self._h)
        k = cnt.value
        return np.frombuffer(buf, dtype=np.int32, count=2 * k).reshape(k, 2).astype(np.int64)

    def voltages(self) -> np.ndarray:
        out = np.empty(self.C, np.float64)
        _check(lib().sim_read_voltages(self._h, _p(out), self.C), self._h)
        return out

    def gates(self):
        m, h, n = (np.empty(self.C, np.float64) for _ in range(3))
        _check(lib().sim_read_gates(self._h, _p(m), _p(h), _p(n), self.C), self._h)
        return m, h, n

    def conductances(self) -> np.ndarray:
        out = np.empty(max(self.S, 1), np.float64)
        _check(lib().sim_read_conductances(self._h, _p(out), max(self.S, 1)), self._h)
        return out[:self.S]

    def spikes(self) -> np.ndarray:
        """(neuron, step) pairs sorted by step then neuron, int64 [n, 2]."""
        tot = C.c_int64(0)
        _check(lib().sim_spikes(self._h, None, 0, C.byref(tot)), self._h)
        n = tot.value
        buf = (Spike * max(n, 1))()
        _check(lib().sim_spikes(self._h, C.cast(buf, C.c_void_p), n, C.byref(tot)), self._h)
        arr = np.frombuffer(buf, dtype=np.int32, count=2 * n).reshape(n, 2)
        return arr.astype(np.int64)

    def neuron_timings(self, reset: bool = False) -> np.ndarray:
        out = np.empty(self.N, np.float64)
        _check(lib().sim_neuron_timings(self._h, _p(out), self.N, int(reset)), self._h)
        return out

    def features(self) -> np.ndarray:
        out = np.empty((self.N, N_FEATURES), np.float32)
        _check(lib().sim_features(self._h, _p(out), out.size), self._h)
        return out

    # ---- layout introspection --------------------------------------------

    def pack_count(self) -> int:
        return int(lib().sim_pack_count(self._h))

    def pack_info(self, pack: int) -> dict:
        info = PackInfo()
        _check(lib().sim_pack_info(self._h, int(pack), C.byref(info)), self._h)
        return {name: getattr(info, name) for name, _ in PackInfo._fields_}

    def pack_neurons(self, pack: int) -> np.ndarray:
        n = self.pack_info(pack)["n_neurons"]
        out = np.empty(n, np.int32)
        _check(lib().sim_pack_neurons(self._h, int(pack), _p(out), n), self._h)
        return out

    def class_launch(self, cls: int):
        """(workgroups, threads, LDS bytes) of size class cls."""
        n, t, b = C.c_int32(0), C.c_int32(0), C.c_int64(0)
        _check(lib().sim_class_launch(self._h, int(cls), C.byref(n), C.byref(t), C.byref(b)),
               self._h)
        return n.value, t.value, b.value

    def workgroup_packs(self, cls: int, wg: int) -> np.ndarray:
        n = C.c_int32(0)
        _check(lib().sim_workgroup_packs(self._h, int(cls), int(wg), None, 0, C.byref(n)),
               self._h)
        out = np.empty(n.value, np.int32)
        _check(lib().sim_workgroup_packs(self._h, int(cls), int(wg), _p(out), out.size,
                                         C.byref(n)), self._h)
        return out

    def contraction_schedule(self, neuron: int, n_comp: int):
        """(items [n_comp, 4] = (k, n1, n2, flags), round offsets); flags bit 0:
        n1 is k's parent, bits 1 and 2: k's coupling to n1 / n2 was made by an
        earlier elimination."""
        nr = C.c_int32(0)
        _check(lib().sim_contraction_schedule(self._h, int(neuron), None, 0, None, 0,
                                              C.byref(nr)), self._h)
        items = np.empty((n_comp, 4), np.int32)
        ro = np.empty(nr.value + 1, np.int32)
        _check(lib().sim_contraction_schedule(self._h, int(neuron), _p(items), items.size,
                                              _p(ro), ro.size, C.byref(nr)), self._h)
        return items, ro

    def pack_contraction_items(self, pack: int) -> np.ndarray:
        """The pack's contraction items as the epoch kernel reads them (a
        planned layout under the contraction solver; see
        sim_pack_contraction_items)."""
        n = C.c_int64(0)
        _check(lib().sim_pack_contraction_items(self._h, int(pack), None, 0, C.byref(n)), self._h)
        out = np.empty(n.value, np.uint64)
        _check(lib().sim_pack_contraction_items(self._h, int(pack), _p(out), out.size,
                                                C.byref(n)), self._h)
        return out

    def set_kernel_timing(self, on: bool) -> None:
        _check(lib().sim_set_kernel_timing(self._h, int(on)), self._h)

    def kernel_time(self):
        """(total ms, count) of the timed epochs."""
        ms, n = C.c_double(0), C.c_int64(0)
        _check(lib().sim_kernel_time(self._h, C.byref(ms), C.byref(n)), self._h)
        return ms.value, n.value

    def class_time(self, cls: int):
        """(total ms, launches, compartments per step, compartment-updates) of
        size class cls over the timed launches."""
        ms, n, c, u = C.c_double(0), C.c_int64(0), C.c_int64(0), C.c_int64(0)
        _check(lib().sim_class_time(self._h, cls, C.byref(ms), C.byref(n), C.byref(c),
                                    C.byref(u)), self._h)
        return ms.value, n.value, c.value, u.value


# ---- cost model ---------------------------------------------------------------

def mlp_nparams() -> int:
    return int(lib().sim_mlp_nparams())


def mlp_init(x: np.ndarray, y: np.ndarray, seed: int = 1234) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    p = np.zeros(mlp_nparams(), np.float32)
    _check(lib().sim_mlp_init(_p(p), _p(x), _p(y), x.shape[0], seed))
    return p


def mlp_forward(params: np.ndarray, x: np.ndarray) -> np.ndarray:
    params = np.ascontiguousarray(params, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    out = np.empty(x.shape[0], np.float32)
    _check(lib().sim_mlp_forward(_p(params), _p(x), x.shape[0], _p(out)))
    return out


def mlp_loss_grad(params: np.ndarray, x: np.ndarray, y: np.ndarray):
    params = np.ascontiguousarray(params, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    loss = np.zeros(1, np.float32)
    grad = np.zeros_like(params)
    _check(lib().sim_mlp_loss_grad(_p(params), _p(x), _p(y), x.shape[0], _p(loss), _p(grad)))
    return float(loss[0]), grad


def mlp_train(params: np.ndarray, x: np.ndarray, y: np.ndarray, epochs: int = 500,
              lr: float = 3e-3):
    p = np.array(params, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    loss = np.zeros(1, np.float32)
    _check(lib().sim_mlp_train(_p(p), _p(x), _p(y), x.shape[0], int(epochs), float(lr), _p(loss)))
    return p, float(loss[0])
