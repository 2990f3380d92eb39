"""The C ABI without a GPU: the built library loads, exports every function
include/sim.h declares (and the binding binds exactly those), and the
host-side checks of sim_create reject bad problems before touching a device.
No simulation runs here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2005_06332_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sim.h")
DECL = re.compile(r"^(?:const\s+)?[a-z0-9_]+[\s*]+(sim_[a-z0-9_]+)\s*\(", re.M)


def declared():
    with open(HEADER) as f:
        return sorted(set(DECL.findall(f.read())))


@pytest.fixture(scope="module")
def S():
    from paper_2005_06332_amd import sim
    sim.lib()
    return sim


def test_header_declares_the_boundary():
    names = declared()
    for must in ("sim_create", "sim_step", "sim_read_voltages", "sim_spikes", "sim_destroy",
                 "sim_mlp_forward", "sim_mlp_loss_grad", "sim_mlp_train", "sim_class_time"):
        assert must in names


def test_library_exports_every_declared_function(S):
    lib = C.CDLL(S.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_binds_exactly_the_header(S):
    assert sorted(S.EXPORTS) == declared()


def test_defaults_and_sizes_without_device(S):
    p = S.default_params()
    assert p.dt_ms == 0.025 and p.theta == 0.5 and p.tau_syn_ms == 2.0
    assert p.precision == S.FP32_GATING and p.solver == S.SOLVE_EXACT
    assert p.packing == S.PACK_COUNT and p.use_graph == 1
    from oracle import mlp_ref
    assert S.mlp_nparams() == mlp_ref.NP


def _bad(prob, key, fn):
    bad = dict(prob)
    bad[key] = fn(np.array(prob[key]))
    return bad


@pytest.mark.parametrize("case", [
    "delay_zero", "parent_forward", "detector_range", "syn_comp_range", "bad_precision",
    "bad_solver", "bad_threads", "epoch_too_long", "nan_length",
])
def test_validation_rejects_before_device(S, case):
    prob = W.mini(n_neurons=12, n_steps=40)
    kw = {}
    if case == "delay_zero":
        prob = _bad(prob, "syn_delay", lambda a: np.where(np.arange(a.size) == 0, 0, a))
    elif case == "parent_forward":
        def f(a):
            a = a.copy()
            a[int(prob["comp_off"][0]) + 3] = 5  # parent not before the child
            return a
        prob = _bad(prob, "parent", f)
    elif case == "detector_range":
        prob = _bad(prob, "detector", lambda a: a + 100000)
    elif case == "syn_comp_range":
        prob = _bad(prob, "syn_comp", lambda a: a + 100000)
    elif case == "bad_precision":
        kw["precision"] = 7
    elif case == "bad_solver":
        kw["solver"] = 5
    elif case == "bad_threads":
        kw["threads"] = 100
    elif case == "epoch_too_long":
        kw["epoch_steps"] = int(prob["syn_delay"].min()) + 1
    elif case == "nan_length":
        prob = _bad(prob, "length_um", lambda a: np.where(np.arange(a.size) == 2, np.nan, a))
    with pytest.raises(S.SimError) as e:
        S.Simulation(prob, **kw)
    assert e.value.code == S.SIM_EINVAL, str(e.value)


def test_valid_problem_without_gpu_reports_no_device(S):
    """A valid problem passes validation and then stops at the device check
    (this test only runs where no GPU is visible)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(S.SimError) as e:
        S.Simulation(W.mini(n_neurons=8, n_steps=40))
    assert e.value.code == S.SIM_EDEVICE


def test_failure_text_is_per_thread(S):
    """Failures without a handle keep their text per calling thread: two
    threads failing sim_create for different reasons each read their own."""
    import threading
    prob = W.mini(n_neurons=12, n_steps=40)
    cases = [(dict(threads=100), "threads must be"), (dict(solver=5), "unknown solver")]
    bad = []

    def worker(kw, want):
        for _ in range(200):
            try:
                S.Simulation(prob, **kw)
            except S.SimError as e:
                if want not in str(e):
                    bad.append(str(e))
            else:
                bad.append("no error")

    ts = [threading.Thread(target=worker, args=c) for c in cases]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not bad, bad[:3]


def test_one_hip_runtime_per_process():
    """Loading the library and then torch leaves a single HIP runtime (and a
    single ROCr runtime) mapped in the process: the binding brings torch in
    first, so the library binds to torch's copy."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2005_06332_amd import sim\n"
        "sim.lib()\n"
        "import torch\n"
        "maps = open('/proc/self/maps').read().split()\n"
        "print(len({m for m in maps if 'libamdhip64' in m}),"
        " len({m for m in maps if 'libhsa-runtime64' in m}))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300, check=True).stdout.split()
    assert out == ["1", "1"], out
