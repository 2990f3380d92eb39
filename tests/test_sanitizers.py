"""The oracle and the library's host layout code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

Both are built with gcc/g++ here (no device code) and run on a small seeded
problem written as raw arrays: the oracle simulates it in both precision modes
and replays it from its own raster; the layout planner lays it out for every
solver, packing, scheduler and two LDS budgets and walks every introspection
call. Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2005_06332_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")


def write_problem(prob, d):
    for k in ("comp_off", "parent", "length_um", "diam_um", "mech", "detector", "iext_nA",
              "syn_pre", "syn_post", "syn_comp", "syn_delay", "syn_w"):
        dt = {"comp_off": np.int64, "length_um": np.float64, "diam_um": np.float64,
              "mech": np.uint8, "iext_nA": np.float64, "syn_w": np.float64}.get(k, np.int32)
        np.ascontiguousarray(prob[k], dt).tofile(os.path.join(d, k + ".bin"))


def problem():
    mini = W.mini(seed=3, n_neurons=24, n_steps=120)
    star = W.star_network(n_neurons=4)
    # a network of both: mini neurons, then the high fan-out ones
    keep = [mini, star]
    parts = {k: [] for k in ("parent", "length_um", "diam_um", "mech")}
    n_comp, det, iext, pre, post, comp, delay, w = [], [], [], [], [], [], [], []
    base = 0
    for p in keep:
        for k in parts:
            parts[k].append(p[k])
        n_comp.append(p["n_comp"])
        det.append(p["detector"])
        iext.append(p["iext_nA"])
        pre.append(p["syn_pre"] + base)
        post.append(p["syn_post"] + base)
        comp.append(p["syn_comp"])
        delay.append(p["syn_delay"])
        w.append(p["syn_w"])
        base += p["n_comp"].shape[0]
    n = np.concatenate(n_comp)
    out = {k: np.concatenate(v) for k, v in parts.items()}
    out.update(n_comp=n, comp_off=np.concatenate([[0], np.cumsum(n)]).astype(np.int64),
               detector=np.concatenate(det), iext_nA=np.concatenate(iext),
               syn_pre=np.concatenate(pre), syn_post=np.concatenate(post),
               syn_comp=np.concatenate(comp), syn_delay=np.concatenate(delay),
               syn_w=np.concatenate(w))
    return out


@pytest.fixture(scope="module")
def data(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("san"))
    write_problem(problem(), d)
    return d


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_is_clean_under_sanitizers(data, tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-std=c99", *SAN, "-ffp-contract=off", "-fopenmp",
                    os.path.join(ROOT, "tests", "c", "oracle_sanitize.c"), "-lm", "-o", exe],
                   check=True)
    r = subprocess.run([exe, data, "120"], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert int(r.stdout.split()[-1]) > 0


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or HIP headers missing")
def test_layout_planner_is_clean_under_sanitizers(data, tmp_path):
    exe = str(tmp_path / "plan_san")
    subprocess.run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(ROOT, "paper_2005_06332_amd", "csrc", "host.cpp"),
                    os.path.join(ROOT, "tests", "c", "plan_sanitize.cpp"),
                    "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                   check=True)
    r = subprocess.run([exe, data], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "planned 24 variants" in r.stdout
