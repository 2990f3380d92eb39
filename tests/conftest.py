import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running case")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


class SharedWorkloads:
    """Full-size workloads, generated once per test session.

    The generators are deterministic and the large ones are slow (the 1e5-neuron
    network takes over a minute on eight host cores), while several GPU tests run
    the same network under different solvers, packings and precisions. Each call
    returns a fresh top-level dict with fresh params and channels dicts over
    read-only arrays, so no test can change what another one sees."""

    def __init__(self):
        self._cache = {}

    def __call__(self, cfg, **kw):
        from paper_2005_06332_amd import workload as W
        key = (cfg, tuple(sorted(kw.items())))
        if key not in self._cache:
            prob = W.make(cfg, **kw)
            for v in prob.values():
                if isinstance(v, np.ndarray):
                    v.flags.writeable = False
            self._cache[key] = prob
        prob = self._cache[key]
        out = dict(prob)
        out["params"] = dict(prob["params"])
        out["channels"] = dict(prob["channels"])
        return out


class SharedOracleRuns:
    """The oracle's run of a shared full-size workload, once per (workload,
    steps, precision) and session: (voltages, spikes) as read-only arrays. The
    oracle does not depend on the GPU-side variant under test, so every solver,
    packing and launch variant is compared with the same run."""

    def __init__(self, orc, workloads):
        self._orc, self._w, self._cache = orc, workloads, {}

    def __call__(self, cfg, steps, precision, **kw):
        key = (cfg, tuple(sorted(kw.items())), steps, precision)
        if key not in self._cache:
            ref = self._orc.Sim(self._w(cfg, **kw), max_steps=steps, precision=precision)
            try:
                ref.step(steps)
                v, s = ref.voltages(), ref.spikes()
            finally:
                ref.close()
            v.flags.writeable = False
            s.flags.writeable = False
            self._cache[key] = (v, s)
        return self._cache[key]


@pytest.fixture(scope="session")
def full_workload():
    return SharedWorkloads()


@pytest.fixture(scope="session")
def oracle_full(orc, full_workload):
    return SharedOracleRuns(orc, full_workload)
