"""The algorithmic byte model behind bench.py's roofline, against the
per-update figures of the measurement plan: V read and written in FP64 (16 B),
the three gates read and written (48 B in FP64, 24 B with FP32 gating), 24 B of
per-compartment constants where morphologies differ, and each synapse's
conductance read and written (8 B with FP32 gating, 16 B in FP64) spread over
the compartments. A dropped term, a gate width taken from the wrong precision
or constants counted for identical neurons each move a figure below."""
import numpy as np
import pytest

import bench
from paper_2005_06332_amd import workload as W


@pytest.mark.parametrize("cfg,precision,expect", [
    (2, 0, 16 + 48 + 0 + 0.05 * 16),   # 8,192 identical neurons, 409,600 synapses
    (2, 1, 16 + 24 + 0 + 0.05 * 8),
    (3, 1, 16 + 24 + 24 + 1638400 / 9293129 * 8),  # 65.41
])
def test_algorithmic_bytes_per_update(cfg, precision, expect):
    prob = W.make(cfg, precision=precision)
    C = int(prob["comp_off"][-1])
    multi = len(np.unique(prob["n_comp"])) > 1
    b = bench.bytes_per_update(precision, multi, prob["syn_pre"].shape[0] / C)
    assert b == pytest.approx(expect, rel=1e-12)
    assert multi == (cfg != 2)


def test_benchmark_workload_prices_at_65_4_bytes():
    """The figure the class-0 roofline of the default run uses."""
    prob = W.make(3)
    C = int(prob["comp_off"][-1])
    b = bench.bytes_per_update(1, True, prob["syn_pre"].shape[0] / C)
    assert round(b, 2) == 65.41
