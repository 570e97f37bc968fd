"""Section 4 S/N against time and frequency resolution on the GPU path (fp32 dedispersion
of a rendered 1 ms rectangular pulse at DM 30 through greedy and all-nonzero sample sets)
against the oracle on the same inputs."""
import math

import numpy as np
import pytest

import bench
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch  # noqa: F401
    import paper_1301_3968_amd as dd
    return dd


@pytest.mark.parametrize("a,b", [(1.0, 1.0), (0.5, 2.0)])
def test_resolution_points_match_oracle(dd, orc, otables, a, b):
    got = {}
    for rule in ("greedy", "allnonzero"):
        snr, plan, dt, cw, x = bench.resolution_point(dd, workloads, a, b, rule)
        lo, bw = bench.RES_BAND
        C = int(round(bw / cw))
        f = workloads.channel_centres(lo, bw, C)
        s, n = otables(plan, f, cw, dt, [bench.RES_DM], rule, width_s=bench.RES_TAU)
        y = orc.dedisperse_f64(x.astype(np.float64), s, n)[0]
        ref = y.max() / math.sqrt(float(n.sum())) * math.sqrt(dt / (C * bench.RES_TAU))
        assert snr == pytest.approx(ref, rel=1e-5)
        got[rule] = snr
    # the greedy set maximises the S/N of this pulse model; all non-zero samples cannot beat it
    assert got["greedy"] >= got["allnonzero"] * (1.0 - 1e-3)
