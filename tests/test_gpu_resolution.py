"""Section 4 S/N against time and frequency resolution on the GPU path (fp32 dedispersion
of a rendered 1 ms rectangular pulse at DM 30 through greedy and all-nonzero sample sets)
against the oracle on the same inputs: the whole dedispersed series at the corners,
the centre and two inner points of the grid."""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch  # noqa: F401
    import paper_1301_3968_amd as dd
    return dd


@pytest.mark.parametrize("a,b", [(1.0, 1.0), (0.5, 2.0), (0.125, 0.125), (8.0, 8.0),
                                 (0.125, 8.0), (8.0, 0.125)])
def test_resolution_points_match_oracle(dd, orc, otables, an, a, b):
    import torch
    got = {}
    for rule in ("greedy", "allnonzero"):
        snr, plan, dt, cw, x = an.resolution_point(dd, workloads, a, b, rule)
        lo, bw = an.RES_BAND
        C = int(round(bw / cw))
        f = workloads.channel_centres(lo, bw, C)
        s, n = otables(plan, f, cw, dt, [an.RES_DM], rule, width_s=an.RES_TAU)
        y = orc.dedisperse_f64(x.astype(np.float64), s, n)[0]
        # the whole series: fp32 sums of positive terms, 1e-5 of the fp64 value (of the
        # series' peak for the near-zero tails)
        yg = plan.dedisperse(torch.from_numpy(x).cuda())[0].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(yg, y, rtol=1e-5, atol=1e-6 * y.max())
        ref = y.max() / math.sqrt(float(n.sum())) * math.sqrt(dt / (C * an.RES_TAU))
        assert snr == pytest.approx(ref, rel=1e-5)
        got[rule] = snr
    # the greedy set maximises the S/N of this pulse model; all non-zero samples cannot beat it
    assert got["greedy"] >= got["allnonzero"] * (1.0 - 1e-3)
