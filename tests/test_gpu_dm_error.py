"""Section 5.2 DM-error attenuation on the GPU path (greedy sample set of trial DM 30,
batched fp32 dedispersion of rendered rectangular test pulses) against the oracle on the
same inputs."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch  # noqa: F401
    import paper_1301_3968_amd as dd
    return dd


def test_dm_error_profiles_match_oracle(dd, orc, otables, an):
    flo, band, C, dt, tau, dm = an.DM_ERROR_CASE
    xs = np.array([0.0, -3.0, 2.5, -0.5, 8.0])
    plan, prof, _ = an.dm_error_profiles(dd, workloads, xs)
    f = workloads.channel_centres(flo, band, C)
    s, n = otables(plan, f, band / C, dt, [dm], "greedy", width_s=tau)
    T = plan.max_span + 128
    unit = (1.0 / C) * np.sqrt(dm * dm + orc.dm_diag(f, band / C, dt) ** 2
                               + orc.dm_tau(f, band / C, tau) ** 2)
    assert an.dm_error_unit() == pytest.approx(unit, rel=1e-12)
    ys = []
    for d in [dm] + [dm + x * unit for x in xs]:
        x = workloads.render_rect_pulse(f, band / C, dt, T, float(d), tau, 64 * dt)
        ys.append(orc.dedisperse_f64(x.astype(np.float64), s, n)[0])
    ref = np.array(ys[1:]) / ys[0].max()
    # fp32 sums of positive terms: 1e-5 of the fp64 value (of the profile's peak for the
    # near-zero tails)
    np.testing.assert_allclose(prof, ref, rtol=1e-5, atol=1e-6)
    peak = prof.max(axis=1)
    assert peak[0] == pytest.approx(1.0, rel=1e-6)
    assert np.all(peak[1:] < 1.0)
