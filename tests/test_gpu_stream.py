"""Streams pushed in blocks (Section 2.1's real-time setting): the dedispersed outputs
of the blocks, joined, equal the oracle's dedispersion of the whole stream bit for bit,
and the per-trial best over the blocks equals the oracle's search of the whole stream;
blocks shorter than the carried tail, and a single-sample block, are accepted."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

CHUNKS = [700, 1300, 50, 1, 997]      # then the rest of the 4096 samples


@pytest.fixture(scope="module")
def dd():
    import torch  # noqa: F401
    import paper_1301_3968_amd as dd
    return dd


def _blocks(x):
    import torch
    edges = np.cumsum([0] + CHUNKS + [x.shape[1] - sum(CHUNKS)])
    return [torch.from_numpy(np.ascontiguousarray(x[:, a:b])).cuda()
            for a, b in zip(edges[:-1], edges[1:])]


def test_stream_dedisperse_matches_whole_block(dd, orc, otables):
    wl = workloads.cfg1()
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule)
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, wl.rule)
    yo = orc.dedisperse_u8(wl.x, s, n)
    st = dd.StreamDedisperser(p)
    parts, nxt = [], 0
    for blk in _blocks(wl.x):
        y, t0 = st.push(blk)
        if y is None:
            continue
        assert t0 == nxt                       # no gap, no overlap
        parts.append(y.cpu().numpy())
        nxt += y.shape[1]
    got = np.concatenate(parts, axis=1).astype(np.int64)
    assert np.array_equal(got, yo)


def test_stream_search_matches_whole_block(dd, orc, otables):
    import torch
    wl = workloads.cfg1()
    widths = [1, 2, 4, 8, 16, 32]
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule)
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, wl.rule)
    y64 = orc.dedisperse_u8(wl.x, s, n).astype(np.float64)
    M, S = orc.boxcar_norm(n, widths, wl.chan_mean, wl.chan_sigma)
    so, to, wo = orc.boxcar_detect(y64, widths, M, S)
    mu = torch.from_numpy(np.asarray(wl.chan_mean, dtype=np.float64)).cuda()
    sg = torch.from_numpy(np.asarray(wl.chan_sigma, dtype=np.float64)).cuda()
    st = dd.StreamSearch(p, widths, mu, sg)
    searched = 0
    for blk in _blocks(wl.x):
        r = st.push(blk)
        if r is not None:
            searched += 1
            snr_b, t_b, w_b, t0 = r
            # a block's candidates are windows of the whole stream
            tb, wb = t_b.cpu().numpy(), w_b.cpu().numpy()
            for d in np.nonzero(tb >= 0)[0][:8]:
                j = widths.index(int(wb[d]))
                B = float(np.sum(y64[d, t0 + tb[d]:t0 + tb[d] + wb[d]]))
                assert snr_b[d].item() == pytest.approx((B - M[d, j]) / S[d, j], rel=1e-12)
    assert searched >= 3
    snr, t, w = [v.cpu().numpy() for v in st.best()]
    assert np.allclose(snr, so, rtol=1e-12, atol=0)
    for d in np.nonzero((t != to) | (w != wo))[0]:
        j = widths.index(int(w[d]))
        B = float(np.sum(y64[d, t[d]:t[d] + w[d]]))
        assert (B - M[d, j]) / S[d, j] == pytest.approx(so[d], rel=1e-12)
