"""The allocation-free search entry point (dedisp_search_noalloc) against the
workspace search (dedisp_search), through the C ABI, on two calls in a row (the
second with a shorter block), and its refusals: a plan whose tables are not on the
device yet, a block whose workspace exceeds the scratch array."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _outs(torch, D):
    return (torch.empty(D, dtype=torch.float64, device="cuda"),
            torch.empty(D, dtype=torch.int32, device="cuda"),
            torch.empty(D, dtype=torch.int32, device="cuda"))


def test_noalloc_matches_workspace_search():
    import torch
    import paper_1301_3968_amd as dd
    wl = workloads.cfg2(nsamp=20000, ndm=200)
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule)
    mu = torch.as_tensor(wl.chan_mean, dtype=torch.float64).cuda()
    sg = torch.as_tensor(wl.chan_sigma, dtype=torch.float64).cuda()
    D = len(wl.dms)
    xa = torch.from_numpy(wl.x).cuda()
    # before any search with this plan its device tables do not exist: refused
    with pytest.raises(dd.DedispError) as e:
        p.search_noalloc(xa, wl.widths, mu, sg, _outs(torch, D))
    assert e.value.status == 1
    rng = np.random.default_rng(31)
    xb = torch.from_numpy(workloads.u8_noise(rng, 336, 9000)).cuda()   # a shorter block
    for x in (xa, xb):
        ref = [v.cpu().numpy() for v in p.search(x, wl.widths, mu, sg)]
        assert p.last_search_tile() >= 8            # the matrix-core search
        got = p.search_noalloc(x, wl.widths, mu, sg, _outs(torch, D))
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert np.array_equal(a, b.cpu().numpy())


def test_noalloc_refuses_oversized_workspace():
    import torch
    import paper_1301_3968_amd as dd
    wl = workloads.cfg2(nsamp=8000, ndm=1024)
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule)
    mu = torch.as_tensor(wl.chan_mean, dtype=torch.float64).cuda()
    sg = torch.as_tensor(wl.chan_sigma, dtype=torch.float64).cuda()
    p.search(torch.from_numpy(wl.x).cuda(), wl.widths, mu, sg)   # builds the device tables
    # 1024 trials x 32 widths of noise tables plus 1024 trials x ~1300 time tiles of
    # candidates is more than the 16 MiB scratch array
    big = torch.full((336, 1_300_000), 128, dtype=torch.uint8, device="cuda")
    with pytest.raises(dd.DedispError) as e:
        p.search_noalloc(big, wl.widths, mu, sg, _outs(torch, 1024))
    assert e.value.status == 1 and "exceeds" in str(e.value)
