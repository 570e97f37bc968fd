import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")


def pytest_collection_modifyitems(config, items):
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def otables(orc):
    """The oracle's sample-set tables for a plan's rule (so that no oracle input comes from
    the library), after checking that the plan's own tables equal them (starts compared
    where a channel takes samples)."""
    import numpy as np

    def tables(plan, freqs, bw, dt, dms, rule, width_s=0.0, ktaps=1):
        s = orc.delay_start(freqs, bw, dt, dms)
        if rule == "smear":
            n = orc.taps_smear(freqs, bw, dt, dms)
        elif rule == "allnonzero":
            n = orc.taps_allnonzero(freqs, bw, dt, dms, width_s)
        elif rule == "fixed":
            n = np.full(s.shape, ktaps, dtype=np.int64)
        elif rule == "greedy":
            s, n, _ = orc.greedy_tables(freqs, bw, dt, dms, width_s)
        else:
            raise ValueError(rule)
        s, n = s.astype(np.int32), n.astype(np.int32)
        ps, pn = plan.tables()
        assert np.array_equal(pn, n)
        assert np.array_equal(np.where(n > 0, ps, 0), np.where(n > 0, s, 0))
        return s, n

    return tables
