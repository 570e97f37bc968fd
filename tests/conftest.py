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


def oracle_threads() -> int:
    """Host threads for oracle loops: the host cores, at most 16."""
    return max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="session")
def opar(orc):
    """The oracle's trial-by-trial loops run over disjoint trial ranges in threads (each
    range is an ordinary oracle call; ctypes releases the GIL while it runs)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    class Par:
        @staticmethod
        def ranges(D, parts=None):
            parts = parts or oracle_threads()
            edges = np.linspace(0, D, min(D, parts) + 1).round().astype(int)
            return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]

        @classmethod
        def dedisperse_u8(cls, x, s, n, tout):
            with ThreadPoolExecutor(oracle_threads()) as ex:
                parts = list(ex.map(lambda r: orc.dedisperse_u8(x, s[r[0]:r[1]], n[r[0]:r[1]],
                                                                 tout=tout),
                                    cls.ranges(s.shape[0])))
            return np.concatenate(parts, axis=0)

        @classmethod
        def detect(cls, y64, widths, M, S):
            with ThreadPoolExecutor(oracle_threads()) as ex:
                parts = list(ex.map(lambda r: orc.boxcar_detect(y64[r[0]:r[1]], widths,
                                                                M[r[0]:r[1]], S[r[0]:r[1]]),
                                    cls.ranges(y64.shape[0])))
            return tuple(np.concatenate([p[i] for p in parts]) for i in range(3))

        @staticmethod
        def map(fn, items):
            with ThreadPoolExecutor(oracle_threads()) as ex:
                return list(ex.map(fn, items))

    return Par


@pytest.fixture(scope="session")
def an():
    """The package's analyses of Sections 4-5 (run through the library)."""
    from paper_1301_3968_amd import analyses
    return analyses
