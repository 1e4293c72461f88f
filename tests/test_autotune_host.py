"""The plan autotuner's cache on the host: the committed choices are found
under the keys the measured workloads produce on gfx950, are among the
candidates, and a saved result reads back."""
import json

import pytest

import workloads


@pytest.fixture
def gfx950(monkeypatch):
    import torch
    from paper_2608_13686_amd import autotune

    class Props:
        gcnArchName = "gfx950:sramecc+:xnack-"
    monkeypatch.setattr(torch.cuda, "current_device", lambda: 0)
    monkeypatch.setattr(torch.cuda, "get_device_properties", lambda dev: Props())
    return autotune


def test_committed_choices_found_for_measured_workloads(gfx950):
    n2 = workloads.workload_n2_fixed(1 << 20)
    wb = workloads.workload_batched(32768)
    for probs, prec in ((n2["problems"], "fp64"), (n2["problems"], "mixed"),
                        (wb["problems"], "mixed")):
        t = gfx950.cached(probs, prec)
        assert t is not None, gfx950.cache_key(probs, prec)
        assert t[:4] + (8,) in gfx950.CANDIDATES and t[4] in gfx950.RERUN_LANES


def test_keys_separate_precision_potential_and_basis(gfx950):
    n2, h2 = [workloads.n2(0.0)], [workloads.h2_softcore()]
    keys = {gfx950.cache_key(n2, "fp64"), gfx950.cache_key(n2, "mixed"),
            gfx950.cache_key(h2, "fp64"), gfx950.cache_key(n2 + h2, "fp64")}
    assert len(keys) == 4
    assert all(k.startswith("gfx950_") for k in keys)


def test_save_then_cached(gfx950, tmp_path, monkeypatch):
    probs = [workloads.h2_softcore()]
    res = {"key": gfx950.cache_key(probs, "fp64"), "best": [1, 12, 2, 1],
           "table": [], "workload": {}}
    path = gfx950.save(res, str(tmp_path))
    assert json.load(open(path))["best"] == [1, 12, 2, 1]
    monkeypatch.setattr(gfx950, "CACHE_DIR", str(tmp_path))
    assert gfx950.cached(probs, "fp64") == (1, 12, 2, 1, 8)
    assert gfx950.cached(probs, "mixed") is None
