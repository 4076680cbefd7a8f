"""The seeded input generators (CPU only): deterministic, with the hard-input
share the workloads promise, and loud when a hard set is missing."""
import numpy as np
import pytest

from paper_2605_15547_amd import inputs


def test_workloads_are_deterministic():
    for f in ("expf", "log1pf", "sinf", "atanf"):
        a = inputs.workload_f32(f, 4096)
        b = inputs.workload_f32(f, 4096)
        assert a.dtype == np.float32 and np.array_equal(a.view(np.uint32), b.view(np.uint32))
    a = inputs.workload_f64("log", 4096)
    assert np.array_equal(a.view(np.uint64), inputs.workload_f64("log", 4096).view(np.uint64))


@pytest.mark.parametrize("func", inputs.EXPLOG_FAMILY)
def test_explog_workload_carries_the_hard_share(func):
    """5% of the exp/log-family elements come from the function's hard set."""
    n = 1 << 16
    x = inputs.workload_f32(func, n)
    hs = set(inputs.hard_set(func).view(np.uint32).tolist())
    share = np.mean([v in hs for v in x.view(np.uint32).tolist()])
    assert 0.045 < share < 0.06, share


def test_missing_hard_set_raises(monkeypatch, tmp_path):
    """Without its hard set a workload would silently change: it must fail."""
    monkeypatch.setattr(inputs, "GOLDEN", str(tmp_path))
    with pytest.raises(FileNotFoundError):
        inputs.hard_set("expf")
    with pytest.raises(FileNotFoundError):
        inputs.workload_f32("logf", 1024)
    with pytest.raises(FileNotFoundError):
        inputs.workload_f64("exp", 4096)
