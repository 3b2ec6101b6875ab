"""Host logic of the autotuner's cache (no device work): keys, round trip, bad files."""
import json

from paper_2507_15209_amd import autotune as at
from paper_2507_15209_amd import _lib


class _StubPlan:
    """Only the attributes the cache reads and writes."""

    def __init__(self, n=64, nbins=8, lmax=4, summation="nodal", precision="f32", batch=1):
        self.n, self.nbins, self.lmax, self.batch = n, nbins, lmax, batch
        self.summation, self.precision, self.device = summation, precision, None
        self.knobs = {"zpass_wgs": 4096, "contract_wgs": 4096, "fft_x_plan": 0, "deposit_tile": 8,
                      "deposit_wgs": 2048}

    def tune_set(self, k, v):
        assert k in _lib.TUNE_KNOBS
        self.knobs[k] = v

    def tune_get(self, k):
        return self.knobs[k]

    def tuning(self):
        return dict(self.knobs)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    p = _StubPlan()
    p.knobs["zpass_wgs"] = 8192
    p.knobs["deposit_tile"] = 16
    at.save_tuning(p, {"zpass_wgs": 1.5}, path)
    q = _StubPlan()
    assert at.load_tuning(q, path)
    assert q.knobs["zpass_wgs"] == 8192 and q.knobs["deposit_tile"] == 16
    data = json.load(open(path))
    assert data[at.cache_key(p)]["ms"] == {"zpass_wgs": 1.5}


def test_cache_keys_separate_configurations(tmp_path):
    path = str(tmp_path / "tuning.json")
    a = _StubPlan(n=64)
    a.knobs["fft_x_plan"] = 1
    at.save_tuning(a, None, path)
    for other in (_StubPlan(n=128), _StubPlan(nbins=9), _StubPlan(lmax=5), _StubPlan(summation="gamma"),
                  _StubPlan(precision="f64"), _StubPlan(batch=2)):
        assert at.cache_key(other) != at.cache_key(a)
        assert not at.load_tuning(other, path)
        assert other.knobs["fft_x_plan"] == 0


def test_missing_or_corrupt_cache_is_ignored(tmp_path):
    p = _StubPlan()
    assert not at.load_tuning(p, str(tmp_path / "absent.json"))
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert not at.load_tuning(p, str(bad))
    at.save_tuning(p, None, str(bad))          # a corrupt file is replaced
    assert at.load_tuning(p, str(bad))


def test_candidates_are_within_the_abi_ranges():
    for k, vals in at.CANDIDATES.items():
        assert k in _lib.TUNE_KNOBS
        for v in vals:
            if k.endswith("_wgs"):
                assert 64 <= v <= 65536
            elif k == "fft_x_plan":
                assert v in (0, 1)
            elif k == "fused_waves":
                assert 0 <= v <= 8
            elif k == "item_group":
                assert 0 <= v <= 1024
            elif k == "gamma_adjoint":
                assert v in (0, 1)
            else:
                assert v in (4, 8, 16)
