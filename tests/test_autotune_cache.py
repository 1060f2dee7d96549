"""Host logic of the autotune cache: a stored choice is reused for the same
(device, library, batch) key and timing happens only on a miss."""
import json

from paper_2505_09324_amd import _lib, autotune


class FakeTuner:
    def __init__(self, best):
        self.best, self.calls = best, 0

    def __call__(self, sizes, targets, xy, chol, rgb, candidates, reps=5):
        self.calls += 1
        return self.best, [1.0 + i for i in range(len(candidates))]


def test_cache_hit_miss_and_keys(tmp_path, monkeypatch):
    fake = FakeTuner(best=4)
    monkeypatch.setattr(_lib, "autotune_batch", fake)
    path = str(tmp_path / "sub" / "autotune.json")
    sizes = [(320, 240, 3000), (1920, 1080, 50000)]
    kw = dict(cache_path=path, device_name="gpu0", library="abc")
    cfg, ms, cached = autotune.tuned_batch_config(sizes, None, None, None, None, **kw)
    assert cfg == (32, 2) and not cached and fake.calls == 1 and ms["8/1"] == 1.0
    cfg2, ms2, cached2 = autotune.tuned_batch_config(sizes, None, None, None, None, **kw)
    assert cfg2 == (32, 2) and cached2 and ms2 == {} and fake.calls == 1
    # any part of the key changing means a new tuning
    autotune.tuned_batch_config(sizes[::-1], None, None, None, None, **kw)
    autotune.tuned_batch_config(sizes, None, None, None, None, cache_path=path,
                                device_name="gpu1", library="abc")
    autotune.tuned_batch_config(sizes, None, None, None, None, cache_path=path,
                                device_name="gpu0", library="def")
    assert fake.calls == 4
    data = json.load(open(path))
    assert len(data) == 4 and all(v["best"] == [32, 2] for v in data.values())


def test_no_cache_and_unreadable_file(tmp_path, monkeypatch):
    fake = FakeTuner(best=0)
    monkeypatch.setattr(_lib, "autotune_batch", fake)
    sizes = [(64, 64, 100)]
    autotune.tuned_batch_config(sizes, None, None, None, None, cache_path=None)
    autotune.tuned_batch_config(sizes, None, None, None, None, cache_path=None)
    assert fake.calls == 2
    path = tmp_path / "bad.json"
    path.write_text("{not json")
    cfg, _, cached = autotune.tuned_batch_config(sizes, None, None, None, None,
                                                 cache_path=str(path), device_name="g",
                                                 library="x")
    assert cfg == (8, 1) and not cached and fake.calls == 3
    assert json.load(open(path))  # rewritten as valid JSON
