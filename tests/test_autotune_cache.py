"""Autotune cache bookkeeping on the CPU (a stand-in context; no timing)."""
import json

from paper_1908_01762_amd import autotune, cases


class FakeCtx:
    def __init__(self, case, best):
        self.case = case
        self.variant = 1
        self.best = best
        self.calls = 0

    def autotune(self, reps):
        self.calls += 1
        return self.best, [10.0 + v for v in range(6)]


def test_key_buckets_by_kind_and_size():
    a = cases.taylor_green(100, kernel="wendland", hdx=1.3, precision="mixed")
    b = cases.taylor_green(101, kernel="wendland", hdx=1.3, precision="mixed")
    c = cases.taylor_green(100, precision="fp64")
    assert autotune.key(a) == autotune.key(b)
    assert autotune.key(a) != autotune.key(c)


def test_tune_times_once_then_reuses(tmp_path):
    path = str(tmp_path / "t.json")
    case = cases.taylor_green(40)
    x = FakeCtx(case, best=4)
    rec = autotune.tune(x, cache_path=path)
    assert rec["variant"] == 4 and x.variant == 4 and x.calls == 1
    y = FakeCtx(case, best=0)
    autotune.tune(y, cache_path=path)
    assert y.calls == 0 and y.variant == 4
    z = FakeCtx(case, best=2)
    assert autotune.apply_cached(z, cache_path=path) and z.variant == 4
    autotune.tune(z, cache_path=path, force=True)
    assert z.calls == 1 and json.load(open(path))[autotune.key(case)]["variant"] == 2
    assert not autotune.apply_cached(FakeCtx(cases.taylor_green(300), 0), cache_path=path)
