"""Host logic of the autotuner (paper_2007_02306_amd/tune.py) with a stand-in
context: the fastest candidate is chosen, the choice is cached per shape
class and architecture, and a cached class is not measured again."""

import json

import pytest
import torch

from paper_2007_02306_amd.tune import GEN_CHOICES, SEARCH_CHOICES, SORT_CHOICES, Tuner


class FakeCtx:
    """Records knob settings; 'kernel time' is a function of the knobs."""

    device = 0

    def __init__(self, gen_ms, search_ms, batch_ms):
        self.knobs = {"gen_images_per_group": 2, "search_tile_m": 256, "gen_sort_triangles": 2}
        self.gen_ms, self.search_ms, self.batch_ms = gen_ms, search_ms, batch_ms
        self.calls = []
        self._last = {}

    def set_tuning(self, k, v):
        self.knobs[k] = v

    def get_tuning(self, k):
        return self.knobs[k]

    def timing(self, on=True):
        pass

    def timing_reset(self):
        self._last = {}

    def timing_get(self, kernel):
        return self._last.get(kernel, 0.0), 1

    def generate(self, pos, tri, opp, opn, R, out=None, stream=None):
        g, o = self.knobs["gen_images_per_group"], self.knobs["gen_sort_triangles"]
        self.calls.append(("generate", g, o, opp.shape[0]))
        # gen_ms maps (group, order) -> (preparation ms, generation ms)
        self._last["gen_prep"], self._last["gen"] = self.gen_ms[(g, o)]
        return out

    def distance_rank(self, n, h, t, **kw):
        self.calls.append(("rank", self.knobs["search_tile_m"], h.shape[0]))
        self._last["search"] = self.search_ms[self.knobs["search_tile_m"]]
        return None, None

    def batch(self, jobs, R):
        ctx = self
        knobs = dict(self.knobs)

        class Plan:
            def run(self):
                ctx._last["batch"] = ctx.batch_ms[(knobs["gen_images_per_group"], knobs["search_tile_m"],
                                                   knobs["gen_sort_triangles"])]

            def close(self):
                pass
        self.calls.append(("batch", knobs["gen_images_per_group"], knobs["search_tile_m"],
                           knobs["gen_sort_triangles"], len(jobs)))
        return Plan()


def _mesh(nt=300, nv=200, n=50):
    g = torch.Generator().manual_seed(0)
    return (torch.rand(nv, 3, generator=g), torch.randint(0, nv, (nt, 3), generator=g, dtype=torch.int32),
            torch.rand(n, 3, generator=g), torch.rand(n, 3, generator=g))


@pytest.fixture(autouse=True)
def _no_cuda_sync(monkeypatch):
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)


def test_generation_picks_fastest_and_caches(tmp_path):
    # (group, order) -> (prep ms, gen ms): the Morton order's costlier
    # preparation decides between (4, 0) and (4, 1)
    ms = {(2, 0): (0.1, 5.0), (2, 1): (0.5, 4.9), (4, 0): (0.1, 3.0), (4, 1): (0.5, 2.8)}
    ctx = FakeCtx(ms, {256: 1.0, 128: 2.0}, {})
    path = tmp_path / "tune.json"
    t = Tuner(ctx, str(path), reps=2, gen_sample=16, arch="gfx-test")
    pos, tri, opp, opn = _mesh()
    assert t.tune_generate(pos, tri, opp, opn, 0.3) == (4, 0)
    assert {(g, o) for g in GEN_CHOICES for o in SORT_CHOICES} == {m[1] for m in t.measurements}
    assert all(c[3] == 16 for c in ctx.calls)              # calibration subset only
    assert ctx.knobs["gen_images_per_group"] == 2           # restored after tuning
    assert ctx.knobs["gen_sort_triangles"] == 2
    data = json.loads(path.read_text())
    assert list(data["gfx-test"].values()) == [[4, 0]]
    # a fresh tuner reads the cache and measures nothing
    ctx2 = FakeCtx({k: (0.0, 9.0) for k in ms}, {}, {})
    t2 = Tuner(ctx2, str(path), arch="gfx-test")
    t2.generate(pos, tri, opp, opn, 0.3)
    assert t2.measurements == [] and ctx2.calls == [("generate", 4, 0, 50)]
    # another architecture is tuned anew
    ms3 = {(2, 0): (0.1, 2.0), (2, 1): (0.2, 1.0), (4, 0): (0.1, 3.0), (4, 1): (0.2, 2.5)}
    t3 = Tuner(FakeCtx(ms3, {}, {}), str(path), arch="gfx-other")
    assert t3.tune_generate(pos, tri, opp, opn, 0.3) == (2, 1)
    # a cache written before the order knob existed (a bare group) still reads
    path2 = tmp_path / "old.json"
    path2.write_text(json.dumps({"gfx-test": {Tuner.gen_class(pos, tri, opp, 0.3): 4}}))
    assert Tuner(FakeCtx(ms, {}, {}), str(path2), arch="gfx-test").tune_generate(pos, tri, opp, opn, 0.3) == (4, 2)


def test_search_classes_and_choice(tmp_path):
    assert Tuner.search_class(100, 23352) == Tuner.search_class(128, 30000)
    assert Tuner.search_class(129, 23352) != Tuner.search_class(128, 23352)
    assert Tuner.search_class(5000, 10) == Tuner.search_class(9000, 10)     # capped
    ctx = FakeCtx({}, {256: 2.0, 128: 1.5}, {})
    t = Tuner(ctx, None, arch="gfx-test", search_haystack_sample=100)
    n = torch.zeros(40, 64, 64, dtype=torch.int32)
    h = torch.zeros(1000, 64, 64, dtype=torch.int32)
    ti = torch.arange(40, dtype=torch.int32)
    assert t.tune_search(n, h, ti) == 128
    assert {m[1] for m in t.measurements} == set(SEARCH_CHOICES)
    assert all(c[2] == 100 for c in ctx.calls)              # haystack subset
    t.distance_rank(n, h, ti)
    assert ctx.calls[-1] == ("rank", 128, 1000)


def test_batch_tunes_all_three_knobs_on_a_subset():
    ms = {(2, 256, 0): 4.0, (2, 128, 0): 5.0, (4, 256, 0): 3.0, (4, 128, 0): 6.0,
          (2, 256, 1): 4.1, (2, 128, 1): 5.1, (4, 256, 1): 2.9, (4, 128, 1): 6.1}
    ctx = FakeCtx({}, {}, ms)
    t = Tuner(ctx, None, arch="gfx-test")
    jobs = [dict(triangles=torch.zeros(10 * (k + 1), 3), op_positions=torch.zeros(k + 1, 3)) for k in range(40)]
    assert t.tune_batch(jobs, 0.3, sample_jobs=8) == (4, 256, 1)
    sizes = [c[4] for c in ctx.calls if c[0] == "batch"]
    assert sizes == [8] * 8
    assert ctx.knobs["gen_sort_triangles"] == 2             # restored after tuning
    t.batch(jobs, 0.3)
    assert ctx.calls[-1] == ("batch", 4, 256, 1, 40)
