"""Host logic of the autotuner: the fastest setting is kept, settings whose
lists would outgrow the limit are skipped, slow settings are timed once, and
the choice is left set on the context."""
import math

from paper_2607_26901_amd import autotune


class FakeCtx:
    def __init__(self):
        self.t = {"cell_scale": 1.0, "pair_split": 1, "pair_reuse": 1, "pair_skin": 0, "broad_phase": 0,
                  "direct_regions": 0}
        self.calls = []

    def set_tuning(self, **kw):
        self.t.update({k: v for k, v in kw.items() if v is not None})
        self.calls.append(dict(self.t))

    def get_tuning(self):
        return dict(self.t)


def test_tune_picks_fastest_and_skips():
    ctx = FakeCtx()
    runs = []
    cost = {(1, 0): 10.0, (2, 0): 7.0, (3, 0): 6.0, (4, 0): 40.0, (1, 1): 8.0}
    big = {(4, 0)}

    def run(limit):
        key = (ctx.t["pair_reuse"], ctx.t["pair_skin"])
        runs.append((key, limit))
        nbytes = (1 << 30) * (100 if key in big else 1)
        if limit is not None and nbytes > limit:
            raise autotune.TooLarge()
        return cost[key] * ctx.t["cell_scale"], nbytes

    logs = []
    out = autotune.tune(ctx, run, candidates=(1.0, 0.5), splits=(1,), modes=list(cost), log=logs.append)
    assert (out["cell_scale"], out["pair_reuse"], out["pair_skin"]) == (0.5, 3, 0)
    assert ctx.t["cell_scale"] == 0.5 and ctx.t["pair_reuse"] == 3
    assert math.isinf(out["ms"]["1.0/1/4/0/0/0"]) and math.isinf(out["ms"]["0.5/1/4/0/0/0"])
    # the first run sets the limit: four times its bytes
    assert runs[0][1] is None and all(l == 4 * (1 << 30) for _, l in runs[1:])
    # (1, 0) at cell 1.0 is timed three times (first record, then two repeats)
    assert sum(1 for k, _ in runs if k == (1, 0)) >= 3
    assert len(logs) == 2 * len(cost)


def test_slow_setting_timed_once():
    ctx = FakeCtx()
    runs = []

    def run(limit):
        key = ctx.t["pair_reuse"]
        runs.append(key)
        return {1: 5.0, 2: 50.0}[key], 1 << 20

    out = autotune.tune(ctx, run, candidates=(1.0,), splits=(1,), modes=[(1, 0), (2, 0)], log=None)
    assert out["pair_reuse"] == 1
    assert runs.count(2) == 1 and runs.count(1) == 3


def test_hierarchy_timed_once_per_mode_and_chosen_when_faster():
    """The hierarchy has no cell or split knob: it is timed once per mode (at
    the neutral cell scale and one lane), and kept when it is the fastest."""
    ctx = FakeCtx()
    seen = []

    def run(limit):
        t = dict(ctx.t)
        seen.append(t)
        if t["broad_phase"] == 1:
            return 2.0 + t["pair_reuse"], 1 << 20
        return 5.0 * t["cell_scale"] + t["pair_split"], 1 << 20

    out = autotune.tune(ctx, run, candidates=(0.5, 1.0), splits=(1, 3), modes=[(1, 0), (2, 0)], log=None,
                        broad_phases=(0, 1))
    assert (out["broad_phase"], out["pair_reuse"]) == (1, 1) and ctx.t["broad_phase"] == 1
    lbvh = {(t["cell_scale"], t["pair_split"]) for t in seen if t["broad_phase"] == 1}
    assert lbvh == {(1.0, 1)}
    assert set(out["ms"]) == {f"{c}/{sp}/{ru}/0/0/0" for c in (0.5, 1.0) for sp in (1, 3) for ru in (1, 2)} | \
        {"1.0/1/1/0/1/0", "1.0/1/2/0/1/0"}


def test_direct_regions_tried_on_the_best_setting():
    """The narrow phase's direct slot writes are timed once, on the best of the
    other settings, and kept only when faster."""
    for direct_ms, want in ((2.0, 1), (9.0, 0)):
        ctx = FakeCtx()

        def run(limit):
            if ctx.t["direct_regions"]:
                return direct_ms, 1 << 20
            return 5.0 * ctx.t["cell_scale"], 1 << 20

        out = autotune.tune(ctx, run, candidates=(0.5, 1.0), splits=(1,), modes=[(1, 0)], log=None, directs=(0, 1))
        assert out["direct_regions"] == want and ctx.t["direct_regions"] == want
        assert out["cell_scale"] == 0.5 and "0.5/1/1/0/0/1" in out["ms"] and "1.0/1/1/0/0/1" not in out["ms"]
