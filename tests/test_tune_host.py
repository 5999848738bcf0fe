"""The autotuners' host logic on the CPU: which rules they time, that they
apply and cache the fastest, and that a cached choice is reused.  A fake
decoder stands in for the GPU one; its decode time depends only on the rule
it was given, so the expected choice is known."""
from __future__ import annotations

import time

import pytest

torch = pytest.importorskip("torch")


class FakeBatchedDecoder:
    """Records the tile rules it is given; a decode 'takes' a time set by
    the current rule (fastest: the rule in `best`)."""

    def __init__(self, best):
        self.n, self.m = 64, 512
        self.best = tuple(best)
        self.rule = None
        self.rules_seen = []

    def set_batched_config(self, atoms128_above, atoms64_above, atoms32_above=0):
        self.rule = (atoms128_above, atoms64_above, atoms32_above)
        self.rules_seen.append(self.rule)

    def get_batched_config(self):
        a128, a64, a32 = self.rule
        return dict(atoms128_above=a128, atoms64_above=a64, atoms32_above=a32)

    def solve_batched(self, Y, eps, max_iters, want_r=True):
        time.sleep(0.0005 if self.rule == self.best else 0.003)


@pytest.fixture
def tuner(tmp_path, monkeypatch):
    from paper_0809_1833_amd import tune
    monkeypatch.setenv("MP_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(tune, "batched_key",
                        lambda dec, nb, caps, arch=None: f"batched|test|{dec.n}|{dec.m}|{nb}")
    return tune


def test_batched_tuner_times_pairs_then_small_tiles(tuner):
    best = (tuner.NEVER, 64, 0)
    dec = FakeBatchedDecoder(best)
    Y = torch.zeros(64, 10)
    res = tuner.tune_batched(dec, Y, 1e-5, [10] * 10, reps=1)
    pairs = tuner.batched_rules()
    # every pair once (its warm-up and timed decode share the rule), then the
    # 16-atom switch points on the fastest pair
    assert len(res["timings"]) == len(pairs) + len(tuner.ATOMS32_ABOVE)
    assert [tuple(t[k] for k in ("atoms128_above", "atoms64_above", "atoms32_above"))
            for t in res["timings"]][-len(tuner.ATOMS32_ABOVE):] == \
        [(best[0], best[1], a32) for a32 in tuner.ATOMS32_ABOVE]
    assert res["config"] == dict(atoms128_above=best[0], atoms64_above=best[1], atoms32_above=0)
    assert dec.rule == best and not res["cached"]


def test_batched_tuner_picks_a_small_tile_rule_and_caches_it(tuner):
    """With the rules given, exactly those are timed (no 16-atom stage); the
    fastest is applied, cached, and reused without timing anything."""
    best = (tuner.NEVER, 96, tuner.ATOMS32_ABOVE[1])
    dec = FakeBatchedDecoder(best)
    Y = torch.zeros(64, 10)
    res = tuner.tune_batched(dec, Y, 1e-5, [10] * 10, reps=1,
                             rules=[(tuner.NEVER, 96, 0), best, (64, 32, 0)])
    assert len(res["timings"]) == 3
    assert res["config"]["atoms32_above"] == best[2] and dec.rule == best
    dec2 = FakeBatchedDecoder((0, 0, 0))
    again = tuner.tune_batched(dec2, Y, 1e-5, [10] * 10)
    assert again["cached"] and dec2.rule == best and dec2.rules_seen == [best]


class FakeRaggedDecoder:
    def __init__(self, best):
        self.best = tuple(best)
        self.cfg = None
        self.storage, self.count = "f32", 3
        self.ns, self.ms = [64, 64, 128], [256, 256, 512]
        self.x_off = [0, 256, 512, 1024]

    def set_config(self, threads, cols_per_wave, wgs_per_cu, split=0):
        self.cfg = (threads, cols_per_wave, wgs_per_cu, split)

    def get_config(self):
        t, c, w, sp = self.cfg
        return dict(threads=t, cols_per_wave=c, wgs_per_cu=w, split=sp)

    def solve(self, y, eps, caps, want_r=True, x_out=None):
        # the best shape is a little faster at every split, much faster at its own
        if self.cfg == self.best:
            time.sleep(0.0005)
        else:
            time.sleep(0.002 if self.cfg[:3] == self.best[:3] else 0.004)


def test_ragged_tuner_tries_splits_on_the_fastest_shapes(tmp_path, monkeypatch):
    from paper_0809_1833_amd import tune
    monkeypatch.setenv("MP_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(tune, "workload_key", lambda dec, arch=None: "ragged|test")
    monkeypatch.setattr(torch, "empty", lambda *a, **k: None)
    shapes = [(256, 1, 1), (512, 2, 1), (1024, 4, 2), (256, 2, 2)]
    # best: a split other than the default, on a shape only a little ahead at the default
    dec = FakeRaggedDecoder((512, 2, 1, 4))
    res = tune.tune_ragged(dec, torch.zeros(4), 1e-5, [5, 5, 5], reps=1, shapes=shapes)
    n_other = len(tune.SPLITS) - 1
    assert len(res["timings"]) == len(shapes) + min(len(shapes), tune.SPLIT_SHAPES) * n_other
    assert res["config"] == dict(threads=512, cols_per_wave=2, wgs_per_cu=1, split=4)
