"""Host logic of the split and launch choice, without a GPU: timings within
the tie band are broken by order, a short step is timed in back-to-back
batches, a long one evaluation at a time, and the slow-split cutoff never
cuts a first run faster than its floor.  The timing functions run against a
fake workload whose evaluations advance a fake clock (torch's synchronize
replaced by a no-op)."""
import types

import pytest

from paper_2608_01467_amd import tune


def test_first_within_takes_the_first_tie():
    rows = [("a", 1.005), ("b", 1.0), ("c", 1.2)]
    assert tune.first_within(rows) == "a"              # within 1% of the fastest, listed first
    assert tune.first_within(rows, tie=0.001) == "b"   # a narrower band: the fastest
    assert tune.first_within([("x", 2.0), ("y", 1.0)]) == "y"
    assert tune.first_within([("only", 3.0)]) == "only"


class _Ctx:
    def __init__(self):
        self.launch_config = (0, 0, 0, 0)

    def set_launch_config(self, *cfg):
        self.launch_config = tuple(cfg)


class _Workload:
    """Each evaluation advances the clock by step(partition, launch); the
    first evaluation of a (partition, launch) pair also by `capture`."""

    def __init__(self, clock, step, capture=2e-3):
        self.clock, self.step, self.capture = clock, step, capture
        self.ctx = _Ctx()
        self.seen = set()
        self.calls = 0

    def run(self, partition, plain=False):
        key = (tuple(partition), self.ctx.launch_config)
        self.clock.t += self.step(tuple(partition), self.ctx.launch_config)
        if key not in self.seen:
            self.clock.t += self.capture
            self.seen.add(key)
        self.calls += 1


@pytest.fixture
def clock(monkeypatch):
    import torch
    c = types.SimpleNamespace(t=0.0)
    monkeypatch.setattr(tune, "time", types.SimpleNamespace(perf_counter=lambda: c.t))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    return c


def test_short_step_timed_in_batches(clock):
    wl = _Workload(clock, lambda p, l: 40e-6)
    t = tune.time_split(wl, (1, 2), reps=2)
    assert t == pytest.approx(40e-6)
    # the capture run, one lone run, then at least 5 batches of SHORT_BATCH
    assert wl.calls == 2 + 5 * tune.SHORT_BATCH


def test_long_step_timed_one_at_a_time(clock):
    wl = _Workload(clock, lambda p, l: 0.1)
    assert tune.time_split(wl, (1, 2), reps=3) == pytest.approx(0.1)
    assert wl.calls == 1 + 3


def test_cutoff_floor(clock):
    # a short step whose capture run exceeds the cutoff is still timed in full
    wl = _Workload(clock, lambda p, l: 40e-6)
    assert tune.time_split(wl, (1, 2), reps=2, cutoff=1e-4) == pytest.approx(40e-6)
    # a slow split past the floor is measured once, by its first run
    wl = _Workload(clock, lambda p, l: 0.2)
    t = tune.time_split(wl, (1, 2), reps=3, cutoff=0.1)
    assert t == pytest.approx(0.2 + wl.capture) and wl.calls == 1


def test_exhaustive_keeps_the_first_of_tied_splits(clock):
    times = {(1, 2): 40.0e-6, (3, 4): 39.9e-6, (5, 6): 60e-6, (7, 8): 30e-6}
    wl = _Workload(clock, lambda p, l: times[p])
    rows, best = tune.exhaustive(wl, [(1, 2), (3, 4), (5, 6)], reps=2)
    assert [c for c, _ in rows] == [(1, 2), (3, 4), (5, 6)]
    assert best == (1, 2)                       # 0.25% slower than (3, 4): a tie, listed first
    _, best = tune.exhaustive(wl, [(1, 2), (7, 8)], reps=2)
    assert best == (7, 8)                       # 25% faster: no tie


def test_autotune_launch_first_of_tied_shapes(clock):
    # interpreted shapes 0.70 ms at 4 blocks per CU and 0.75 ms otherwise;
    # compiled 35 us whatever the shape, except one lane per history at 4
    # blocks per CU (40 us): the compiled shapes are tried at the
    # interpreter's best block count (4), where two lanes per history win
    def step(p, launch):
        h, chunk, bpc, dispatch = launch
        if dispatch != 3:
            return 0.70e-3 if bpc == 4 else 0.75e-3
        return 40e-6 if (h, bpc) == (1, 4) else 35e-6
    wl = _Workload(clock, step)
    best, log = tune.autotune_launch(wl, (1, 2), reps=2)
    compiled = [(c, t) for c, t in log if c[3] == 3]
    fastest = min(t for _, t in log)
    first_tied = next(c for c, t in log if t <= fastest * (1 + tune.TIE))
    assert best == first_tied
    assert best[3] == 3 and best[0] == 2 and best[2] == 4
    assert wl.ctx.launch_config == best
    assert {c[0] for c, _ in compiled} == {1, 2} and all(c[2] == 4 for c, _ in compiled)
