"""Host logic of the plan search (no GPU): the staged search visits only
valid plans, covers every tile shape, and finds the optimum of separable
cost models within the two best shapes."""
import itertools

import pytest

from paper_2509_12138_amd import autotune


def cost_model(seed):
    # separable: a cost per tile shape, schedule, chunk, waves and sums
    import random
    r = random.Random(seed)
    tiles = {t: r.uniform(1, 3) for t in autotune.TILES}
    sched = {s: r.uniform(0, 1) for s in autotune.SCHEDULES}
    chunk = {c: r.uniform(0, 1) for c in (0, 64, 128)}
    waves = {w: r.uniform(0, 1) for w in (1, 2, 4)}
    det = {d: r.uniform(0, 1) for d in (False, True)}
    return lambda p: tiles[p[0]] + sched[p[1]] + chunk[p[2]] + waves[p[3]] + det[p[4]]


@pytest.mark.parametrize("seed,stored", [(s, st) for s in range(6) for st in (True, False)])
def test_staged_search_valid_plans_and_best(seed, stored):
    f = cost_model(seed)
    seen = []

    def measure(plan):
        plan = autotune.normalize(plan)
        if not stored and plan[2]:
            return None
        assert autotune.valid(plan), plan
        seen.append(plan)
        return f(plan)

    autotune.staged_search(measure, stored)
    assert {p[0] for p in seen} == set(autotune.TILES)
    # every valid plan of the two best shapes (by their first plan) ...
    first = {}
    for p in seen:
        first.setdefault(p[0], f(p))
    top = sorted(first, key=first.get)[:2]
    space = [p for p in itertools.product(top, autotune.SCHEDULES, (0, 64, 128), (1, 2, 4),
                                          (False, True))
             if autotune.valid(p) and (stored or p[2] == 0)]
    best_seen = min(f(p) for p in seen)
    # ... a separable model's optimum among them is found by the coordinate
    # steps, up to the coupling of the schedule with the forward waves
    assert best_seen <= min(f(p) for p in space) + 1.0
    assert len(seen) < 60
