"""The four-way co-rank selection, as a plain model, against brute force.

The four-way merge passes find each tile's co-ranks by selecting the shares
of four sorted runs among their d smallest elements in the order (key, run),
by stride halving (the co-rank kernel of the four-way pass).  This model
restates the algorithm step by step so that its logic (the count per
level, the candidates below the largest selected sample, the removals and
the sentinels past a run's end) is checked on the CPU against the plain
definition; the GPU tests check the kernel through every four-way sort.
Test code only: neither the library nor the oracle uses it.
"""
import random

import pytest


def _at(runs, r, j):
    # element j of run r in the order (key, run); past the end a sentinel,
    # after every element, sentinels of different runs ordered by r
    return (0, runs[r][j], r) if j < len(runs[r]) else (1, r, 0)


def select_model(runs, d, read_ahead=32):
    """Shares (w_0..w_3) of the four runs among the d smallest elements, and
    the number of dependent rounds of reads."""
    widths = [len(x) for x in runs]
    lg = 0
    while (1 << lg) < max(widths):
        lg += 1
    w = [0] * 4
    top = [None] * 4          # each run's largest selected sample
    rounds = 0
    for lev in range(lg, -1, -1):
        s = 1 << lev
        target = d >> lev     # floor(d / s) samples selected at stride s
        base = [2 * x for x in w]
        w = base[:]
        old_top = top[:]
        cand = [_at(runs, r, (base[r] + 1) * s - 1) for r in range(4)]
        ahead = [base[r] > 0 and s < read_ahead for r in range(4)]
        before = [_at(runs, r, (base[r] - 1) * s - 1) if ahead[r] else None for r in range(4)]
        rounds += 1
        sel = [r for r in range(4) if w[r] > 0]
        if sel:
            y = max(top[r] for r in sel)
            for r in range(4):
                if cand[r] < y:
                    w[r] += 1
                    top[r] = cand[r]
        cnt = sum(w)
        while cnt > target:   # at most three times
            r = max((r for r in range(4) if w[r] > 0), key=lambda r: top[r])
            w[r] -= 1
            cnt -= 1
            if w[r] > 0:
                q = w[r] - base[r]
                if q == 0:
                    top[r] = old_top[r]
                elif q == -1 and ahead[r]:
                    top[r] = before[r]
                else:
                    top[r] = _at(runs, r, w[r] * s - 1)
                    rounds += 1
        while cnt < target:   # one candidate, or several at the first level
            nxt = [(cand[r] if w[r] == base[r] else (1, r, 0), r) for r in range(4)]
            e, r = min(nxt)
            w[r] += 1
            top[r] = e
            cnt += 1
    return w, rounds


def brute(runs, d):
    order = sorted((v, r, j) for r in range(4) for j, v in enumerate(runs[r]))
    w = [0] * 4
    for v, r, j in order[:d]:
        w[r] += 1
    return w


@pytest.mark.parametrize("seed", range(6))
def test_selection_matches_brute_force(seed):
    rng = random.Random(seed)
    for _ in range(400):
        key_range = rng.choice([1, 2, 5, 50, 10 ** 6])
        runs = [sorted(rng.randrange(key_range)
                       for _ in range(rng.choice([0, 1, 2, 3, 4, 7, 8, 9, 16, 17, 33,
                                                  rng.randrange(0, 150)])))
                for _ in range(4)]
        n = sum(map(len, runs))
        for d in sorted({0, n, rng.randrange(n + 1), rng.randrange(n + 1)}):
            got, _ = select_model(runs, d)
            assert got == brute(runs, d), (runs, d)
            # the read-ahead only saves rounds, it never changes the result
            assert select_model(runs, d, read_ahead=1)[0] == got


def test_selection_rounds_are_logarithmic():
    # one round of reads per level (13 levels for runs of 4096), plus the
    # removals that need a read of their own: well under the nested
    # bisection's ~13 * 14 / 2 dependent probes
    rng = random.Random(9)
    total = 0
    for _ in range(20):
        runs = [sorted(rng.randrange(1 << 30) for _ in range(4096)) for _ in range(4)]
        d = rng.randrange(4 * 4096 + 1)
        w, rounds = select_model(runs, d)
        assert w == brute(runs, d)
        assert 13 <= rounds <= 2 * 13
        total += rounds
    assert total / 20 < 1.6 * 13


def corank_model(runs, d):
    """The four-way co-rank as the kernel takes it: if the runs' ranges do
    not overlap in run order, or in reverse run order, the shares fill the
    runs in that order; else the selection."""
    def first(r):
        return _at(runs, r, 0)

    def last(r):
        return _at(runs, r, len(runs[r]) - 1) if runs[r] else _at(runs, r, 0)
    nonempty = [r for r in range(4) if runs[r]]
    up = all(last(a) < first(b) for a, b in zip(nonempty, nonempty[1:]))
    rev = nonempty[::-1]
    down = all(last(a) < first(b) for a, b in zip(rev, rev[1:]))
    if up or down:
        w, rem = [0] * 4, d
        for r in (range(4) if up else range(3, -1, -1)):
            w[r] = min(rem, len(runs[r]))
            rem -= w[r]
        return w
    return select_model(runs, d)[0]


@pytest.mark.parametrize("seed", range(4))
def test_disjoint_runs_fast_path_matches_brute_force(seed):
    rng = random.Random(100 + seed)
    for _ in range(400):
        kind = rng.choice(["up", "down", "equal", "random", "touching"])
        lens = [rng.choice([0, 1, 2, 5, 16, rng.randrange(0, 60)]) for _ in range(4)]
        if kind == "up":        # presorted: run r holds keys above run r - 1's
            runs = [sorted(rng.randrange(100 * r, 100 * r + 100) for _ in range(n))
                    for r, n in enumerate(lens)]
        elif kind == "down":    # reverse-sorted: run r holds keys below run r - 1's
            runs = [sorted(rng.randrange(400 - 100 * r, 500 - 100 * r) for _ in range(n))
                    for r, n in enumerate(lens)]
        elif kind == "equal":   # one value everywhere: ties broken by run
            runs = [[7] * n for n in lens]
        elif kind == "touching":  # neighbouring runs share their boundary key
            runs = [sorted([10 * r] * (n // 2) + [10 * (r + 1)] * (n - n // 2))
                    for r, n in enumerate(lens)]
        else:
            runs = [sorted(rng.randrange(50) for _ in range(n)) for n in lens]
        n = sum(lens)
        for d in sorted({0, n, rng.randrange(n + 1), rng.randrange(n + 1)}):
            assert corank_model(runs, d) == brute(runs, d), (kind, runs, d)
