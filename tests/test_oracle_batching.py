"""Pins of the query batching of Sec. 6 (oracle side, CPU).

* Fig. 2 worked by hand (tests/golden/fig2_greedy.txt): the free merge of the
  first two groups costs the 180 interactions the paper states; Min and Max
  batch sizes and totals for several bounds; Periodic totals of Fig. 2;
* the structure of free merges: a merge adds no interactions only when the
  two candidate ranges are identical and their hull adds no bin, so the
  groups of the first pass lie inside the runs of identical ranges, keep
  their members' range, and no two neighbours merge for free (checked on
  random inputs);
* special cases: Min with bound 1 keeps the first pass; a bound of at least
  |Q| gives one batch; with pairwise different ranges Min is Periodic;
* invariants of the second pass on random inputs (greedy minimality for Min,
  maximality for Max, contiguous partition in t_start order);
* planted slips (Min with <=, the literal Max swap, no first pass) each break
  a Fig. 2 pin;
* candidate ranges and two-segment GreedySetSplit cases worked by hand on
  Fig. 1's bins (tests/golden/fig1_sec4_ranges.txt): a bin that starts
  before the interval ends but ends before it starts is not a candidate
  bin, and two segments with identical ranges merge for free only if their
  hull adds no bin; the superset range "first bin ending after a .. last bin
  starting before b" (a planted slip) breaks these pins.
"""
import numpy as np
import pytest

from golden_io import fig1, fig1_sec4, fig2, fig2_greedy
from oracle import batching as ob


def _fig2_setup():
    t0, t1, _, _ = fig1()
    o = ob.entry_order(t0)
    bins = ob.bin_table(t0[o], t1[o], 4)
    batches, _ = fig2()
    qa = np.concatenate([[a] * n for n, a, b in batches])
    qb = np.concatenate([[b] * n for n, a, b in batches])
    return bins, qa, qb


def test_fig1_bins():
    bins, _, _ = _fig2_setup()
    assert list(bins.first) == [0, 6, 9, 12] and list(bins.last) == [5, 8, 11, 14]
    assert list(bins.start) == [0.0, 3.9, 6.5, 9.3]


def test_fig2_periodic_totals():
    bins, qa, qb = _fig2_setup()
    _, totals = fig2()
    for s, (want, _printed) in totals.items():
        assert ob.total_interactions(bins, ob.periodic(bins, qa, qb, s)) == want


def test_fig2_free_merge_of_first_twenty():
    bins, qa, qb = _fig2_setup()
    groups = ob.free_merges(bins, ob.singletons(bins, qa, qb))
    assert groups[0].n == 20 and ob.num_ints(bins, groups[0]) == 180  # Sec. 6 states 180
    assert [g.n for g in groups] == [20, 10, 10, 10, 10]


def test_fig2_greedy_golden():
    bins, qa, qb = _fig2_setup()
    rows = fig2_greedy()
    assert len(rows) == 10
    for variant, bound, sizes, total in rows:
        got = ob.greedy_set_split(bins, qa, qb, bound, variant)
        assert [b.n for b in got] == sizes, (variant, bound)
        assert ob.total_interactions(bins, got) == total, (variant, bound)


def _random_case(seed, n_e=400, n_q=300, m=37):
    rng = np.random.default_rng(seed)
    t0 = np.round(rng.uniform(0, 100, n_e), 1)
    t1 = t0 + np.round(rng.exponential(3.0, n_e), 1) + 0.1
    o = ob.entry_order(t0)
    bins = ob.bin_table(t0[o], t1[o], m)
    # query starts on a coarse grid so that equal ranges occur in runs
    qa = np.round(rng.uniform(-5, 105, n_q) / 2.0) * 2.0
    qb = qa + rng.choice([0.5, 1.0, 2.0, 6.0], n_q)
    return bins, qa, qb


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_free_merges_within_runs_of_identical_ranges(seed):
    """A free merge needs identical ranges, so each group of the first pass
    lies inside one maximal run of identical per-segment ranges; a run splits
    further only where the hull of the group so far reaches a bin that none
    of its members overlaps (Fig. 1 has such a case)."""
    bins, qa, qb = _random_case(seed)
    one = ob.singletons(bins, qa, qb)
    rng_of = [ob.batch_range(bins, b) for b in one]
    run_start = [k == 0 or rng_of[k - 1] != rng_of[k] for k in range(len(one))]
    groups = ob.free_merges(bins, one)
    starts = {g.pos for g in groups}
    assert all(k in starts for k in range(len(one)) if run_start[k])
    for g in groups:
        assert not any(run_start[k] for k in range(g.pos + 1, g.pos + g.n))
    assert len(groups) < len(one)  # the case has runs to merge
    # free merges add no interactions
    assert ob.total_interactions(bins, groups) == ob.total_interactions(bins, one)


def test_special_cases():
    bins, qa, qb = _random_case(4)
    one = ob.singletons(bins, qa, qb)
    groups = ob.free_merges(bins, one)
    for v in ("min", "max"):
        assert [b.n for b in ob.greedy_set_split(bins, qa, qb, 1, "min")] == [g.n for g in groups]
        single = ob.greedy_set_split(bins, qa, qb, len(one), v)
        assert len(single) == 1 and single[0].n == len(one)
    # pairwise different ranges: no free merge, Min with bound s is Periodic(s)
    t0 = np.arange(40, dtype=float)
    t1 = t0 + 1.0
    b2 = ob.bin_table(t0, t1, 40)
    qa2 = np.arange(0.25, 39, 1.0)
    qb2 = qa2 + np.linspace(0.1, 3.0, qa2.size)  # ends in different bins
    one2 = ob.singletons(b2, qa2, qb2)
    assert len(set(ob.batch_range(b2, b) for b in one2)) == len(one2)
    for s in (1, 3, 7):
        g = ob.greedy_set_split(b2, qa2, qb2, s, "min")
        p = ob.periodic(b2, qa2, qb2, s)
        assert [(b.pos, b.n) for b in g] == [(b.pos, b.n) for b in p]


@pytest.mark.parametrize("seed", [5, 6])
@pytest.mark.parametrize("bound", [2, 7, 40])
def test_second_pass_invariants(seed, bound):
    bins, qa, qb = _random_case(seed)
    one = ob.singletons(bins, qa, qb)
    groups = ob.free_merges(bins, one)
    starts = {g.pos for g in groups}
    for v in ("min", "max"):
        bs = ob.greedy_set_split(bins, qa, qb, bound, v)
        # contiguous partition of the ordered list, made of whole groups
        pos = 0
        for b in bs:
            assert b.pos == pos and b.pos in starts
            pos += b.n
        assert pos == len(one)
        for k, b in enumerate(bs):
            inner = sorted(g.pos for g in groups if b.pos <= g.pos < b.pos + b.n)
            last_group = [g for g in groups if g.pos == inner[-1]][0]
            if v == "min":
                if k < len(bs) - 1:
                    assert b.n >= bound
                if len(inner) > 1:  # the batch took its last group only while short
                    assert b.n - last_group.n < bound
            else:
                if len(inner) > 1:
                    assert b.n <= bound
                if k < len(bs) - 1:  # the next group did not fit
                    nxt = [g for g in groups if g.pos == b.pos + b.n][0]
                    assert b.n + nxt.n > bound


def test_planted_slips_are_caught():
    bins, qa, qb = _fig2_setup()
    rows = {(v, bd): (sizes, tot) for v, bd, sizes, tot in fig2_greedy()}

    def second_pass(groups, keep_merging):
        out, cur = [], groups[0]
        for nxt in groups[1:]:
            if keep_merging(cur, nxt):
                cur = cur.merged(nxt)
            else:
                out.append(cur)
                cur = nxt
        return out + [cur]

    groups = ob.free_merges(bins, ob.singletons(bins, qa, qb))
    # Min with <= instead of <
    slip = second_pass(groups, lambda c, n: c.n <= 20)
    assert [b.n for b in slip] != rows[("min", 20)][0]
    # Max read literally as "merge while the batch holds at most bound"
    slip = second_pass(groups, lambda c, n: c.n <= 10)
    assert [b.n for b in slip] != rows[("max", 10)][0]
    # no first pass
    slip = second_pass(ob.singletons(bins, qa, qb), lambda c, n: c.n < 1)
    assert [b.n for b in slip] != rows[("min", 1)][0]


def _fig1_bins():
    t0, t1, _, _ = fig1()
    o = ob.entry_order(t0)
    return ob.bin_table(t0[o], t1[o], 4)


def _pin_fig1_sec4(candidate_range):
    """Failures of the hand-worked Fig. 1 cases under a candidate-range function."""
    bins = _fig1_bins()
    ranges, greedy = fig1_sec4()
    fails = []
    for a, b, f, l in ranges:
        got = candidate_range(bins, a, b)
        want = None if l < f else (f, l)
        if got != want:
            fails.append(f"range ({a}, {b}): {got} != {want}")
    for variant, bound, segs, sizes, total in greedy:
        qa = np.array([x[0] for x in segs])
        qb = np.array([x[1] for x in segs])
        got = ob.greedy_set_split(_fig1_bins(), qa, qb, bound, variant)
        if [x.n for x in got] != sizes or ob.total_interactions(_fig1_bins(), got) != total:
            fails.append(f"greedy {variant} {bound} {segs}: {[x.n for x in got]}")
    return fails


def test_fig1_sec4_ranges_and_merges():
    assert _pin_fig1_sec4(ob.candidate_range) == []


def test_superset_range_slip_is_caught(monkeypatch):
    """The superset range (first bin whose running maximum end exceeds a ..
    last bin whose start is below b) takes bins that end before the interval
    starts; it must break the Fig. 1 pins."""
    def superset(bins, a, b):
        runmax = np.maximum.accumulate(bins.end)
        j1 = int(np.searchsorted(runmax, a, side="right"))
        j2 = int(np.searchsorted(bins.start, b, side="left")) - 1
        if j1 > j2 or j1 >= bins.start.size or j2 < 0:
            return None
        return int(bins.first[j1]), int(bins.last[j2])
    monkeypatch.setattr(ob, "candidate_range", superset)
    assert _pin_fig1_sec4(superset) != []


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_candidate_range_brute_force(seed):
    """Against a direct scan of the entries: the range is the index hull of
    every entry in an overlapping bin, and it holds every entry whose span
    overlaps the interval."""
    rng = np.random.default_rng(seed)
    n = 300
    t0 = np.round(rng.uniform(0, 40, n), 1)
    t1 = t0 + np.round(rng.exponential(4.0, n), 1) + 0.1
    o = ob.entry_order(t0)
    e0, e1 = t0[o], t1[o]
    m = 23
    bins = ob.bin_table(e0, e1, m)
    width = (e1.max() - e0[0]) / m
    j = np.clip(np.floor((e0 - e0[0]) / width), 0, m - 1).astype(int)
    for a, b in zip(rng.uniform(-3, 45, 200), rng.uniform(0.05, 5, 200)):
        b = a + b
        members = []
        for k in np.unique(j):
            mk = np.nonzero(j == k)[0]
            if e0[mk].min() < b and e1[mk].max() > a:
                members.extend(mk.tolist())
        got = ob.candidate_range(bins, a, b)
        if not members:
            assert got is None
            continue
        assert got == (min(members), max(members))
        ov = np.nonzero((e0 < b) & (e1 > a))[0]
        assert ov.size == 0 or (got[0] <= ov.min() and ov.max() <= got[1])


def test_free_merge_structure():
    """After the first pass every group's range equals each member's own range
    (a free merge keeps the range), and merging two neighbouring groups would
    add interactions."""
    for seed in (1, 2, 3):
        bins, qa, qb = _random_case(seed)
        one = ob.singletons(bins, qa, qb)
        groups = ob.free_merges(bins, one)
        for g in groups:
            r = ob.batch_range(bins, g)
            for k in range(g.pos, g.pos + g.n):
                assert ob.batch_range(bins, one[k]) == r
        for g, h in zip(groups, groups[1:]):
            assert ob.num_ints(bins, g.merged(h)) > ob.num_ints(bins, g) + ob.num_ints(bins, h)
