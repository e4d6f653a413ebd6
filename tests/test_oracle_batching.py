"""Pins of the query batching of Sec. 6 (oracle side, CPU).

* Fig. 2 worked by hand (tests/golden/fig2_greedy.txt): the free merge of the
  first two groups costs the 180 interactions the paper states; Min and Max
  batch sizes and totals for several bounds; Periodic totals of Fig. 2;
* the structure of free merges: a merge adds no interactions exactly when
  the two candidate ranges are identical, so the first pass gives the
  maximal runs of identical ranges (checked on random inputs);
* special cases: Min with bound 1 keeps the first pass; a bound of at least
  |Q| gives one batch; with pairwise different ranges Min is Periodic;
* invariants of the second pass on random inputs (greedy minimality for Min,
  maximality for Max, contiguous partition in t_start order);
* planted slips (Min with <=, the literal Max swap, no first pass) each break
  a Fig. 2 pin.
"""
import numpy as np
import pytest

from golden_io import fig1, fig2, fig2_greedy
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
def test_free_merges_are_runs_of_identical_ranges(seed):
    bins, qa, qb = _random_case(seed)
    one = ob.singletons(bins, qa, qb)
    rng_of = [ob.batch_range(bins, b) for b in one]
    runs = []
    for k, r in enumerate(rng_of):
        if runs and rng_of[k - 1] == r:
            runs[-1] += 1
        else:
            runs.append(1)
    groups = ob.free_merges(bins, one)
    assert [g.n for g in groups] == runs
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
