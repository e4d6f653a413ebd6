"""The oracle against its pins, plus mutation checks that show the pins bite.

CPU only. Each mutant is a copy of oracle.c with one plausible slip planted
(dropped term, flipped sign, wrong operand, wrong index, a relaxed compare),
compiled elsewhere; every mutant must fail at least one pin.
"""
import numpy as np
import pytest

import gen
import oracle
from oracle.build import SRC, build
import oracle_pins

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(lib, pin):
    assert pin(lib) == []


def test_fixtures_have_content(lib):
    from gen import fixtures as fx
    db, q = fx.random_small()
    h = oracle.search(db, q, lib=lib)
    assert 5 < len(h) < h.n_overlap
    db, q = fx.dense_box()
    h = oracle.search(db, q, lib=lib)
    assert len(h) > 50


def test_c1_shape(lib):
    db, q, m = gen.make_config("C1")
    assert len(db) == 20000 and len(q) == 1000 and m == 100
    h = oracle.search(db, q, lib=lib)
    # every query segment overlaps the 200 entries of its unit time step
    assert h.n_overlap == 200 * 1000
    assert np.all(np.diff(h.q) >= 0)


def test_invalid_inputs(lib):
    from gen import fixtures as fx
    db, q = fx.random_small()
    bad = db.subset(np.arange(len(db)))
    bad.t1[3] = bad.t0[3]
    with pytest.raises(ValueError):
        oracle.search(bad, q, lib=lib)
    q2 = q.with_d(-1.0)
    with pytest.raises(ValueError):
        oracle.search(db, q2, lib=lib)
    q3 = q.subset(np.arange(len(q)))
    q3.x0[0] = np.nan
    with pytest.raises(ValueError):
        oracle.search(db, q3, lib=lib)


def test_empty_inputs(lib):
    from gen import fixtures as fx
    db, q = fx.random_small()
    h = oracle.search(db.subset(np.arange(0)), q, lib=lib)
    assert len(h) == 0 and h.n_overlap == 0
    h = oracle.search(db, q.subset(np.arange(0)), lib=lib)
    assert len(h) == 0


MUTANTS = {
    "a_drops_z": ("double a = fma(Vz, Vz, fma(Vy, Vy, Vx * Vx));",
                  "double a = fma(Vy, Vy, Vx * Vx);"),
    "B_sign": ("double B = fma(Dz, Vz, fma(Dy, Vy, Dx * Vx));",
               "double B = -fma(Dz, Vz, fma(Dy, Vy, Dx * Vx));"),
    "te_wrong_index": ("double te = tlo - e->t0;", "double te = tlo - q->t0;"),
    "overlap_not_strict": ("if (!(tlo < thi)) return -1;", "if (!(tlo <= thi)) return -1;"),
    "Vx_transposed": ("double Vx = q->vx - e->vx;", "double Vx = e->vx - q->vx;"),
    "no_vertex_test": ("int vtx = (B < 0.0) && (fma(a, T, B) > 0.0) && (fma(B, B, -(a * c)) >= 0.0);",
                       "int vtx = 0;"),
    "wrong_root": ("double a_ = in0 ? tlo : tlo + dmax(lo, 0.0);",
                   "double a_ = in0 ? tlo : tlo + dmax(hi, 0.0);"),
    "velocity_no_dt": ("s->vy = (a[5][i] - a[1][i]) / dt;", "s->vy = (a[5][i] - a[1][i]);"),
    "c_wrong_dd": ("double c = fma(Dz, Dz, fma(Dy, Dy, fma(Dx, Dx, -dd)));",
                   "double c = fma(Dz, Dz, fma(Dy, Dy, fma(Dx, Dx, -2.0 * dd)));"),
    "fT_drops_2B": ("int inT = fma(fma(a, T, B + B), T, c) <= 0.0;",
                    "int inT = fma(fma(a, T, B), T, c) <= 0.0;"),
    "thi_uses_max": ("double thi = dmin(q->t1, e->t1);", "double thi = dmax(q->t1, e->t1);"),
    "Pe_from_query": ("fma(e->vx, te, e->x0)", "fma(e->vx, te, q->x0)"),
    "dd_is_d": ("double dd = qd[i] * qd[i];", "double dd = qd[i];"),
    # the tangency collapse of reading R8: no value, and the span's start
    "collapse_nan": ("        a_ = tlo + tv;\n        b_ = a_;", "        a_ = NAN;\n        b_ = a_;"),
    "collapse_to_tlo": ("        a_ = tlo + tv;\n        b_ = a_;", "        a_ = tlo;\n        b_ = a_;"),
    "no_collapse": ("    if (a_ > b_) {", "    if (0) {"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    text = SRC.read_text()
    assert text.count(old) == 1, f"mutation site for {name} not found once"
    lib_path = build(out=tmp_path, src_text=text.replace(old, new))
    mlib = oracle.load(lib_path)
    results = oracle_pins.run_all(mlib)
    failing = [k for k, v in results.items() if v]
    assert failing, f"mutant {name} passed every pin"
