"""Planted mistakes: every plausible slip in the oracle must trip a pin.

Each case copies the oracle's C source with one change, builds the copy with
gcc in a temporary directory and runs one of the independent pins against
it.  The pin must reject the mutant (and, as a control, accept the real
oracle in the pin tests).
"""
import math
import os

import numpy as np
import pytest

import foamgen as fg
import oracle
from tests.exact_hit import exact_first_hit
from tests.philox_ref import load_kat

SRC = os.path.join(os.path.dirname(oracle.__file__), "rtmc_oracle.c")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _build_variant(tmp_path, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    oracle.compile_source(str(path), so)
    return oracle.Variant(so)


# ---- pins, each returning True when the oracle under test passes

def pin_exact_first_hit(o):
    for seed in (0, 1):
        m = fg.random_soup(48, seed=seed)
        m.flags = 0
        rng = np.random.default_rng(100 + seed)
        lo, hi = np.array(m.box_lo), np.array(m.box_hi)
        org = lo + (hi - lo) * (rng.integers(1, 64, size=(120, 3)) / 64.0)
        d = rng.normal(size=(120, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        rays = np.concatenate([org, d], axis=1)
        tri, t, _ = o.first_hit(m, rays)
        for i in range(len(rays)):
            eid, et = exact_first_hit(m.verts, m.tris, m.box_lo, m.box_hi, False, rays[i])
            if tri[i] != eid or abs(t[i] - float(et)) > 1e-12 * max(1.0, float(et)):
                return False
    return True


def pin_flat_yield(o):
    tab = fg.make_tables("vaughan")
    for E, th in ((500.0, 0.0), (100.0, 30.0), (1000.0, 60.0)):
        n = 20000
        r = o.trace(fg.flat_plane(), tab, E, th, n, seed=11, max_gen=6)
        ref = float(fg.bilinear_reference(tab, E, th))
        f = ref - math.floor(ref)
        if abs(r["yield"] - ref) > 3.0 * math.sqrt(f * (1 - f) / n):
            return False
    return True


def pin_cosine_law(o):
    tab = fg.make_tables("constant", const=1.0)
    n = 20000
    r = o.trace(fg.flat_plane(), tab, 200.0, 0.0, n, seed=5, max_gen=1, n_abins=90)
    b = np.deg2rad(np.linspace(0, 90, 91))
    emp = np.concatenate([[0], np.cumsum(r["a_hist"])]) / n
    return bool(np.max(np.abs(emp - np.sin(b) ** 2)) < 1.63 / math.sqrt(n))


def pin_conservation(o):
    m = fg.make_grf_foam(10, 0.6, 2.0, seed=3)
    r = o.trace(m, fg.make_tables("vaughan"), 800.0, -80.0, 500, seed=9, per_primary=True)
    pp = r["per_primary"]
    return bool(np.allclose(pp["e_esc"] + pp["e_dep"], 800.0, rtol=1e-9, atol=0))


def pin_trench(o):
    tab = fg.make_tables("vaughan")
    n = 20000
    r = o.trace(fg.trench(), tab, 500.0, 0.0, n, seed=21, max_gen=1)
    d0 = float(fg.bilinear_reference(tab, 500.0, 0.0))
    F = math.sqrt(1 + 1.5 ** 2) - 1.5
    expect = d0 * (1 / 3 + 2 / 3 * F)
    return abs(r["yield"] - expect) <= 3.0 * max(r["yield_sigma"], 1e-9)


def pin_philox(o):
    return all(list(o.philox4x32_10(c, k)) == out for c, k, out in load_kat(os.path.join(GOLD, "philox4x32_10_kat.txt")))


def _paper_flat(o, const, n, seed=41):
    tab = fg.make_tables("constant", const=const, emission="paper", esee_const=100.0)
    return o.trace(fg.flat_plane(), tab, 500.0, 0.0, n, seed=seed, max_gen=1, per_primary=True)


def pin_paper_lone(o):
    r = _paper_flat(o, 1.0, 2000)
    return bool(np.all(r["per_primary"]["e_esc"] == 100.0))


def pin_paper_pair_sum(o):
    from tests.test_oracle_paper_mode import _pair_sum_cdf
    n = 20000
    r = _paper_flat(o, 2.0, n)
    s = np.sort(r["per_primary"]["e_esc"] / 100.0)
    if s[0] < 1.0 - 1e-12 or s[-1] > 1.25 + 1e-12:
        return False
    return bool(np.max(np.abs(np.arange(1, n + 1) / n - _pair_sum_cdf(s))) < 1.63 / math.sqrt(n))


def pin_paper_slot(o):
    from tests.test_oracle_paper_mode import _slot_clear
    w, h, tw = 2.0, 3.0, 1.0
    x = (np.arange(1000) + 0.5) / 1000 * w
    xi = (np.arange(2000) + 0.5) / 2000
    X, XI = np.meshgrid(x, xi, indexing="ij")
    b1 = np.arcsin(np.sqrt(XI))
    p2 = tw / (w + tw) + w / (w + tw) * float((_slot_clear(X, b1, w, h) * _slot_clear(X, np.pi / 2 - b1, w, h)).mean())
    n = 40000
    tab = fg.make_tables("constant", const=2.0, emission="paper", esee_const=100.0)
    r = o.trace(fg.trench(w=w, h=h, tw=tw), tab, 500.0, 0.0, n, seed=43, max_gen=1, per_primary=True)
    est = float((r["per_primary"]["escaped"] == 2).mean())
    return abs(est - p2) <= 4.0 * math.sqrt(p2 * (1 - p2) / n)


def pin_cutoff(o):
    from tests.test_oracle_pins import _cutoff_slot, _slot_one_bounce
    for E0 in (5.0, 10.0):
        r = o.trace(fg.flat_plane(), fg.make_tables("constant", const=1.0, Ec=10.0), E0, 0.0, 500, seed=3)
        if r["n_escaped"] != 0:
            return False
    n = 40000
    p = _slot_one_bounce()
    return abs(_cutoff_slot(o, n, max_gen=6)["yield"] - p) <= 3.0 * math.sqrt(p * (1 - p) / n)


def pin_sigma(o):
    tab = fg.make_tables("vaughan")
    n = 40000
    for E, th in ((500.0, 0.0), (60.0, 80.0)):
        r = o.trace(fg.flat_plane(), tab, E, th, n, seed=11, max_gen=6)
        ref = float(fg.bilinear_reference(tab, E, th))
        f = ref - math.floor(ref)
        exact = math.sqrt(f * (1 - f) / n)
        if abs(r["yield_sigma"] - exact) > 0.03 * exact:
            return False
    return True


def pin_substrate(o):
    from tests.test_oracle_pins import _empty_substrate_cell
    tab = fg.make_tables("vaughan")
    n = 20000
    for E, th in ((500.0, 0.0), (100.0, 50.0)):
        r = o.trace(_empty_substrate_cell(), tab, E, th, n, seed=13, max_gen=6)
        ref = float(fg.bilinear_reference(tab, E, th))
        f = ref - math.floor(ref)
        if abs(r["yield"] - ref) > 3.0 * math.sqrt(f * (1 - f) / n):
            return False
    return True


MUTANTS = [
    ("cull the wrong side",
     "if (det <= DET_EPS * norm3(L1) * norm3(L2) * dn) continue;",
     "if (-det <= DET_EPS * norm3(L1) * norm3(L2) * dn) continue;", pin_exact_first_hit),
    ("printed barycentric limit u^2 + v^2 <= 1",
     "if (v < 0.0 || u + v > 1.0) continue;",
     "if (v < 0.0 || u * u + v * v > 1.0) continue;", pin_exact_first_hit),
    ("printed Cramer denominator (D x L2) . L2",
     "double det = dot3(P, L1);", "double det = dot3(P, L2) + dot3(P, L1) * 1e-30;", pin_exact_first_hit),
    ("keep the farthest hit",
     "if (best < 0 || t < bt || (t == bt && T->id < m->t[best].id)) {",
     "if (best < 0 || t > bt || (t == bt && T->id < m->t[best].id)) {", pin_exact_first_hit),
    ("stochastic rounding inverted",
     "int nd = (int)fl + (u1[0] < delta - fl ? 1 : 0);",
     "int nd = (int)fl + (u1[0] >= delta - fl ? 1 : 0);", pin_flat_yield),
    ("incidence angle as printed (obtuse)",
     "double cosa = -dot3(ray.d, p.n);", "double cosa = dot3(ray.d, p.n);", pin_flat_yield),
    ("bilinear term dropped",
     "(1 - fx) * fy * y01 + fx * fy * y11;", "(1 - fx) * fy * y01;", pin_flat_yield),
    ("sin(beta) uniform instead of sin^2(beta)",
     "double sb = sqrt(s2), cb = sqrt(1.0 - s2)", "double sb = s2, cb = sqrt(1.0 - s2 * s2)",
     pin_cosine_law),
    ("daughter energy not taken from the parent",
     "          Eav -= Ed;\n", "\n", pin_conservation),
    ("periodic re-entry through the same face",
     "p[a] = D[a] > 0.0 ? m->lo[a] : m->hi[a];", "p[a] = D[a] > 0.0 ? m->hi[a] - 1e-9 : m->lo[a] + 1e-9;",
     pin_trench),
    ("Philox key schedule dropped",
     "      k[0] += 0x9E3779B9u;\n", "\n", pin_philox),
    ("paper rule: second daughter's energy from a fresh xi",
     "Ed = (1.0 - xi_pair) * es;", "Ed = (1.0 - u[1]) * es;", pin_paper_pair_sum),
    ("paper rule: first daughter's energy without the square root",
     "Ed = es * sqrt(xi_pair);", "Ed = es * xi_pair;", pin_paper_pair_sum),
    ("paper rule: second daughter at the first one's angle",
     "s2 = 1.0 - xi_pair;", "s2 = xi_pair;", pin_paper_slot),
    ("paper rule: lone daughter's energy from the spectrum",
     "Ed = es;\n", "Ed = tab_cdf_inv(&T, u[0] * tab_cdf(&T, Eav));\n", pin_paper_lone),
    ("emission cut-off ignored",
     "if (ray.E <= T.Ec) {", "if (ray.E <= 0.0) {", pin_cutoff),
    ("emission cut-off exclusive (a ray at E_c still emits)",
     "if (ray.E <= T.Ec) {", "if (ray.E < T.Ec) {", pin_cutoff),
    ("standard error without the 1 / N",
     "res->yield_sigma = sqrt(var / N);", "res->yield_sigma = sqrt(var);", pin_sigma),
    ("variance without the squared mean",
     "double var = N > 1 ? (g_c2 - N * mean * mean) / (N - 1.0) : 0.0;",
     "double var = N > 1 ? g_c2 / (N - 1.0) : 0.0;", pin_sigma),
    ("substrate normal pointing down",
     "        r->n[2] = 1.0;\n", "        r->n[2] = -1.0;\n", pin_substrate),
]


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_rejects_planted_mistake(tmp_path, name, old, new, pin):
    mutant = _build_variant(tmp_path, old, new)
    assert not pin(mutant), f"pin {pin.__name__} did not catch: {name}"


@pytest.mark.parametrize("pin", sorted({m[3] for m in MUTANTS}, key=lambda f: f.__name__))
def test_pins_accept_the_oracle(oracle_lib, pin):
    assert pin(oracle_lib)
