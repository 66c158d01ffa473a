"""Pins of the oracle's paper emission rule (section 2.2: E_SEE, the
two-daughter split), each against a closed form on the flat plane, where
every daughter escapes unobstructed (its escape polar angle is its angle
from the normal, its escaped energy its birth energy)."""
import math

import numpy as np
import pytest

import foamgen as fg

KS1 = 1.63  # Kolmogorov-Smirnov critical value at 1 % (times 1/sqrt(n))
ES = 100.0  # constant E_SEE of the table (eV)


def _flat(oracle_lib, const, esee, E0=500.0, n=20000, seed=41, **kw):
    tab = fg.make_tables("constant", const=const, emission="paper", esee_const=esee)
    return oracle_lib.trace(fg.flat_plane(), tab, E0, 0.0, n, seed=seed, max_gen=1, per_primary=True, **kw)


def test_lone_daughter_gets_E_SEE_exactly(oracle_lib):
    n = 5000
    r = _flat(oracle_lib, 1.0, ES, n=n, n_ebins=500, n_abins=90)
    assert r["n_escaped"] == n
    assert np.all(r["per_primary"]["e_esc"] == ES)
    assert np.all(r["per_primary"]["e_dep"] == 500.0 - ES)
    # all in the bin of 100 eV; cosine-law directions
    assert r["e_hist"][100] == n
    b = np.deg2rad(np.linspace(0, 90, 91))
    emp = np.concatenate([[0], np.cumsum(r["a_hist"])]) / n
    assert np.max(np.abs(emp - np.sin(b) ** 2)) < KS1 / math.sqrt(n)


def _pair_sum_cdf(y):
    """CDF of E1 + E2 = E_SEE (s + 1 - s^2), s = sqrt(xi), xi uniform, in units of E_SEE."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros_like(y)
    inside = (y >= 1.0) & (y < 1.25)
    r = np.sqrt(np.clip(1.0 - 4.0 * (y - 1.0), 0.0, None))
    s1, s2 = (1.0 - r) / 2.0, (1.0 + r) / 2.0
    out[inside] = (s1 ** 2 + 1.0 - s2 ** 2)[inside]
    out[y >= 1.25] = 1.0
    return out


def test_pair_energies_share_one_xi(oracle_lib):
    """Two daughters: E1 = E_SEE sqrt(xi), E2 = (1 - xi) E_SEE with the same xi.
    Their sum per primary lies in [E_SEE, 1.25 E_SEE] with a closed-form law;
    drawing E2 from an independent xi would spread it over [0, 2 E_SEE]."""
    n = 20000
    r = _flat(oracle_lib, 2.0, ES, n=n, n_ebins=500)
    assert r["n_escaped"] == 2 * n
    s = np.sort(r["per_primary"]["e_esc"] / ES)
    assert s[0] >= 1.0 - 1e-12 and s[-1] <= 1.25 + 1e-12
    emp = np.arange(1, n + 1) / n
    assert np.max(np.abs(emp - _pair_sum_cdf(s))) < KS1 / math.sqrt(n)
    # escaped-energy histogram: the mixture of the laws of E1 (CDF (e/E_SEE)^2)
    # and E2 (uniform on [0, E_SEE])
    edges = np.linspace(0, 500.0, 501)
    u = np.clip(edges / ES, 0, 1)
    cdf = 0.5 * u ** 2 + 0.5 * u
    emp_e = np.concatenate([[0], np.cumsum(r["e_hist"])]) / (2 * n)
    assert np.max(np.abs(emp_e - cdf)) < KS1 / math.sqrt(n)


def test_pair_angles_are_complementary_cosine_laws(oracle_lib):
    """beta1 = asin(sqrt(xi)) is a cosine law; beta2 = pi/2 - beta1 has
    sin^2 beta2 = 1 - xi, also uniform: both escape angles follow P(beta < b) =
    sin^2 b."""
    n = 20000
    r = _flat(oracle_lib, 2.0, ES, n=n, n_abins=180)
    b = np.deg2rad(np.linspace(0, 90, 181))
    emp = np.concatenate([[0], np.cumsum(r["a_hist"])]) / (2 * n)
    assert np.max(np.abs(emp - np.sin(b) ** 2)) < KS1 / math.sqrt(n)


def test_three_daughters_are_a_pair_and_a_lone_one(oracle_lib):
    n = 10000
    r = _flat(oracle_lib, 3.0, ES, n=n)
    assert r["n_escaped"] == 3 * n
    s = np.sort(r["per_primary"]["e_esc"] / ES - 1.0)  # the lone daughter adds E_SEE
    assert s[0] >= 1.0 - 1e-12 and s[-1] <= 1.25 + 1e-12
    emp = np.arange(1, n + 1) / n
    assert np.max(np.abs(emp - _pair_sum_cdf(s))) < KS1 / math.sqrt(n)


@pytest.mark.parametrize("esee,expect", [(-5.0, 0.0), (1000.0, 500.0)])
def test_energies_are_clamped_to_what_is_available(oracle_lib, esee, expect):
    n = 2000
    r = _flat(oracle_lib, 1.0, esee, n=n)
    assert r["n_escaped"] == n
    assert np.all(r["per_primary"]["e_esc"] == expect)
    assert np.all(r["per_primary"]["e_esc"] + r["per_primary"]["e_dep"] == 500.0)


@pytest.mark.parametrize("E0", [100.0, 400.0, 1000.0])
def test_paper_tungsten_flat_curve(oracle_lib, E0):
    """The paper's own fits end to end: a flat tungsten surface at normal
    incidence returns Eq. seey's yield (1.49 near 400 eV)."""
    tab = fg.make_tables("paper_w")
    assert tab.emission == 1
    n = 40000
    r = oracle_lib.trace(fg.flat_plane(), tab, E0, 0.0, n, seed=17, max_gen=6)
    ref = float(fg.bilinear_reference(tab, E0, 0.0))
    assert abs(ref - fg.paper_w_yield(E0, 0.0)) < 0.01
    f = ref - math.floor(ref)
    assert abs(r["yield"] - ref) <= 3.0 * math.sqrt(f * (1 - f) / n)


def _slot_clear(x, beta, w, h):
    """Probability over a uniform azimuth that a ray leaving the slot floor at
    x (0 <= x <= w) with polar angle beta clears walls of height h."""
    R = h * np.tan(beta)
    with np.errstate(divide="ignore", invalid="ignore"):
        hi = np.where(R > 0, np.clip((w - x) / R, -1, 1), 1.0)
        lo = np.where(R > 0, np.clip(-x / R, -1, 1), -1.0)
    return (np.arccos(lo) - np.arccos(hi)) / np.pi


def test_pair_angles_are_complementary_in_a_slot(oracle_lib):
    """In a slot, whether the two daughters escape together depends on how
    their angles pair: with beta2 = pi/2 - beta1 one leaves steeply when the
    other grazes.  P(both escape) from a quadrature of the slot geometry:
    0.366 for the paper's pairing, 0.433 if beta2 = beta1."""
    w, h, tw = 2.0, 3.0, 1.0
    x = (np.arange(2000) + 0.5) / 2000 * w
    xi = (np.arange(4000) + 0.5) / 4000
    X, XI = np.meshgrid(x, xi, indexing="ij")
    b1 = np.arcsin(np.sqrt(XI))
    both = float((_slot_clear(X, b1, w, h) * _slot_clear(X, np.pi / 2 - b1, w, h)).mean())
    p2 = tw / (w + tw) + w / (w + tw) * both  # wall tops: both always escape
    n = 40000
    tab = fg.make_tables("constant", const=2.0, emission="paper", esee_const=ES)
    r = oracle_lib.trace(fg.trench(w=w, h=h, tw=tw), tab, 500.0, 0.0, n, seed=43, max_gen=1, per_primary=True)
    est = float((r["per_primary"]["escaped"] == 2).mean())
    assert abs(est - p2) <= 4.0 * math.sqrt(p2 * (1 - p2) / n), (est, p2)
