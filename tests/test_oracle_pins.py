"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: every expected value comes
from a closed form, an exact rational computation, a published test vector
or an invariant of the method.
"""
import math
import os

import numpy as np
import pytest

import foamgen as fg
from tests.exact_hit import exact_first_hit
from tests.philox_ref import load_kat, philox4x32_10, uniform01

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- Philox

def test_philox_known_answers(oracle_lib):
    for ctr, key, out in load_kat(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        assert list(oracle_lib.philox4x32_10(ctr, key)) == out
        assert list(philox4x32_10(np.array(ctr), np.array(key))) == out


def test_philox_python_vs_oracle_many(oracle_lib):
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(2000, 2), dtype=np.uint64).astype(np.uint32)
    ref = philox4x32_10(ctr, key)
    for i in range(0, 2000, 97):
        assert np.array_equal(oracle_lib.philox4x32_10(ctr[i], key[i]), ref[i])


def test_philox_uniformity():
    n = 1 << 18
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint32)
    u = uniform01(philox4x32_10(ctr, np.zeros((n, 2), dtype=np.uint32))).ravel()
    assert u.min() > 0.0 and u.max() <= 1.0
    h, _ = np.histogram(u, bins=64, range=(0, 1))
    e = u.size / 64
    chi2 = ((h - e) ** 2 / e).sum()
    # 63 degrees of freedom: p = 1e-4 at about 116
    assert chi2 < 116


# --------------------------------------------------------------- first hit

def _soup_rays(mesh, n, seed):
    rng = np.random.default_rng(seed)
    lo, hi = np.array(mesh.box_lo), np.array(mesh.box_hi)
    o = lo + (hi - lo) * (rng.integers(1, 64, size=(n, 3)) / 64.0)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.concatenate([o, d], axis=1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_first_hit_matches_exact_rational(oracle_lib, seed):
    m = fg.random_soup(48, seed=seed)
    m.flags = 0  # no periodic wrap: exact checker handles one segment
    rays = _soup_rays(m, 150, 100 + seed)
    tri, t, _ = oracle_lib.first_hit(m, rays)
    n_hit = 0
    for i in range(len(rays)):
        eid, et = exact_first_hit(m.verts, m.tris, m.box_lo, m.box_hi, False, rays[i])
        assert tri[i] == eid, (i, tri[i], eid)
        assert abs(t[i] - float(et)) <= 1e-12 * max(1.0, float(et))
        n_hit += eid >= 0
    assert n_hit > 20


def test_first_hit_through_periodic_wraps(oracle_lib):
    # plane z = 1 in a 4 x 4 cell; a shallow ray must wrap in x several times
    m = fg.flat_plane(L=4.0, z0=1.0, height=4.0)
    o = np.array([3.5, 2.25, 5.0])
    d = np.array([0.99, 0.0, -math.sqrt(1 - 0.99 ** 2)])
    tri, t, w = oracle_lib.first_hit(m, np.concatenate([o, d])[None])
    t_exact = (5.0 - 1.0) / -d[2]
    x_end = o[0] + t_exact * d[0]
    assert abs(t[0] - t_exact) < 1e-9 * t_exact
    assert w[0] == int(x_end // 4.0)
    xe = x_end % 4.0
    # triangle 0 covers y <= x, triangle 1 covers y >= x (both CCW seen from +z)
    assert tri[0] == (0 if 2.25 <= xe else 1)


def test_first_hit_culls_back_faces(oracle_lib):
    m = fg.flat_plane(L=4.0, z0=1.0, height=4.0)
    up = np.array([[1.0, 1.0, 0.5, 0.0, 0.0, 1.0]])  # from below the plane, moving up
    tri, t, _ = oracle_lib.first_hit(m, up)
    assert tri[0] == -1 and abs(t[0] - 4.5) < 1e-12


# --------------------------------------------------------------- tables

def test_table_interpolation_rules(oracle_lib):
    t = fg.make_tables("vaughan")
    Eax, tax = t.E_axis(), t.theta_axis()
    # grid nodes return the stored value
    for i, j in [(0, 0), (17, 5), (90, 45), (127, 45), (64, 20)]:
        assert oracle_lib.table_yield(t, Eax[i], tax[j]) == pytest.approx(float(t.yld[i, j]), rel=1e-12)
    # a table linear in (ln E, alpha) is reproduced exactly between nodes
    lin = fg.make_tables("constant")
    X, Y = np.meshgrid(np.log(Eax), tax, indexing="ij")
    lin.yld = (0.1 * X + 0.01 * Y).astype(np.float32)
    rng = np.random.default_rng(0)
    for _ in range(50):
        E = float(np.exp(rng.uniform(np.log(1.0), np.log(1e4))))
        a = float(rng.uniform(0, 90))
        exact = fg.bilinear_reference(lin, E, a)
        assert oracle_lib.table_yield(lin, E, a) == pytest.approx(float(exact), rel=1e-9, abs=1e-9)
    # clamped outside the grid
    assert oracle_lib.table_yield(t, 0.1, 0.0) == pytest.approx(float(t.yld[0, 0]), rel=1e-12)
    assert oracle_lib.table_yield(t, 1e6, 90.0) == pytest.approx(float(t.yld[-1, -1]), rel=1e-12)


def test_energy_sampling_matches_chung_everhart(oracle_lib):
    t = fg.make_tables("vaughan")
    xs = np.linspace(0.01, 0.99, 99)
    for E_av in (50.0, 500.0):
        Ftop = fg.ce_cdf(E_av) / fg.ce_cdf(t.E_max)
        for x in xs:
            e = oracle_lib.sample_energy(t, x, E_av)
            exact = float(fg.ce_inverse(x * Ftop * fg.ce_cdf(t.E_max)))
            # piecewise-linear CDF on a log grid: well under 1 % of the energy
            assert abs(e - exact) <= 0.01 * exact + 1e-3
            assert e <= E_av
    # the median of the untruncated spectrum is the work function
    assert oracle_lib.sample_energy(t, 0.5, t.E_max) == pytest.approx(4.5, rel=2e-3)


def test_onb_orthonormal(oracle_lib):
    rng = np.random.default_rng(1)
    for _ in range(200):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        t1, t2 = oracle_lib.onb(n)
        B = np.stack([t1, t2, n])
        assert np.allclose(B @ B.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(t1, t2), n, atol=1e-12)


def test_vaughan_and_paper_tables():
    assert fg.vaughan_yield(650.0, 0.0) == pytest.approx(1.4, abs=1e-15)
    assert fg.vaughan_yield(650.0, 90.0) == pytest.approx(1.4 * math.exp(0.5), rel=1e-14)
    # Eq. (seey) at normal incidence peaks at the paper's flat-W value
    gold = {}
    for line in open(os.path.join(GOLD, "paper_flat_w.txt")):
        if line.strip() and not line.startswith("#"):
            k, v, tol = line.split()
            gold[k] = (float(v), float(tol))
    E = np.linspace(50, 1000, 95001)
    y = fg.paper_w_yield(E, 0.0)
    v, tol = gold["max_yield_normal"]
    assert abs(y.max() - v) < tol
    assert 380 < E[y.argmax()] < 450


def test_zero_area_triangles_dropped(oracle_lib):
    m = fg.flat_plane()
    v = np.concatenate([m.verts, np.array([[1, 1, 1], [2, 2, 2], [3, 3, 3]], dtype=np.float32)])
    tr = np.concatenate([m.tris, np.array([[4, 5, 6], [0, 0, 1]], dtype=np.int32)])
    m2 = fg.Mesh(v, tr, m.box_lo, m.box_hi, m.flags, {})
    assert oracle_lib.mesh_dropped(m2) == 2
    bad = fg.Mesh(v, np.array([[0, 1, 99]], dtype=np.int32), m.box_lo, m.box_hi, m.flags, {})
    with pytest.raises(ValueError):
        oracle_lib.mesh_dropped(bad)


# --------------------------------------------------------------- whole cascade

FLAT_CASES = [(500.0, 0.0), (100.0, 30.0), (1000.0, 60.0), (60.0, 80.0)]


@pytest.mark.parametrize("E,theta", FLAT_CASES)
def test_flat_plane_reproduces_table_yield(oracle_lib, E, theta):
    """Every daughter of a flat surface escapes: the yield is the table value."""
    tab = fg.make_tables("vaughan")
    n = 40000
    r = oracle_lib.trace(fg.flat_plane(), tab, E, theta, n, seed=11, max_gen=6)
    ref = float(fg.bilinear_reference(tab, E, theta))
    f = ref - math.floor(ref)
    sigma = math.sqrt(max(f * (1 - f), 1e-12) / n)
    assert abs(r["yield"] - ref) <= 3.0 * sigma
    assert r["n_escaped"] == r["n_rays"] - n
    assert r["n_lost"] == 0


@pytest.mark.parametrize("const", [0.0, 1.0, 2.0])
def test_flat_plane_integral_yields_are_exact(oracle_lib, const):
    tab = fg.make_tables("constant", const=const)
    n = 3000
    r = oracle_lib.trace(fg.flat_plane(), tab, 300.0, 20.0, n, seed=3, max_gen=6, per_primary=True)
    assert r["n_escaped"] == int(const) * n
    assert r["yield_sigma"] == 0.0
    if const == 0.0:
        assert r["e_escaped"] == 0.0
        assert r["e_deposited"] == pytest.approx(300.0 * n, rel=1e-12)


def test_flat_plane_energy_spectrum_and_cosine_law(oracle_lib):
    """With one daughter per hit the escaped energies follow the truncated
    Chung-Everhart law and the escape angles the cosine law."""
    from scipy import stats
    tab = fg.make_tables("constant", const=1.0)
    n = 20000
    E0 = 200.0
    r = oracle_lib.trace(fg.flat_plane(), tab, E0, 0.0, n, seed=5, max_gen=1, n_ebins=400, n_abins=90)
    assert r["n_escaped"] == n
    # energy histogram vs the closed-form CDF truncated at E0
    edges = np.linspace(0, E0, 401)
    cdf = fg.ce_cdf(edges) / fg.ce_cdf(E0)
    emp = np.concatenate([[0], np.cumsum(r["e_hist"])]) / n
    assert np.max(np.abs(emp - cdf)) < 1.63 / math.sqrt(n) + 0.01 * 0  # KS at 1 %
    # polar angle histogram: P(beta < b) = sin^2 b
    b = np.deg2rad(np.linspace(0, 90, 91))
    emp_a = np.concatenate([[0], np.cumsum(r["a_hist"])]) / n
    assert np.max(np.abs(emp_a - np.sin(b) ** 2)) < 1.63 / math.sqrt(n)
    # mean energy from the per-ray sums equals the truncated-law mean
    Eg = np.linspace(0, E0, 200001)
    pdf = np.gradient(fg.ce_cdf(Eg) / fg.ce_cdf(E0), Eg)
    mean_exact = float(np.trapezoid(Eg * pdf, Eg))
    assert r["e_escaped"] / n == pytest.approx(mean_exact, rel=0.03)
    assert stats is not None


@pytest.mark.parametrize("w,h,tw", [(2.0, 3.0, 1.0), (1.0, 1.0, 1.0)])
def test_trench_view_factor(oracle_lib, w, h, tw):
    """Slot of width w, depth h: floor daughters escape with the crossed-string
    view factor of the opening; wall-top daughters always escape."""
    tab = fg.make_tables("vaughan")
    E = 500.0
    n = 40000
    r = oracle_lib.trace(fg.trench(w=w, h=h, tw=tw), tab, E, 0.0, n, seed=21, max_gen=1)
    d0 = float(fg.bilinear_reference(tab, E, 0.0))
    F = math.sqrt(1 + (h / w) ** 2) - h / w
    expect = d0 * (tw / (w + tw) + w / (w + tw) * F)
    assert abs(r["yield"] - expect) <= 3.0 * r["yield_sigma"], (r["yield"], expect, r["yield_sigma"])
    assert r["n_wraps"] > 0


def test_conservation_per_primary(oracle_lib):
    m = fg.make_grf_foam(12, 0.6, 2.0, seed=3)
    tab = fg.make_tables("vaughan")
    n = 3000
    r = oracle_lib.trace(m, tab, 800.0, -80.0, n, seed=9, max_gen=6, per_primary=True)
    pp = r["per_primary"]
    assert np.allclose(pp["e_esc"] + pp["e_dep"], 800.0, rtol=1e-9, atol=0)
    assert r["n_rays"] == r["n_escaped"] + r["n_absorbed"] + r["n_truncated"] + r["n_lost"]
    assert int(pp["escaped"].sum()) == r["n_escaped"]
    assert int(pp["rays"].sum()) == r["n_rays"]
    assert int(r["e_hist"].sum()) == r["n_escaped"] == int(r["a_hist"].sum())


def test_resume_and_thread_invariance(oracle_lib):
    m = fg.make_grf_foam(12, 0.5, 2.0, seed=4)
    tab = fg.make_tables("vaughan")
    full = oracle_lib.trace(m, tab, 300.0, 20.0, 2000, seed=7, per_primary=True, n_threads=4)
    a = oracle_lib.trace(m, tab, 300.0, 20.0, 700, seed=7, per_primary=True, n_threads=1)
    b = oracle_lib.trace(m, tab, 300.0, 20.0, 1300, seed=7, pid0=700, per_primary=True, n_threads=3)
    for key in ("escaped", "rays"):
        assert np.array_equal(full["per_primary"][key],
                              np.concatenate([a["per_primary"][key], b["per_primary"][key]]))
    assert np.array_equal(full["e_hist"], a["e_hist"] + b["e_hist"])
    assert full["n_tri_tests"] == a["n_tri_tests"] + b["n_tri_tests"]


def test_foam_yield_falls_with_porosity(oracle_lib):
    """Qualitative trend of section 3.2: more porous foams emit less."""
    tab = fg.make_tables("vaughan")
    ys = []
    for p in (0.3, 0.8):
        m = fg.make_grf_foam(16, p, 2.0, seed=0)
        ys.append(oracle_lib.trace(m, tab, 500.0, 0.0, 4000, seed=2)["yield"])
    flat = float(fg.bilinear_reference(tab, 500.0, 0.0))
    assert ys[1] < ys[0] < flat


def test_absorption_depth_on_a_flat_plane(oracle_lib):
    """Every primary ends on the plane z0 = 1 of a cell spanning z in [0, 5]:
    one absorption event per primary at depth 0.8; daughters all escape."""
    n = 3000
    for const in (0.0, 2.0):
        tab = fg.make_tables("constant", const=const)
        r = oracle_lib.trace(fg.flat_plane(L=4.0, z0=1.0, height=4.0), tab, 300.0, 0.0, n, seed=3, max_gen=6,
                             n_zbins=10)
        z = r["z_hist"]
        assert z[8] == n and z.sum() == n


def test_absorption_depth_in_a_slot(oracle_lib):
    """Slot of width 2 between walls 1 thick and 3 high, cell z in [-1, 5]:
    at normal incidence a primary ends on a wall top (depth 1/3) with
    probability 1/3, on the floor (depth 5/6) otherwise."""
    n = 30000
    r = oracle_lib.trace(fg.trench(w=2.0, h=3.0, tw=1.0), fg.make_tables("constant", const=0.0), 300.0, 0.0, n,
                         seed=5, max_gen=1, n_zbins=7)
    z = r["z_hist"]
    assert z.sum() == n and z[2] + z[5] == n
    assert abs(z[2] / n - 1 / 3) <= 4 * math.sqrt(2 / 9 / n)


# --------------------------------------------------------------- emission cut-off, standard error, substrate

def test_no_emission_at_or_below_the_cutoff(oracle_lib):
    """A ray whose energy is at or below E_c emits nothing when it hits
    (section 2.2).  On a flat plane with a yield of 1 everywhere, primaries at
    and below E_c are absorbed and leave their whole energy; just above E_c
    every primary emits its one daughter, which escapes."""
    n = 2000
    for E0 in (5.0, 10.0):
        tab = fg.make_tables("constant", const=1.0, Ec=10.0)
        r = oracle_lib.trace(fg.flat_plane(), tab, E0, 0.0, n, seed=3, per_primary=True)
        assert r["n_escaped"] == 0 and r["yield"] == 0.0
        assert r["n_rays"] == r["n_absorbed"] == n
        assert np.all(r["per_primary"]["e_dep"] == E0)
    r = oracle_lib.trace(fg.flat_plane(), fg.make_tables("constant", const=1.0, Ec=10.0), 10.5, 0.0, n, seed=3)
    assert r["n_escaped"] == n


def _cutoff_slot(o, n, max_gen, seed=23):
    # one daughter of 100 eV per emitting hit (the paper's rule with a
    # constant E_SEE), E_c = 200 eV: only the 500 eV primaries can emit
    tab = fg.make_tables("constant", const=1.0, emission="paper", esee_const=100.0, Ec=200.0)
    return o.trace(fg.trench(w=2.0, h=3.0, tw=1.0), tab, 500.0, 0.0, n, seed=seed, max_gen=max_gen)


def _slot_one_bounce(w=2.0, h=3.0, tw=1.0):
    # primaries at normal incidence land on a wall top (fraction tw / (w + tw),
    # its daughter escapes) or on the floor (its daughter escapes with the
    # crossed-string view factor of the opening)
    F = math.sqrt(1 + (h / w) ** 2) - h / w
    return tw / (w + tw) + w / (w + tw) * F


def test_daughters_below_the_cutoff_do_not_reemit(oracle_lib):
    """In a slot, daughters below E_c that hit a wall are absorbed however
    deep the cascade may go: the yield is the one-bounce closed form."""
    n = 40000
    p = _slot_one_bounce()
    r = _cutoff_slot(oracle_lib, n, max_gen=6)
    assert abs(r["yield"] - p) <= 3.0 * math.sqrt(p * (1 - p) / n), (r["yield"], p)
    assert r["n_truncated"] == 0


@pytest.mark.parametrize("E,theta", FLAT_CASES)
def test_yield_sigma_is_the_standard_error(oracle_lib, E, theta):
    """On a flat plane every daughter escapes, so a primary's escape count is
    floor(delta), or floor(delta) + 1 with probability f = frac(delta): the
    standard error of the yield over n primaries is sqrt(f (1 - f) / n)."""
    tab = fg.make_tables("vaughan")
    n = 40000
    r = oracle_lib.trace(fg.flat_plane(), tab, E, theta, n, seed=11, max_gen=6)
    ref = float(fg.bilinear_reference(tab, E, theta))
    f = ref - math.floor(ref)
    exact = math.sqrt(f * (1 - f) / n)
    # the sample standard deviation of n = 40000 two-valued counts is within
    # 0.5 % (one standard deviation) of the exact one at these f
    assert abs(r["yield_sigma"] - exact) <= 0.03 * exact, (r["yield_sigma"], exact)


def _empty_substrate_cell(L=4.0, H=4.0):
    return fg.Mesh(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), (0.0, 0.0, 0.0), (L, L, H),
                   fg.PERIODIC_XY | fg.SUBSTRATE, dict(kind="substrate only"))


@pytest.mark.parametrize("E,theta", [(500.0, 0.0), (100.0, 50.0)])
def test_substrate_plane_is_a_flat_surface(oracle_lib, E, theta):
    """The substrate (section 2.2) is an emitting plane at z_min with normal
    +z: alone in a periodic cell it is a flat surface, so the yield is the
    table value at the primary's angle and the escape angles follow the
    cosine law."""
    tab = fg.make_tables("vaughan")
    n = 40000
    r = oracle_lib.trace(_empty_substrate_cell(), tab, E, theta, n, seed=13, max_gen=6, n_abins=90)
    ref = float(fg.bilinear_reference(tab, E, theta))
    f = ref - math.floor(ref)
    assert abs(r["yield"] - ref) <= 3.0 * math.sqrt(f * (1 - f) / n), (r["yield"], ref)
    assert r["n_substrate"] == n and r["n_lost"] == 0
    b = np.deg2rad(np.linspace(0, 90, 91))
    m = r["n_escaped"]
    emp = np.concatenate([[0], np.cumsum(r["a_hist"])]) / m
    assert np.max(np.abs(emp - np.sin(b) ** 2)) < 1.63 / math.sqrt(m)


def test_surfaces_in_a_cell_face_are_rejected(oracle_lib):
    """A triangle lying in a face of the cell would meet the ray exactly where
    it leaves the cell; such meshes are refused.  A triangle touching a face
    along an edge is fine."""
    with pytest.raises(ValueError):
        oracle_lib.mesh_dropped(fg.flat_plane(z0=0.0))  # in the bottom face
    v = np.array([[0, 0, 1], [0, 2, 1], [0, 0, 3], [2, 2, 4], [3, 2, 4], [2, 3, 4]], dtype=np.float32)
    box = ((0.0, 0.0, 0.0), (4.0, 4.0, 4.0))
    for tri in ([0, 1, 2], [3, 4, 5]):  # in the x = 0 face; in the top face
        m = fg.Mesh(v, np.array([tri], dtype=np.int32), *box, fg.PERIODIC_XY, {})
        with pytest.raises(ValueError):
            oracle_lib.mesh_dropped(m)
        with pytest.raises(ValueError):
            oracle_lib.first_hit(m, np.array([[1.0, 1.0, 3.5, 0.0, 0.0, -1.0]]))
    edge = fg.Mesh(np.array([[0, 0, 1], [0, 2, 1], [1, 0, 3]], dtype=np.float32), np.array([[0, 1, 2]], np.int32),
                   *box, fg.PERIODIC_XY, {})
    assert oracle_lib.mesh_dropped(edge) == 0
