"""The paper's emission rule (section 2.2: E_SEE, the two-daughter split) on
the GPU, against the FP64 oracle and the closed forms its pins use."""
import math

import numpy as np
import pytest

import foamgen as fg
from tests.test_oracle_paper_mode import _pair_sum_cdf, _slot_clear

pytestmark = pytest.mark.gpu
KS1 = 1.63


@pytest.fixture(scope="module")
def ctx():
    import paper_1806_00205_amd as rt
    c = rt.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def paper_w():
    return fg.make_tables("paper_w")


@pytest.mark.parametrize("E,theta", [(500.0, 0.0), (200.0, -80.0)])
def test_paired_parity_on_a_foam(ctx, torch, oracle_lib, paper_w, E, theta):
    """Tungsten fits on the 16^3 foam: per-primary escape counts as the oracle's."""
    m = fg.make_grf_foam(16, 0.5, 2.0, seed=0)
    sid = ctx.load_scene(m)
    tid = ctx.load_tables(paper_w)
    n = 8000
    pp = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    g = ctx.trace(sid, tid, E, theta, n, seed=3, per_primary=pp)
    o = oracle_lib.trace(m, paper_w, E, theta, n, seed=3, per_primary=True)
    sig = math.sqrt(g["yield_sigma"] ** 2 + o["yield_sigma"] ** 2)
    assert abs(g["yield"] - o["yield"]) <= 3 * sig
    same = (pp.cpu().numpy().astype(np.int64) == o["per_primary"]["escaped"].astype(np.int64)).mean()
    assert same >= 0.995, same
    # fixed-point energy sums conserve every primary's energy exactly
    assert g["e_escaped"] + g["e_deposited"] == E * n


def test_lone_daughter_energy_is_E_SEE(ctx):
    n = 4000
    tab = fg.make_tables("constant", const=1.0, emission="paper", esee_const=100.0)
    sid = ctx.load_scene(fg.flat_plane())
    tid = ctx.load_tables(tab)
    r = ctx.trace(sid, tid, 500.0, 0.0, n, seed=5, max_gen=1, n_ebins=500)
    assert r["n_escaped"] == n
    assert r["e_escaped"] == 100.0 * n
    assert r["e_hist"][100] == n


def test_pair_energies_and_angles(ctx):
    n = 20000
    tab = fg.make_tables("constant", const=2.0, emission="paper", esee_const=100.0)
    sid = ctx.load_scene(fg.flat_plane())
    tid = ctx.load_tables(tab)
    r = ctx.trace(sid, tid, 500.0, 0.0, n, seed=7, max_gen=1, n_ebins=500, n_abins=180)
    assert r["n_escaped"] == 2 * n
    u = np.clip(np.linspace(0, 500.0, 501) / 100.0, 0, 1)
    emp = np.concatenate([[0], np.cumsum(r["e_hist"])]) / (2 * n)
    assert np.max(np.abs(emp - (0.5 * u ** 2 + 0.5 * u))) < KS1 / math.sqrt(n)
    b = np.deg2rad(np.linspace(0, 90, 181))
    emp_a = np.concatenate([[0], np.cumsum(r["a_hist"])]) / (2 * n)
    assert np.max(np.abs(emp_a - np.sin(b) ** 2)) < KS1 / math.sqrt(n)
    # mean of E1 + E2 per primary: E_SEE (2/3 + 1/2)
    assert r["e_escaped"] / n == pytest.approx(100.0 * (2.0 / 3.0 + 0.5), rel=0.01)


def test_pair_angles_in_a_slot(ctx, torch):
    w, h, tw = 2.0, 3.0, 1.0
    x = (np.arange(1000) + 0.5) / 1000 * w
    xi = (np.arange(2000) + 0.5) / 2000
    X, XI = np.meshgrid(x, xi, indexing="ij")
    b1 = np.arcsin(np.sqrt(XI))
    p2 = tw / (w + tw) + w / (w + tw) * float((_slot_clear(X, b1, w, h) * _slot_clear(X, np.pi / 2 - b1, w, h)).mean())
    n = 40000
    tab = fg.make_tables("constant", const=2.0, emission="paper", esee_const=100.0)
    sid = ctx.load_scene(fg.trench(w=w, h=h, tw=tw))
    tid = ctx.load_tables(tab)
    pp = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    ctx.trace(sid, tid, 500.0, 0.0, n, seed=43, max_gen=1, per_primary=pp)
    est = float((pp.cpu().numpy() == 2).mean())
    assert abs(est - p2) <= 4.0 * math.sqrt(p2 * (1 - p2) / n), (est, p2)


def test_pair_sum_law_through_per_primary_energy(ctx, oracle_lib):
    """The GPU keeps no per-primary energies: compare its escaped-energy
    histogram of three-daughter cascades (a pair plus a lone one) with the
    oracle's on the same primaries, bin by bin within counting noise."""
    n = 10000
    tab = fg.make_tables("constant", const=3.0, emission="paper", esee_const=100.0)
    sid = ctx.load_scene(fg.flat_plane())
    tid = ctx.load_tables(tab)
    g = ctx.trace(sid, tid, 500.0, 0.0, n, seed=9, max_gen=1, n_ebins=50)
    o = oracle_lib.trace(fg.flat_plane(), tab, 500.0, 0.0, n, seed=9, max_gen=1, n_ebins=50, per_primary=True)
    assert g["n_escaped"] == o["n_escaped"] == 3 * n
    # same random numbers: identical histograms up to FP32 rounding at bin edges
    assert np.abs(g["e_hist"].astype(np.int64) - o["e_hist"].astype(np.int64)).sum() <= 0.001 * 3 * n
    s = np.sort(o["per_primary"]["e_esc"] / 100.0 - 1.0)
    assert np.max(np.abs(np.arange(1, n + 1) / n - _pair_sum_cdf(s))) < KS1 / math.sqrt(n)


@pytest.mark.parametrize("E0", [100.0, 400.0, 1000.0])
def test_paper_tungsten_flat_curve(ctx, paper_w, E0):
    n = 100000
    sid = ctx.load_scene(fg.flat_plane())
    tid = ctx.load_tables(paper_w)
    r = ctx.trace(sid, tid, E0, 0.0, n, seed=17, max_gen=6)
    ref = float(fg.bilinear_reference(paper_w, E0, 0.0))
    f = ref - math.floor(ref)
    assert abs(r["yield"] - ref) <= 3.0 * math.sqrt(f * (1 - f) / n)


def test_paper_mode_needs_esee(ctx):
    import paper_1806_00205_amd as rt
    tab = fg.make_tables("constant", const=1.0, emission="paper", esee_const=100.0)
    bad = fg.make_tables("constant", const=1.0, emission="paper", esee_const=100.0)
    bad.esee = None
    with pytest.raises(rt.RtmcError):
        ctx.load_tables(bad)
    tab.esee = tab.esee.copy()
    tab.esee[3, 4] = np.nan
    with pytest.raises(rt.RtmcError):
        ctx.load_tables(tab)


@pytest.mark.parametrize("a,kind", [(0.2, "paper_w"), (0.1, "vaughan")])
def test_cage_parity(ctx, torch, oracle_lib, a, kind):
    """The open cubic cage on its substrate: per-primary escape counts as the oracle's."""
    m = fg.make_cage(a, 16.0, 2)
    tab = fg.make_tables(kind)
    sid = ctx.load_scene(m)
    tid = ctx.load_tables(tab)
    n = 8000
    pp = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    g = ctx.trace(sid, tid, 400.0, 0.0, n, seed=13, max_gen=8, per_primary=pp)
    o = oracle_lib.trace(m, tab, 400.0, 0.0, n, seed=13, max_gen=8, per_primary=True)
    same = (pp.cpu().numpy().astype(np.int64) == o["per_primary"]["escaped"].astype(np.int64)).mean()
    assert same >= 0.995, same
    sig = math.sqrt(g["yield_sigma"] ** 2 + o["yield_sigma"] ** 2)
    assert abs(g["yield"] - o["yield"]) <= 3 * sig
    assert g["n_substrate"] > 0 and g["n_wraps"] > 0


def test_absorption_depth_flat_and_slot(ctx):
    """Depth histogram: the flat plane's single depth, and the slot's wall-top /
    floor split at normal incidence (section 3.2, Fig. pen)."""
    n = 3000
    sid = ctx.load_scene(fg.flat_plane(L=4.0, z0=1.0, height=4.0))
    for const in (0.0, 2.0):
        tid = ctx.load_tables(fg.make_tables("constant", const=const))
        z = ctx.trace(sid, tid, 300.0, 0.0, n, seed=3, max_gen=6, n_zbins=10)["z_hist"]
        assert z[8] == n and z.sum() == n
    n = 30000
    sid = ctx.load_scene(fg.trench(w=2.0, h=3.0, tw=1.0))
    tid = ctx.load_tables(fg.make_tables("constant", const=0.0))
    z = ctx.trace(sid, tid, 300.0, 0.0, n, seed=5, max_gen=1, n_zbins=7)["z_hist"]
    assert z.sum() == n and z[2] + z[5] == n
    assert abs(z[2] / n - 1 / 3) <= 4 * math.sqrt(2 / 9 / n)


@pytest.mark.parametrize("theta", [0.0, -80.0])
def test_absorption_depth_parity_on_a_foam(ctx, oracle_lib, theta):
    """Same primaries on the 16^3 foam: the GPU's depth histogram is the oracle's
    up to FP32 placement of hit points at bin edges."""
    m = fg.make_grf_foam(16, 0.5, 2.0, seed=0)
    tab = fg.make_tables("vaughan")
    sid = ctx.load_scene(m)
    tid = ctx.load_tables(tab)
    n = 6000
    g = ctx.trace(sid, tid, 100.0, theta, n, seed=11, n_zbins=32)
    o = oracle_lib.trace(m, tab, 100.0, theta, n, seed=11, n_zbins=32)
    gz, oz = g["z_hist"].astype(np.int64), o["z_hist"].astype(np.int64)
    assert gz.sum() == g["n_absorbed"] + g["n_truncated"]
    assert oz.sum() == o["n_absorbed"] + o["n_truncated"]
    assert np.abs(gz - oz).sum() <= 0.005 * oz.sum() + 2
