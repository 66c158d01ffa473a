"""GPU path against the FP64 oracle: the parts of section 2.2 the oracle's
pins fix (emission cut-off, standard error, substrate), the queue's chunked
re-issue, angle histograms on a foam, and batched jobs paired primary by
primary with the oracle (the benchmark's whole sweep among them)."""
import math

import numpy as np
import pytest

import foamgen as fg

pytestmark = pytest.mark.gpu


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
def tiny():
    return fg.make_grf_foam(16, 0.5, 2.0, seed=0)


@pytest.fixture(scope="module")
def vaughan():
    return fg.make_tables("vaughan")


def _paired(ppg, ppo):
    """Agreement rate, mean paired difference and its standard error."""
    d = ppg.astype(np.int64) - ppo.astype(np.int64)
    n = d.size
    se = d.std(ddof=1) / math.sqrt(n) if n > 1 else 0.0
    return float((d == 0).mean()), float(d.mean()), float(se)


# ---------------------------------------------------------------- cut-off, sigma, substrate

def test_no_emission_at_or_below_the_cutoff(ctx, torch):
    sid = ctx.load_scene(fg.flat_plane())
    tid = ctx.load_tables(fg.make_tables("constant", const=1.0, Ec=10.0))
    n = 20000
    for E0 in (5.0, 10.0):
        r = ctx.trace(sid, tid, E0, 0.0, n, seed=3)
        assert r["n_escaped"] == 0 and r["n_rays"] == r["n_absorbed"] == n
        assert r["e_deposited"] == E0 * n and r["e_escaped"] == 0.0
    assert ctx.trace(sid, tid, 10.5, 0.0, n, seed=3)["n_escaped"] == n


def test_daughters_below_the_cutoff_do_not_reemit(ctx, torch, oracle_lib):
    """Slot with one 100 eV daughter per emitting hit and E_c = 200 eV: the
    yield is the one-bounce closed form at any cascade depth, and every
    primary's escape count is the oracle's."""
    tab = fg.make_tables("constant", const=1.0, emission="paper", esee_const=100.0, Ec=200.0)
    m = fg.trench(w=2.0, h=3.0, tw=1.0)
    sid = ctx.load_scene(m)
    tid = ctx.load_tables(tab)
    n = 200000
    g = ctx.trace(sid, tid, 500.0, 0.0, n, seed=23, max_gen=6)
    F = math.sqrt(1 + 1.5 ** 2) - 1.5
    p = 1 / 3 + 2 / 3 * F
    assert abs(g["yield"] - p) <= 3 * math.sqrt(p * (1 - p) / n), (g["yield"], p)
    k = 20000
    pp = torch.zeros(k, dtype=torch.int32, device="cuda:0")
    ctx.trace(sid, tid, 500.0, 0.0, k, seed=23, max_gen=6, per_primary=pp)
    o = oracle_lib.trace(m, tab, 500.0, 0.0, k, seed=23, max_gen=6, per_primary=True)
    agree, mean, se = _paired(pp.cpu().numpy(), o["per_primary"]["escaped"])
    assert agree >= 0.9999, agree


@pytest.mark.parametrize("E,theta", [(500.0, 0.0), (100.0, 30.0), (1000.0, 60.0), (60.0, 80.0)])
def test_yield_sigma_is_the_standard_error(ctx, oracle_lib, vaughan, E, theta):
    """Flat plane: sigma is sqrt(f (1 - f) / n) (f = frac of the table yield),
    and the oracle's from the same primaries."""
    sid = ctx.load_scene(fg.flat_plane())
    tid = ctx.load_tables(vaughan)
    n = 200000
    g = ctx.trace(sid, tid, E, theta, n, seed=11)
    ref = float(fg.bilinear_reference(vaughan, E, theta))
    f = ref - math.floor(ref)
    exact = math.sqrt(f * (1 - f) / n)
    assert abs(g["yield_sigma"] - exact) <= 0.03 * exact, (g["yield_sigma"], exact)
    k = 40000
    g = ctx.trace(sid, tid, E, theta, k, seed=11)
    o = oracle_lib.trace(fg.flat_plane(), vaughan, E, theta, k, seed=11)
    assert g["n_escaped"] == o["n_escaped"]
    assert g["yield_sigma"] == pytest.approx(o["yield_sigma"], rel=1e-9)


def test_yield_sigma_on_a_foam(ctx, torch, oracle_lib, tiny, vaughan):
    """On a foam the escape counts are not two-valued: sigma from the same
    primaries agrees with the oracle's, and with the spread of the per-primary
    counts the GPU returns."""
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    n = 10000
    pp = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    g = ctx.trace(sid, tid, 800.0, -80.0, n, seed=37, per_primary=pp)
    c = pp.cpu().numpy().astype(np.float64)
    assert g["yield_sigma"] == pytest.approx(c.std(ddof=1) / math.sqrt(n), rel=1e-9)
    o = oracle_lib.trace(tiny, vaughan, 800.0, -80.0, n, seed=37)
    assert g["yield_sigma"] == pytest.approx(o["yield_sigma"], rel=0.02)


def _empty_substrate_cell():
    return fg.Mesh(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), (0.0, 0.0, 0.0), (4.0, 4.0, 4.0),
                   fg.PERIODIC_XY | fg.SUBSTRATE, {})


@pytest.mark.parametrize("E,theta", [(500.0, 0.0), (100.0, 50.0)])
def test_substrate_plane_is_a_flat_surface(ctx, vaughan, E, theta):
    sid = ctx.load_scene(_empty_substrate_cell())
    tid = ctx.load_tables(vaughan)
    n = 200000
    r = ctx.trace(sid, tid, E, theta, n, seed=13, n_abins=90)
    ref = float(fg.bilinear_reference(vaughan, E, theta))
    f = ref - math.floor(ref)
    assert abs(r["yield"] - ref) <= 3 * math.sqrt(f * (1 - f) / n), (r["yield"], ref)
    assert r["n_substrate"] == n and r["n_lost"] == 0
    m = r["n_escaped"]
    b = np.deg2rad(np.linspace(0, 90, 91))
    emp = np.concatenate([[0], np.cumsum(r["a_hist"])]) / m
    assert np.max(np.abs(emp - np.sin(b) ** 2)) < 1.63 / math.sqrt(m)


def test_surfaces_in_a_cell_face_are_refused(ctx):
    import paper_1806_00205_amd as rt
    m = fg.flat_plane(z0=0.0)
    with pytest.raises(rt.RtmcError) as e:
        ctx.load_mesh(m.verts, m.tris, m.box_lo, m.box_hi, m.flags)
    assert e.value.status == -1 and "face" in str(e.value)
    v = np.array([[0, 0, 1], [0, 2, 1], [0, 0, 3]], dtype=np.float32)
    with pytest.raises(rt.RtmcError):
        ctx.load_mesh(v, np.array([[0, 1, 2]], np.int32), (0, 0, 0), (4, 4, 4), fg.PERIODIC_XY)
    v[2] = (1, 0, 3)  # one edge in the face only
    ctx.load_mesh(v, np.array([[0, 1, 2]], np.int32), (0, 0, 0), (4, 4, 4), fg.PERIODIC_XY)


# ---------------------------------------------------------------- queue overflow

def test_queue_overflow_is_reissued_in_smaller_chunks(torch, oracle_lib):
    """A cascade that doubles at nearly every hit (yield 2 everywhere, E_c = 0,
    a deep narrow slot) outgrows a queue sized for two daughters per primary:
    the trace is re-issued in smaller chunks and drops nothing.  Its integer
    tallies equal those of a trace whose queue was large enough from the
    start, and every primary's escape count equals the oracle's."""
    import paper_1806_00205_amd as rt
    m = fg.trench(w=1.0, h=8.0, tw=0.25)
    tab = fg.make_tables("constant", const=2.0, emission="paper", esee_const=100.0, Ec=0.0)
    n, max_gen = 20000, 4
    keys = ("n_rays", "n_escaped", "n_absorbed", "n_truncated", "n_lost", "n_spawned", "n_tri_tests",
            "n_node_visits", "e_escaped", "e_deposited")
    small = rt.Context(0)  # fresh: its queue is sized by this trace alone
    try:
        sid = small.load_scene(m)
        tid = small.load_tables(tab)
        pp = torch.zeros(n, dtype=torch.int32, device="cuda:0")
        a = small.trace(sid, tid, 500.0, 0.0, n, seed=41, max_gen=max_gen, per_primary=pp)
    finally:
        small.close()
    big = rt.Context(0)
    try:
        sid = big.load_scene(m)
        tid = big.load_tables(tab)
        big.trace(sid, tid, 500.0, 0.0, 64 * n, seed=42, max_gen=0)  # grows the queue to 128 n entries
        b = big.trace(sid, tid, 500.0, 0.0, n, seed=41, max_gen=max_gen)
    finally:
        big.close()
    assert b["n_chunks"] == 1 and a["n_chunks"] > 1, (a["n_chunks"], b["n_chunks"])
    assert b["n_rays"] > 4 * n  # the cascade really outgrew 2 n rays in a generation
    for k in keys:
        assert a[k] == b[k], (k, a[k], b[k])
    assert a["n_rays"] == n + a["n_spawned"]
    o = oracle_lib.trace(m, tab, 500.0, 0.0, n, seed=41, max_gen=max_gen, per_primary=True)
    agree, mean, se = _paired(pp.cpu().numpy(), o["per_primary"]["escaped"])
    assert agree >= 0.995, agree
    assert abs(mean) <= 3 * se + 1e-12


# ---------------------------------------------------------------- histograms on a foam

@pytest.mark.parametrize("E,theta", [(500.0, 0.0), (250.0, -80.0)])
def test_angle_and_energy_histograms_on_a_foam(ctx, oracle_lib, tiny, vaughan, E, theta):
    """Escape-angle and escaped-energy histograms of the same primaries on a
    foam, bin by bin against the oracle: they differ only where a primary's
    tree differs (a near-tie) or a value sits on a bin edge up to FP32
    rounding."""
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    n = 10000
    g = ctx.trace(sid, tid, E, theta, n, seed=43, n_abins=90, n_ebins=128)
    o = oracle_lib.trace(tiny, vaughan, E, theta, n, seed=43, n_abins=90, n_ebins=128)
    for h in ("a_hist", "e_hist"):
        d = np.abs(g[h].astype(np.int64) - o[h].astype(np.int64)).sum()
        assert d <= 0.002 * o["n_escaped"] + 2, (h, d, o["n_escaped"])
    assert g["n_escaped"] == pytest.approx(o["n_escaped"], abs=0.002 * o["n_escaped"] + 2)


# ---------------------------------------------------------------- batched jobs paired with the oracle

def test_two_scene_batch_paired_against_the_oracle(ctx, torch, oracle_lib, tiny, vaughan):
    """Jobs on two foams in one batch (the multi-scene traversal kernel):
    every job's per-primary escape counts against the oracle's."""
    small = fg.make_grf_foam(12, 0.7, 2.0, seed=5)
    s1, s2 = ctx.load_scene(tiny), ctx.load_scene(small)
    tid = ctx.load_tables(vaughan)
    jobs = [(s1, 500.0, 0.0, 3000, 61), (s2, 100.0, 40.0, 2000, 62), (s1, 250.0, -80.0, 2500, 63),
            (s2, 1000.0, 60.0, 1500, 64)]
    meshes = {s1: tiny, s2: small}
    pps = [torch.zeros(n, dtype=torch.int32, device="cuda:0") for _, _, _, n, _ in jobs]
    outs = ctx.trace_batch(tid, jobs, max_gen=6, per_primary=pps)
    for (s, E, th, n, sd), b, pp in zip(jobs, outs, pps):
        o = oracle_lib.trace(meshes[s], vaughan, E, th, n, seed=sd, max_gen=6, per_primary=True)
        ppg = pp.cpu().numpy()
        assert int(ppg.sum()) == b["n_escaped"]
        agree, mean, se = _paired(ppg, o["per_primary"]["escaped"])
        assert agree >= 0.995, (E, th, agree)
        assert abs(mean) <= 3 * se + 1e-12, (E, th, mean, se)
        sig = math.sqrt(b["yield_sigma"] ** 2 + o["yield_sigma"] ** 2)
        assert abs(b["yield"] - o["yield"]) <= 3 * sig + 1e-12


SWEEP = [(E, th) for E in (50.0, 100.0, 250.0, 500.0, 1000.0) for th in (0.0, 20.0, 40.0, 60.0, 80.0)]


@pytest.mark.slow
def test_benchmark_sweep_paired_against_the_oracle(ctx, torch, oracle_lib, vaughan):
    """The benchmark's 128^3 sweep as it is timed (one rtmc_trace_batch, 25
    points x 1e7 primaries, one 2^28-primary chunk): the first 200 primary ids
    of every point against the oracle.  Each point: identical escape counts
    for >= 99.5 % of the ids, |mean paired difference| <= 3 sigma, yield
    within 3 sigma; over the points, the chi^2 of the paired differences."""
    from scipy import stats
    m = fg.make_grf_foam(128, 0.6, 2.0, seed=1)
    sid = ctx.load_scene(m)
    tid = ctx.load_tables(vaughan)
    npp, k = 10_000_000, 200
    jobs = [(sid, E, th, npp, 2000 + i) for i, (E, th) in enumerate(SWEEP)]
    pps = [torch.zeros(npp, dtype=torch.int32, device="cuda:0") for _ in jobs]
    cfg = ctx.get_launch()
    ctx.set_launch(cfg["block"], cfg["wg_per_cu"], cfg["lds_stack"], 1 << 28, cfg["refill"], cfg["occupancy"])
    try:
        outs = ctx.trace_batch(tid, jobs, max_gen=6, per_primary=pps)
    finally:
        ctx.set_launch(**cfg)
    assert outs[0]["n_chunks"] == 1
    chi2, dof = 0.0, 0
    for (s, E, th, n, sd), b, pp in zip(jobs, outs, pps):
        assert int(pp.sum().item()) == b["n_escaped"]
        o = oracle_lib.trace(m, vaughan, E, th, k, seed=sd, max_gen=6, per_primary=True)
        agree, mean, se = _paired(pp[:k].cpu().numpy(), o["per_primary"]["escaped"])
        assert agree >= 0.995, (E, th, agree)
        assert abs(mean) <= 3 * se + 1e-12, (E, th, mean, se)
        if se > 0:
            chi2 += (mean / se) ** 2
        dof += 1
        sig = math.sqrt(b["yield_sigma"] ** 2 + o["yield_sigma"] ** 2)
        assert abs(b["yield"] - o["yield"]) <= 3 * sig, (E, th, b["yield"], o["yield"], sig)
    assert chi2 <= stats.chi2.ppf(0.999, dof), chi2


# ---------------------------------------------------------------- replayed daughters

@pytest.mark.parametrize("gen", [1, 2])
def test_first_hits_of_daughters_the_gpu_spawned(ctx, torch, oracle_lib, tiny, vaughan, gen):
    """Daughter rays exactly as the GPU queued them (FP32 origin and direction,
    read back from the queue of generation gen) re-traced by the oracle: the
    first surface each meets agrees with the GPU's, and so does its distance."""
    from tests.test_gpu_core import _first_hit_parity
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    cap = 20000
    rep = torch.zeros((cap, 6), dtype=torch.float32, device="cuda:0")
    # about 1.4 daughters per primary reach generation 1, 0.045 generation 2
    r = ctx.trace(sid, tid, 500.0, -80.0, 20000 if gen == 1 else 200000, seed=51, max_gen=6, replay=rep,
                  replay_gen=gen)
    n = r["n_replay"]
    assert 2000 < n <= cap, n
    rays = rep[:n].cpu().numpy().astype(np.float64)
    assert np.allclose(np.linalg.norm(rays[:, 3:], axis=1), 1.0, atol=1e-5)
    _first_hit_parity(ctx, torch, oracle_lib, tiny, rays, 0.9999)
