"""GPU path against the FP64 oracle (run on an MI355X through the C interface)."""
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
    """The 16^3 foam at porosity 0.5 (about 4k triangles)."""
    return fg.make_grf_foam(16, 0.5, 2.0, seed=0)


@pytest.fixture(scope="module")
def vaughan():
    return fg.make_tables("vaughan")


# ---------------------------------------------------------------- sort + BVH

@pytest.mark.parametrize("n,bits", [(1, 64), (1000, 63), (4097, 16), (300001, 63), (65536 * 3 + 17, 64)])
def test_radix_sort_matches_torch(ctx, torch, n, bits):
    g = torch.Generator().manual_seed(n)
    keys = torch.randint(-(2 ** 62), 2 ** 62, (n,), generator=g, dtype=torch.int64)
    if bits < 64:
        keys = keys & ((1 << bits) - 1)
    if n > 3:
        keys[: n // 3] = keys[n // 2]  # many equal keys: stability matters
    vals = torch.arange(n, dtype=torch.int32)
    kd, vd = keys.cuda(), vals.cuda()
    ctx.sort_pairs(kd, vd, bits)
    torch.cuda.synchronize()
    # unsigned order: flip the sign bit to sort as signed
    ku = keys ^ (-(2 ** 63)) if bits == 64 else keys
    ref_k, ref_i = torch.sort(ku, stable=True)
    if bits == 64:
        ref_k = ref_k ^ (-(2 ** 63))
    assert torch.equal(kd.cpu(), ref_k)
    assert torch.equal(vd.cpu(), ref_i.to(torch.int32))


def _check_bvh(nodes, tris, n):
    assert nodes.shape[0] == max(n - 1, 1)
    links = nodes[:, 12:14].view(np.int32).view(np.uint32)
    LEAF = np.uint32(0x80000000)
    seen_leaf = np.zeros(n, dtype=np.int64)
    seen_node = np.zeros(nodes.shape[0], dtype=np.int64)
    V = tris.reshape(-1, 3, 4)[:, :, :3]
    tlo, thi = V.min(axis=1), V.max(axis=1)
    for p in range(nodes.shape[0]):
        for side in range(2):
            c = links[p, side]
            box = nodes[p, side * 6: side * 6 + 6]
            if c & LEAF:
                k = int(c & ~LEAF)
                seen_leaf[k] += 1
                assert np.all(box[:3] == tlo[k]) and np.all(box[3:] == thi[k])
            else:
                seen_node[int(c)] += 1
                child = nodes[int(c)]
                lo = np.minimum(child[0:3], child[6:9])
                hi = np.maximum(child[3:6], child[9:12])
                assert np.all(box[:3] == lo) and np.all(box[3:] == hi)
    if n > 1:
        assert np.all(seen_leaf == 1)
        assert seen_node[0] == 0 and np.all(seen_node[1:] == 1)


def _check_bvh_fast(nodes, tris, n):
    """_check_bvh's box checks, vectorized for large trees: every child box
    equals the exact bounds of its triangle or the union of its node's two
    boxes, and every triangle and non-root node is referenced once."""
    links = nodes[:, 12:14].view(np.uint32)
    leaf_bit = np.uint32(0x80000000)
    V = tris.reshape(-1, 3, 4)[:, :, :3]
    tri_box = np.concatenate([V.min(axis=1), V.max(axis=1)], axis=1)
    node_box = np.concatenate([np.minimum(nodes[:, 0:3], nodes[:, 6:9]),
                               np.maximum(nodes[:, 3:6], nodes[:, 9:12])], axis=1)
    for side in range(2):
        c = links[:, side]
        box = nodes[:, side * 6: side * 6 + 6]
        is_leaf = (c & leaf_bit) != 0
        idx = (c & ~leaf_bit).astype(np.int64)
        assert np.array_equal(box[is_leaf], tri_box[idx[is_leaf]])
        assert np.array_equal(box[~is_leaf], node_box[idx[~is_leaf]])
    c = links.ravel()
    is_leaf = (c & leaf_bit) != 0
    assert np.array_equal(np.sort((c[is_leaf] & ~leaf_bit).astype(np.int64)), np.arange(n))
    assert np.array_equal(np.sort(c[~is_leaf].astype(np.int64)), np.arange(1, nodes.shape[0]))


def test_bvh_boxes_of_a_large_tree(ctx):
    """Every box of the 1.9M-triangle tree is exact (the bottom-up pass hands
    boxes from thread to thread through device-scope atomics); built and
    checked three times."""
    m = fg.make_grf_foam(128, 0.6, 2.0, seed=1)
    for rep in range(3):
        sid = ctx.load_scene(m)
        info = ctx.scene_info(sid)  # ingest drops the mesh's few zero-area triangles
        nodes, tris = ctx.bvh_download(sid)
        _check_bvh_fast(nodes, tris, info["n_tris"])
        assert info["bvh_depth"] == 27


def _decode(q, s, o):
    """fmaf(q, s, o) in FP32: q * s is exact (byte times a power of two) and
    its sum with an FP32 origin is exact in FP64 here, so one rounding to
    FP32 reproduces the fused operation."""
    return np.float32(np.float64(q) * np.float64(s) + np.float64(o))


def _check_wide(wide, nodes, tris, n):
    """Quantized 4-wide nodes against the binary tree they are collapsed from,
    walked from the root (node 0 = binary node 0): each node holds the children
    of its binary node, the largest inner slot expanded until four; every
    decoded box contains its child's exact box; the nodes reached from node 0
    reference every triangle exactly once; they fill the first records level
    by level, a node's inner children in consecutive records, the rest zero."""
    links = nodes[:, 12:14].view(np.uint32)
    boxes = nodes[:, :12].reshape(-1, 2, 6)
    tb = tris.reshape(-1, 3, 4)[:, :, :3]
    tri_box = np.concatenate([tb.min(axis=1), tb.max(axis=1)], axis=1)
    leaf_bit = np.uint32(0x80000000)
    empty = np.uint32(0xFFFFFFFF)

    def slots_of(i):
        # i's children, then the inner slot of largest surface area (FP32, first
        # of equals) replaced by its two children until four slots are filled
        out = [(links[i, 0], boxes[i, 0]), (links[i, 1], boxes[i, 1])]
        while len(out) < 4:
            best, ba = -1, np.float32(-1.0)
            for j, (link, b) in enumerate(out):
                if link & leaf_bit:
                    continue
                d = (b[3:] - b[:3]).astype(np.float32)
                area = np.float32(np.float32(d[0] * d[1]) + np.float32(d[1] * d[2])) + np.float32(d[2] * d[0])
                if area > ba:
                    best, ba = j, area
            if best < 0:
                break
            link = out[best][0]
            out[best] = (links[link, 0], boxes[link, 0])
            out.append((links[link, 1], boxes[link, 1]))
        return out

    seen = np.zeros(n, dtype=np.int64)
    queue = [(0, 0)]  # (record, binary node), breadth first
    level_of = {0: 0}
    for r, i in queue:
        w = wide[r]
        o = w[0:3].view(np.float32)
        sc = [w[k:k + 1].view(np.float32)[0] for k in (3, 14, 15)]
        for a in range(3):  # powers of two
            assert sc[a] > 0 and np.frexp(sc[a])[0] == 0.5
        expect = slots_of(i)
        assert 2 <= len(expect) <= 4
        inner = []
        for j in range(4):
            link = w[4 + j]
            if j >= len(expect):
                assert link == empty
                continue
            el, ebox = expect[j]
            if el & leaf_bit:
                assert link == el
            else:
                assert not (link & leaf_bit) and link != empty
                inner.append(int(link))
            q = [(w[8 + k] >> np.uint32(8 * j)) & np.uint32(0xFF) for k in range(6)]
            lo = [_decode(q[a], sc[a], o[a]) for a in range(3)]
            hi = [_decode(q[3 + a], sc[a], o[a]) for a in range(3)]
            assert np.all(np.array(lo) <= ebox[:3]) and np.all(np.array(hi) >= ebox[3:]), (i, j)
            # quantisation keeps boxes tight: at most two steps of 2^e beyond the exact bound
            for a in range(3):
                assert ebox[a] - lo[a] <= 2 * sc[a] and hi[a] - ebox[3 + a] <= 2 * sc[a]
            if link & leaf_bit:
                k = int(link & ~leaf_bit)
                assert np.all(ebox[:3] <= tri_box[k, :3]) and np.all(ebox[3:] >= tri_box[k, 3:])
                seen[k] += 1
            else:
                queue.append((int(link), int(el)))
                level_of[int(link)] = level_of[r] + 1
        # inner children: consecutive records, right after everything queued before them
        if inner:
            assert inner == list(range(inner[0], inner[0] + len(inner))), (r, inner)
    assert np.all(seen == 1) if n > 1 else seen[0] == 2
    recs = [r for r, _ in queue]
    assert sorted(recs) == list(range(len(recs)))  # compact: records 0 .. reached - 1
    lv = [level_of[r] for r in range(len(recs))]
    assert lv == sorted(lv)  # level by level
    assert not wide[len(recs):].any()


@pytest.mark.parametrize("n,p,seed", [(8, 0.5, 1), (16, 0.5, 0), (24, 0.7, 2)])
def test_wide_nodes(ctx, n, p, seed):
    m = fg.make_grf_foam(n, p, 2.0, seed=seed)
    sid = ctx.load_scene(m)
    nodes, tris = ctx.bvh_download(sid)
    _check_wide(ctx.bvh_download_wide(sid), nodes, tris, m.n_tris)


def test_wide_node_of_one_triangle(ctx):
    m = fg.flat_plane()
    sid = ctx.load_mesh(m.verts, m.tris[:1], m.box_lo, m.box_hi, m.flags)
    ctx.build_bvh(sid)
    nodes, tris = ctx.bvh_download(sid)
    _check_wide(ctx.bvh_download_wide(sid), nodes, tris, 1)


@pytest.mark.parametrize("n,p,seed", [(8, 0.5, 1), (16, 0.5, 0), (24, 0.7, 2)])
def test_bvh_structure(ctx, n, p, seed):
    m = fg.make_grf_foam(n, p, 2.0, seed=seed)
    sid = ctx.load_scene(m)
    info = ctx.scene_info(sid)
    assert info["n_tris"] == m.n_tris and info["n_dropped"] == 0
    nodes, tris = ctx.bvh_download(sid)
    _check_bvh(nodes, tris, m.n_tris)
    # every caller triangle appears once in the sorted array, unchanged
    oid = tris[:, 3].view(np.int32)
    assert np.array_equal(np.sort(oid), np.arange(m.n_tris))
    assert np.array_equal(tris.reshape(-1, 3, 4)[:, :, :3], m.verts[m.tris[oid]])
    assert 1 <= info["bvh_depth"] < 100


@pytest.mark.parametrize("k", [2, 3, 5, 64, 257])
def test_bvh_of_a_few_triangles(ctx, k):
    """Trees of a few triangles (one workgroup of the level-by-level refit,
    the root reached after one or a few levels, a tree deeper than its
    triangle count suggests when codes collide): every box exact, the depth
    that of the tree."""
    m = fg.make_grf_foam(16, 0.5, 2.0, seed=0)
    sub = fg.Mesh(m.verts, m.tris[:k], m.box_lo, m.box_hi, m.flags, {})
    sid = ctx.load_scene(sub)
    info = ctx.scene_info(sid)
    nodes, tris = ctx.bvh_download(sid)
    _check_bvh(nodes, tris, k)
    links = nodes[:, 12:14].view(np.uint32)

    def height(p):  # internal levels below and including node p (a leaf adds none)
        h = 0
        for side in range(2):
            c = int(links[p, side])
            if not c & 0x80000000:
                h = max(h, height(c))
        return h + 1
    assert info["bvh_depth"] == height(0)


def test_bvh_single_and_empty(ctx):
    m = fg.flat_plane()
    one = fg.Mesh(m.verts, m.tris[:1], m.box_lo, m.box_hi, m.flags, {})
    sid = ctx.load_scene(one)
    nodes, tris = ctx.bvh_download(sid)
    assert nodes.shape[0] == 1
    empty = fg.Mesh(m.verts, m.tris[:0], m.box_lo, m.box_hi, m.flags, {})
    ctx.load_scene(empty)


# ---------------------------------------------------------------- first hit

def _t_tolerance(mesh, rays, tri, t):
    """Bound on |t_GPU - t_oracle| from the FP32 arithmetic of the GPU path.

    Every plane the path crosses -- each periodic wrap face, then the plane it
    ends on (the hit triangle, the substrate or the exit face) -- is located to
    within 16 half-ulps of the cell's largest coordinate magnitude; along the
    ray that error grows as 1 / |cos| of the angle between ray and plane
    normal (clamped at 1e-3).  At least 1e-5 relative."""
    lo, hi = np.array(mesh.box_lo, np.float64), np.array(mesh.box_hi, np.float64)
    q = 16 * 2.0 ** -24 * np.max(np.abs(np.concatenate([lo, hi])))
    o, d = rays[:, :3], rays[:, 3:]
    end = o + np.where(np.isfinite(t), t, 0.0)[:, None] * d
    cos_end = np.ones(len(t))
    hit = tri >= 0
    V = mesh.verts[mesh.tris[tri[hit]]].astype(np.float64)
    n = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    cos_end[hit] = np.abs(np.sum(n * d[hit], axis=1))
    cos_end[tri == -2] = np.abs(d[tri == -2, 2])
    esc = tri == -1
    periodic = bool(mesh.flags & 1)
    if periodic:
        cos_end[esc] = np.abs(d[esc, 2])
    else:  # the exit face: the box face the end point lies on
        gap = np.minimum(np.abs(end - lo), np.abs(end - hi))
        cos_end[esc] = np.abs(d[esc, np.argmin(gap[esc], axis=1)])
    planes = 1.0 / np.maximum(cos_end, 1e-3)
    if periodic:
        for a in (0, 1):
            L = hi[a] - lo[a]
            n_wrap = np.abs(np.floor((end[:, a] - lo[a]) / L) - np.floor((o[:, a] - lo[a]) / L))
            planes += n_wrap / np.maximum(np.abs(d[:, a]), 1e-3)
    return np.maximum(1e-5 * t, q * planes)


def _first_hit_parity(ctx, torch, oracle_lib, mesh, rays64, min_agree, far_t=None):
    """GPU first hits against the oracle's, ray by ray: the same element (or
    a near-tie: a different element at the same distance) and the same path
    length within `_t_tolerance`.  With far_t, a ray whose oracle path is
    longer (tens of grazing periodic wraps, where FP32 re-entry points drift)
    may meet the same triangle one or more cells earlier or later along the
    periodic lattice: the difference of the two hit points must then be a
    lattice vector (n_x L_x, n_y L_y, 0) to within the tolerance."""
    rays32 = rays64.astype(np.float32)
    sid = ctx.load_scene(mesh)
    tri_g, t_g = ctx.first_hit(sid, torch.from_numpy(rays32).cuda())
    tri_g = tri_g.cpu().numpy()
    t_g = t_g.cpu().numpy().astype(np.float64)
    r = rays32.astype(np.float64)
    tri_o, t_o, _ = oracle_lib.first_hit(mesh, r)
    agree = tri_g == tri_o
    frac = agree.mean()
    assert frac >= min_agree, (frac, np.nonzero(~agree)[0][:10])
    fin = tri_o >= -2  # a surface or the exit; lost rays carry no distance
    tol = _t_tolerance(mesh, r, tri_o, t_o)
    err = np.abs(t_g - t_o)
    ok = err <= tol
    if far_t is not None:
        lo, hi = np.array(mesh.box_lo, np.float64), np.array(mesh.box_hi, np.float64)
        delta = np.where(fin & np.isfinite(t_g), t_g - t_o, 0.0)[:, None] * r[:, 3:]
        per = np.array([hi[0] - lo[0], hi[1] - lo[1], np.inf])
        lattice = np.where(np.isfinite(per), np.round(delta / per) * per, 0.0)
        shifted = np.all(np.abs(delta - lattice) <= tol[:, None], axis=1)
        ok |= (t_o > far_t) & agree & shifted
    # the same element at the same distance; disagreements must be near-ties:
    # both found a surface at the same distance
    bad = fin & ~ok
    assert not bad.any(), list(zip(tri_g[bad][:5], tri_o[bad][:5], t_g[bad][:5], t_o[bad][:5], tol[bad][:5]))
    return frac


def test_first_hit_primaries_tiny_foam(ctx, torch, oracle_lib, tiny):
    rays = fg.top_rays(tiny, 20000, seed=7, theta_max_deg=80.0)
    _first_hit_parity(ctx, torch, oracle_lib, tiny, rays, 0.9999)


def test_first_hit_surface_rays_tiny_foam(ctx, torch, oracle_lib, tiny):
    rays = fg.surface_rays(tiny, 20000, seed=8)
    _first_hit_parity(ctx, torch, oracle_lib, tiny, rays, 0.9999)


def test_first_hit_soup_and_plane(ctx, torch, oracle_lib):
    m = fg.random_soup(200, seed=3)
    rng = np.random.default_rng(4)
    o = rng.uniform(0.1, 3.9, size=(5000, 3))
    d = rng.normal(size=(5000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    _first_hit_parity(ctx, torch, oracle_lib, m, np.concatenate([o, d], 1), 0.9999)
    _first_hit_parity(ctx, torch, oracle_lib, fg.trench(), fg.top_rays(fg.trench(), 4000, seed=5), 0.9999)


def _axis_rays(mesh, n, seed):
    """Rays along the axes, rays with one zero direction component and rays
    starting on the lower faces of the cell, origins off the grid lines."""
    rng = np.random.default_rng(seed)
    lo, hi = np.array(mesh.box_lo), np.array(mesh.box_hi)
    o = lo + rng.uniform(0.01, 0.99, size=(3 * n, 3)) * (hi - lo)
    d = np.zeros((3 * n, 3))
    ax = rng.integers(0, 3, n)
    d[np.arange(n), ax] = rng.choice([-1.0, 1.0], n)
    planar = rng.normal(size=(n, 3))
    planar[np.arange(n), rng.integers(0, 3, n)] = 0.0
    d[n:2 * n] = planar / np.linalg.norm(planar, axis=1, keepdims=True)
    face = rng.integers(0, 3, n)
    o[2 * n + np.arange(n), face] = lo[face]
    inward = rng.normal(size=(n, 3))
    inward[np.arange(n), face] = np.abs(inward[np.arange(n), face]) + 0.1
    d[2 * n:] = inward / np.linalg.norm(inward, axis=1, keepdims=True)
    return np.concatenate([o, d], 1)


@pytest.mark.parametrize("shift", [0.0, 1000.0, -500.0])
def test_first_hit_axis_parallel_and_face_rays(ctx, torch, oracle_lib, tiny, shift):
    """The node slab test stays conservative where one direction component is
    zero (reciprocal clamped), where origins lie on cell faces, and in a cell
    far from the coordinate origin (where the slab margin, which scales with
    the largest coordinate, is widest relative to the cell)."""
    m = fg.Mesh(tiny.verts + np.float32(shift), tiny.tris, tuple(v + shift for v in tiny.box_lo),
                tuple(v + shift for v in tiny.box_hi), tiny.flags, {})
    L = max(h - l for l, h in zip(m.box_lo, m.box_hi))
    # 18 000 rays, so that the 99.99 % agreement is a measured rate (at most one near-tie)
    rays = np.concatenate([_axis_rays(m, 3000, seed=seed) for seed in (21, 22)])
    _first_hit_parity(ctx, torch, oracle_lib, m, rays, 0.9999, far_t=4 * L)


@pytest.mark.slow
def test_first_hit_sample_of_128_foam(ctx, torch, oracle_lib):
    """Subsample of rays on the 128^3, porosity 0.6 foam (about 1.9M triangles)."""
    m = fg.make_grf_foam(128, 0.6, 2.0, seed=1)
    rays = np.concatenate([fg.top_rays(m, 5000, seed=11), fg.surface_rays(m, 5000, seed=12)])
    _first_hit_parity(ctx, torch, oracle_lib, m, rays, 0.9999)


# ---------------------------------------------------------------- cascades

def test_flat_plane_yield_is_the_table(ctx, vaughan):
    sid = ctx.load_scene(fg.flat_plane())
    tid = ctx.load_tables(vaughan)
    for E, th in [(500.0, 0.0), (100.0, 30.0), (1000.0, 60.0), (60.0, 80.0)]:
        n = 200000
        r = ctx.trace(sid, tid, E, th, n, seed=11)
        ref = float(fg.bilinear_reference(vaughan, E, th))
        f = ref - math.floor(ref)
        assert abs(r["yield"] - ref) <= 3 * math.sqrt(f * (1 - f) / n), (E, th, r["yield"], ref)
        assert r["n_escaped"] == r["n_rays"] - n


@pytest.mark.parametrize("const", [0.0, 1.0, 2.0])
def test_flat_plane_integral_yields(ctx, const):
    sid = ctx.load_scene(fg.flat_plane())
    tid = ctx.load_tables(fg.make_tables("constant", const=const))
    n = 50000
    r = ctx.trace(sid, tid, 300.0, 20.0, n, seed=3)
    assert r["n_escaped"] == int(const) * n and r["yield_sigma"] == 0.0


def test_trench_view_factor(ctx, vaughan):
    sid = ctx.load_scene(fg.trench())
    tid = ctx.load_tables(vaughan)
    r = ctx.trace(sid, tid, 500.0, 0.0, 400000, seed=21, max_gen=1)
    d0 = float(fg.bilinear_reference(vaughan, 500.0, 0.0))
    F = math.sqrt(1 + 1.5 ** 2) - 1.5
    expect = d0 * (1 / 3 + 2 / 3 * F)
    assert abs(r["yield"] - expect) <= 3 * r["yield_sigma"], (r["yield"], expect)


def test_yield_parity_tiny_foam(ctx, torch, oracle_lib, tiny, vaughan):
    """The 16^3 foam, 1e4 primaries at 500 eV, normal incidence: paired and unpaired."""
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    n = 10000
    pp = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    g = ctx.trace(sid, tid, 500.0, 0.0, n, seed=1, per_primary=pp)
    o = oracle_lib.trace(tiny, vaughan, 500.0, 0.0, n, seed=1, per_primary=True)
    sig = math.sqrt(g["yield_sigma"] ** 2 + o["yield_sigma"] ** 2)
    assert abs(g["yield"] - o["yield"]) <= 3 * sig
    ppg = pp.cpu().numpy().astype(np.int64)
    ppo = o["per_primary"]["escaped"].astype(np.int64)
    assert int(ppg.sum()) == g["n_escaped"]
    same = (ppg == ppo).mean()
    assert same >= 0.995, same
    diff = ppg - ppo
    assert abs(diff.mean()) <= 3 * diff.std(ddof=1) / math.sqrt(n) + 1e-12


@pytest.mark.slow
def test_full_size_sweep_batch_equals_single_traces(ctx, vaughan):
    """The benchmark's 128^3 sweep (5 energies x 5 angles, 1e7 primaries per
    point, max_gen 6) in the launch shape it times -- one rtmc_trace_batch with
    2^28-primary chunks (one chunk for all 25 points), the single-scene kernel, a
    directly launched sequence -- gives every point the integer tallies of its
    own rtmc_trace (which the sampled oracle test pins at full size)."""
    m = fg.make_grf_foam(128, 0.6, 2.0, seed=1)
    sid = ctx.load_scene(m)
    tid = ctx.load_tables(vaughan)
    pts = [(E, th) for E in (50.0, 100.0, 250.0, 500.0, 1000.0) for th in (0.0, 20.0, 40.0, 60.0, 80.0)]
    jobs = [(sid, E, th, 10_000_000, 2000 + k) for k, (E, th) in enumerate(pts)]
    cfg = ctx.get_launch()
    ctx.set_launch(cfg["block"], cfg["wg_per_cu"], cfg["lds_stack"], 1 << 28, cfg["refill"], cfg["occupancy"])
    try:
        outs = ctx.trace_batch(tid, jobs, max_gen=6)
    finally:
        ctx.set_launch(**cfg)
    assert outs[0]["n_chunks"] == 1 and outs[0]["kernel_ms"] > 0.0
    for (s, E, th, n, sd), b in zip(jobs, outs):
        r = ctx.trace(s, tid, E, th, n, seed=sd, max_gen=6)
        for key in ("n_rays", "n_escaped", "n_absorbed", "n_truncated", "n_lost", "n_substrate", "n_tri_tests",
                    "n_node_visits", "n_wraps", "n_spawned", "e_escaped", "e_deposited"):
            assert b[key] == r[key], (E, th, key, b[key], r[key])
        assert b["yield_sigma"] == pytest.approx(r["yield_sigma"], rel=1e-12)


@pytest.mark.slow
@pytest.mark.parametrize("grid,porosity,seed,theta,n,max_gen,k", [
    (128, 0.6, 1, 40.0, 10_000_000, 6, 512),    # one point of the 128^3 sweep (1.91M triangles)
    (256, 0.8, 4, -80.0, 100_000_000, 10, 192),  # the 256^3 run (11.0M triangles), random incidence
])
def test_full_size_point_sampled_against_oracle(ctx, torch, oracle_lib, vaughan, grid, porosity, seed, theta, n,
                                                max_gen, k):
    """A point of the benchmark workloads at full size (every primary, the
    default launch shape the benchmark times): the escape counts of the first
    k primaries against the oracle, which traces them one by one over every
    triangle, and the conservation laws over all n primaries."""
    m = fg.make_grf_foam(grid, porosity, 2.0, seed=seed)
    sid = ctx.load_scene(m)
    tid = ctx.load_tables(vaughan)
    pp = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    g = ctx.trace(sid, tid, 250.0, theta, n, seed=2000 + seed, max_gen=max_gen, per_primary=pp)
    o = oracle_lib.trace(m, vaughan, 250.0, theta, k, seed=2000 + seed, max_gen=max_gen, per_primary=True)
    ppg = pp[:k].cpu().numpy().astype(np.int64)
    same = (ppg == o["per_primary"]["escaped"].astype(np.int64)).mean()
    # a primary's whole cascade must take the same branches on both sides; at
    # most one cascade in a hundred may part at a near-tie (observed: none)
    assert same >= 0.99, same
    assert int(pp.sum().item()) == g["n_escaped"]
    assert g["e_escaped"] + g["e_deposited"] == pytest.approx(250.0 * n, rel=1e-12)
    assert g["n_rays"] == g["n_escaped"] + g["n_absorbed"] + g["n_truncated"] + g["n_lost"] == n + g["n_spawned"]
    assert int(g["e_hist"].sum()) == g["n_escaped"] == int(g["a_hist"].sum())
    assert g["n_lost"] == 0


@pytest.mark.parametrize("E,theta", [(100.0, 0.0), (800.0, 40.0), (250.0, -80.0)])
def test_yield_parity_points(ctx, oracle_lib, tiny, vaughan, E, theta):
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    n = 6000
    g = ctx.trace(sid, tid, E, theta, n, seed=2)
    o = oracle_lib.trace(tiny, vaughan, E, theta, n, seed=2)
    sig = math.sqrt(g["yield_sigma"] ** 2 + o["yield_sigma"] ** 2)
    assert abs(g["yield"] - o["yield"]) <= 3 * sig


def test_conservation_and_counts(ctx, tiny, vaughan):
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    n = 50000
    r = ctx.trace(sid, tid, 700.0, -80.0, n, seed=5, max_gen=6)
    assert r["e_escaped"] + r["e_deposited"] == pytest.approx(700.0 * n, rel=1e-12)
    assert r["n_rays"] == r["n_escaped"] + r["n_absorbed"] + r["n_truncated"] + r["n_lost"]
    assert r["n_rays"] == n + r["n_spawned"]
    assert int(r["e_hist"].sum()) == r["n_escaped"] == int(r["a_hist"].sum())


def test_resume_and_determinism(ctx, torch, tiny, vaughan):
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    n, k = 30000, 12345
    full = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    a = torch.zeros(k, dtype=torch.int32, device="cuda:0")
    b = torch.zeros(n - k, dtype=torch.int32, device="cuda:0")
    r = ctx.trace(sid, tid, 400.0, 30.0, n, seed=9, per_primary=full)
    ra = ctx.trace(sid, tid, 400.0, 30.0, k, seed=9, per_primary=a)
    rb = ctx.trace(sid, tid, 400.0, 30.0, n - k, seed=9, pid0=k, per_primary=b)
    assert torch.equal(full, torch.cat([a, b]))
    assert r["n_escaped"] == ra["n_escaped"] + rb["n_escaped"]
    assert np.array_equal(r["e_hist"], ra["e_hist"] + rb["e_hist"])
    r2 = ctx.trace(sid, tid, 400.0, 30.0, n, seed=9)
    for key in ("n_rays", "n_escaped", "n_node_visits", "n_tri_tests", "e_escaped"):
        assert r2[key] == r[key]


def test_chunking_does_not_change_results(ctx, tiny, vaughan):
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    cfg = ctx.get_launch()
    r1 = ctx.trace(sid, tid, 500.0, 0.0, 20000, seed=4)
    ctx.set_launch(cfg["block"], cfg["wg_per_cu"], cfg["lds_stack"], 3000)
    try:
        r2 = ctx.trace(sid, tid, 500.0, 0.0, 20000, seed=4)
    finally:
        ctx.set_launch(**cfg)
    assert r2["n_chunks"] == 7
    for key in ("n_rays", "n_escaped", "n_absorbed", "e_escaped", "n_tri_tests"):
        assert r1[key] == r2[key]
    assert np.array_equal(r1["e_hist"], r2["e_hist"])


def test_batch_equals_single_jobs(ctx, tiny, vaughan):
    s1 = ctx.load_scene(tiny)
    s2 = ctx.load_scene(fg.make_grf_foam(12, 0.7, 2.0, seed=5))
    tid = ctx.load_tables(vaughan)
    jobs = [(s1, 500.0, 0.0, 7000, 1), (s2, 100.0, 40.0, 3000, 2), (s1, 250.0, -80.0, 5000, 3),
            (s2, 1000.0, 60.0, 1, 4)]
    outs = ctx.trace_batch(tid, jobs, max_gen=6)
    for (s, E, th, n, sd), b in zip(jobs, outs):
        r = ctx.trace(s, tid, E, th, n, seed=sd, max_gen=6)
        for key in ("n_rays", "n_escaped", "n_absorbed", "n_truncated", "n_lost", "n_tri_tests", "n_node_visits",
                    "e_escaped"):
            assert b[key] == r[key], (key, b[key], r[key])


def test_batch_of_many_small_jobs(ctx, tiny, vaughan):
    """40 small jobs on two scenes fit one chunk that spans more jobs than
    shading keeps tallies for in LDS: the per-wave tallies and their flushes
    to each job's global block on every change of job must still give every
    job the integer tallies of its own trace."""
    s1 = ctx.load_scene(tiny)
    s2 = ctx.load_scene(fg.make_grf_foam(12, 0.7, 2.0, seed=5))
    tid = ctx.load_tables(vaughan)
    rng = np.random.default_rng(17)
    jobs = [((s1, s2)[k % 3 == 0], float(rng.uniform(30.0, 1500.0)), float(rng.uniform(-85.0, 85.0)),
             int(rng.integers(1, 400)), 500 + k) for k in range(40)]
    outs = ctx.trace_batch(tid, jobs, max_gen=6)
    assert outs[0]["n_chunks"] == 1
    for (s, E, th, n, sd), b in zip(jobs, outs):
        r = ctx.trace(s, tid, E, th, n, seed=sd, max_gen=6)
        for k in ("n_primaries", "n_rays", "n_escaped", "n_absorbed", "n_truncated", "n_lost", "n_tri_tests",
                  "n_node_visits", "n_spawned", "e_escaped", "e_deposited"):
            assert b[k] == r[k], (E, th, n, k, b[k], r[k])


def test_errors_are_reported(ctx, vaughan):
    import paper_1806_00205_amd as rt
    m = fg.flat_plane()
    sid = ctx.load_mesh(m.verts, m.tris, m.box_lo, m.box_hi, m.flags)
    tid = ctx.load_tables(vaughan)
    with pytest.raises(rt.RtmcError) as e:
        ctx.trace(sid, tid, 500.0, 0.0, 10, seed=1)
    assert e.value.status == -4  # no BVH yet
    bad = m.verts.copy()
    bad[0, 0] = np.nan
    with pytest.raises(rt.RtmcError):
        ctx.load_mesh(bad, m.tris, m.box_lo, m.box_hi, m.flags)
    with pytest.raises(rt.RtmcError):
        ctx.load_mesh(m.verts, m.tris + 10, m.box_lo, m.box_hi, m.flags)
    zero = fg.Mesh(np.concatenate([m.verts, m.verts[:1]]), np.concatenate([m.tris, [[4, 4, 0]]]).astype(np.int32),
                   m.box_lo, m.box_hi, m.flags, {})
    s2 = ctx.load_scene(zero)
    assert ctx.scene_info(s2)["n_dropped"] == 1


def test_batch_graph_replays_match_eager(ctx, tiny, vaughan):
    """rtmc_trace_batch records a long launch sequence (here 128-primary
    chunks: over 128 traversal launches) once as a HIP graph and replays it
    for later calls of the same shape: replay it several times, with eager
    traces (other kernels, synchronisations) in between, and check every
    replay against the eager single-job results."""
    s1 = ctx.load_scene(tiny)
    s2 = ctx.load_scene(fg.make_grf_foam(12, 0.7, 2.0, seed=5))
    tid = ctx.load_tables(vaughan)
    keys = ("n_rays", "n_escaped", "n_absorbed", "n_truncated", "n_lost", "n_tri_tests", "n_node_visits",
            "e_escaped", "e_deposited")
    cfg = ctx.get_launch()
    for rep in range(4):
        seeds = (11 + rep, 12 + rep, 13 + rep)
        jobs = [(s1, 500.0, 0.0, 3000, seeds[0]), (s2, 150.0, 30.0, 2000, seeds[1]),
                (s1, 900.0, -80.0, 2500, seeds[2])]
        ctx.set_launch(cfg["block"], cfg["wg_per_cu"], cfg["lds_stack"], 128)
        try:
            outs = ctx.trace_batch(tid, jobs, max_gen=6)
        finally:
            ctx.set_launch(**cfg)
        assert outs[0]["n_kernel_launches"] > 128 and outs[0]["kernel_ms"] == 0.0  # replayed graph
        eager = [ctx.trace(s, tid, E, th, n, seed=sd, max_gen=6) for s, E, th, n, sd in jobs]
        for b, r in zip(outs, eager):
            for k in keys:
                assert b[k] == r[k], (rep, k, b[k], r[k])


def test_same_scene_batch_runs_directly(ctx, tiny, vaughan):
    """A sweep of (E, theta) points on one scene as one batch: a short launch
    sequence runs directly (every launch timed) with the single-scene
    traversal kernel, chunks spanning several points; integer tallies equal
    the points traced one by one."""
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    jobs = [(sid, E, th, 4000 + 500 * k, 30 + k) for k, (E, th) in
            enumerate([(50.0, 0.0), (250.0, 40.0), (1000.0, 80.0), (500.0, -60.0), (100.0, 20.0)])]
    outs = ctx.trace_batch(tid, jobs, max_gen=6)
    assert outs[0]["n_chunks"] == 1 and outs[0]["n_kernel_launches"] == 7
    for (s, E, th, n, sd), b in zip(jobs, outs):
        assert b["kernel_ms"] > 0.0 and b["shade_ms"] > 0.0
        r = ctx.trace(s, tid, E, th, n, seed=sd, max_gen=6)
        for k in ("n_rays", "n_escaped", "n_absorbed", "n_truncated", "n_lost", "n_tri_tests", "n_node_visits",
                  "n_wraps", "e_escaped", "e_deposited"):
            assert b[k] == r[k], (E, th, k, b[k], r[k])


def test_irregular_spectrum_table(ctx, oracle_lib):
    """Secondary energies from an irregular CDF (uneven nodes, plateaus where F
    stays flat, steep jumps): the GPU's look-ups land in the same segments as
    the oracle's scan, so the escaped-energy histograms of the same primaries
    agree bin by bin up to FP32 rounding."""
    rng = np.random.default_rng(3)
    n_cdf = 300
    cE = np.concatenate([[0.0], np.sort(rng.uniform(0.05, 900.0, n_cdf - 1))]).astype(np.float32)
    steps = rng.exponential(1.0, n_cdf - 1)
    steps[rng.random(n_cdf - 1) < 0.2] = 0.0  # plateaus
    steps[rng.integers(0, n_cdf - 1, 5)] *= 40.0  # jumps
    cF = np.concatenate([[0.0], np.cumsum(steps)])
    cF = (cF / cF[-1]).astype(np.float32)
    cF[-1] = 1.0
    assert np.all(np.diff(cE) > 0) and np.all(np.diff(cF) >= 0)
    tab = fg.make_tables("constant", const=1.0)
    tab.cdf_E, tab.cdf_F = cE, cF
    sid = ctx.load_scene(fg.flat_plane())
    tid = ctx.load_tables(tab)
    n = 20000
    E0 = 700.0
    g = ctx.trace(sid, tid, E0, 0.0, n, seed=19, max_gen=1, n_ebins=350)
    o = oracle_lib.trace(fg.flat_plane(), tab, E0, 0.0, n, seed=19, max_gen=1, n_ebins=350)
    assert g["n_escaped"] == o["n_escaped"] == n
    diff = np.abs(g["e_hist"].astype(np.int64) - o["e_hist"].astype(np.int64)).sum()
    assert diff <= 0.002 * n, diff
    assert g["e_escaped"] == pytest.approx(o["e_escaped"], rel=1e-4)


LAUNCHES = [(256, 7, 16, 1 << 24, 48, 0, 0), (128, 12, 8, 5000, 24, 8, 8192), (64, 24, 24, 1 << 20, 64, 0, 64),
            (256, 2, 4, 3000, 1, 0, 512), (256, 6, 16, 1 << 24, 40, 6, 4096), (256, 8, 16, 1 << 24, 48, 7, 2048)]


def test_launch_shapes_do_not_change_results(ctx, tiny, vaughan):
    """Block size, workgroups per CU, LDS stack depth, chunking, refill threshold,
    the register-capped kernel builds and the rays a wave claims at once change
    only speed: every tally, the traversal work counters included, is identical."""
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    cfg = ctx.get_launch()
    keys = ("n_rays", "n_escaped", "n_absorbed", "n_truncated", "n_lost", "n_substrate", "n_wraps",
            "n_node_visits", "n_tri_tests", "n_spawned", "e_escaped", "e_deposited")
    try:
        ref = None
        for launch in LAUNCHES:
            ctx.set_launch(*launch)
            r = ctx.trace(sid, tid, 400.0, -60.0, 12000, seed=23, max_gen=8)
            got = {k: r[k] for k in keys}
            got["e_hist"] = r["e_hist"].tolist()
            if ref is None:
                ref = got
            assert got == ref, launch
    finally:
        ctx.set_launch(**cfg)


def test_autotune_keeps_results(ctx, tiny, vaughan):
    """The tuned launch (block, workgroups per CU, stack, refill, build, rays per
    wave per claim, chunk) keeps every integer tally; a second call with the
    same key takes the cached shape without timing anything."""
    import time
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    cfg = ctx.get_launch()
    try:
        before = ctx.trace(sid, tid, 300.0, 20.0, 8000, seed=29)
        t0 = time.perf_counter()
        best = ctx.autotune(sid, tid, 300.0, 20.0, 20000)
        t_tune = time.perf_counter() - t0
        assert best == ctx.get_launch()
        assert best["block"] in (64, 128, 256) and best["wg_per_cu"] >= 1 and 1 <= best["refill"] <= 64
        assert best["claim"] in (512, 1024, 2048, 4096, 8192)
        # chunks of at least the calibration trace's length are all one chunk to
        # it: the current chunk stays unless a real split (a half, a quarter) wins
        assert best["chunk"] in (10000, 5000, cfg["chunk"])
        after = ctx.trace(sid, tid, 300.0, 20.0, 8000, seed=29)
        for k in ("n_rays", "n_escaped", "n_absorbed", "n_node_visits", "n_tri_tests", "e_escaped", "e_deposited"):
            assert before[k] == after[k], k
        ctx.set_launch(**cfg)
        t0 = time.perf_counter()
        again = ctx.autotune(sid, tid, 300.0, 20.0, 20000)
        t_cached = time.perf_counter() - t0
        assert again == best and ctx.get_launch() == best
        assert t_cached < 0.1 * t_tune, (t_cached, t_tune)
    finally:
        ctx.set_launch(**cfg)


def test_copy_probe_copies_and_measures(ctx, torch):
    import ctypes as C
    n = 1 << 22
    src = torch.arange(n, dtype=torch.float32, device="cuda:0")
    dst = torch.zeros_like(src)
    ms = C.c_double()
    st = ctx.lib.rtmc_copy_probe(ctx.h, C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), n * 4, 3,
                                 C.byref(ms))
    assert st == 0 and ms.value > 0
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    gbps = ctx.copy_probe(1 << 28, reps=3)
    assert 500.0 < gbps < 10000.0


def test_work_on_another_stream(ctx, torch, tiny, vaughan):
    sid = ctx.load_scene(tiny)
    tid = ctx.load_tables(vaughan)
    ref = ctx.trace(sid, tid, 600.0, 0.0, 5000, seed=31)
    s = torch.cuda.Stream()
    try:
        with torch.cuda.stream(s):
            ctx.set_stream(s)
            r = ctx.trace(sid, tid, 600.0, 0.0, 5000, seed=31)
    finally:
        ctx.set_stream(torch.cuda.current_stream())
    for k in ("n_rays", "n_escaped", "n_tri_tests", "e_escaped"):
        assert r[k] == ref[k], k
