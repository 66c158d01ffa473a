"""rtmc_first_hit_noalloc, the first-hit entry point that allocates nothing,
against rtmc_first_hit through the C interface: identical triangle codes
and distances on two calls in a row (the second smaller), no allocation
through the context's allocator, and sizes beyond its limit refused."""
import numpy as np
import pytest

import foamgen as fg

pytestmark = pytest.mark.gpu

MAX_RAYS = 1 << 19


def _rays(m, n, seed):
    return np.concatenate([fg.top_rays(m, n // 2, seed=seed), fg.surface_rays(m, n - n // 2, seed=seed + 10)])


def test_first_hit_without_allocation_equals_first_hit():
    import torch

    import paper_1806_00205_amd as rt
    ctx = rt.Context(0)
    try:
        for grid, seed in ((24, 7), (48, 3)):
            m = fg.make_grf_foam(grid, 0.6, 2.0, seed=seed)
            sid = ctx.load_scene(m)
            for n, rs in ((MAX_RAYS, 1), (777, 2)):
                r = torch.from_numpy(_rays(m, n, rs).astype(np.float32)).cuda()
                tri_ref, t_ref = ctx.first_hit(sid, r)
                tri = torch.full((n,), -7, dtype=torch.int32, device="cuda:0")
                t = torch.full((n,), -1.0, dtype=torch.float32, device="cuda:0")
                torch.cuda.synchronize()
                allocs = torch.cuda.memory_stats()["allocation.all.allocated"]
                ctx.first_hit_noalloc(sid, r, tri, t)
                torch.cuda.synchronize()
                assert torch.cuda.memory_stats()["allocation.all.allocated"] == allocs
                assert torch.equal(tri, tri_ref), (grid, n, int((tri != tri_ref).sum()))
                assert torch.equal(t, t_ref), (grid, n)
                assert int((tri >= 0).sum()) > n // 4
        big = torch.zeros((MAX_RAYS + 1, 6), dtype=torch.float32, device="cuda:0")
        tri = torch.zeros(MAX_RAYS + 1, dtype=torch.int32, device="cuda:0")
        t = torch.zeros(MAX_RAYS + 1, dtype=torch.float32, device="cuda:0")
        with pytest.raises(rt.RtmcError) as e:
            ctx.first_hit_noalloc(sid, big, tri, t)
        assert e.value.status == -1
    finally:
        ctx.close()
