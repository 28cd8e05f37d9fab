"""ts_bin_sort_noalloc (scratch in a static device array, no workspace argument) gives the same
depth order, tile ranges, tile lists, pair count and status as ts_bin_sort with a workspace,
bit for bit, on two calls in a row (the second smaller, so stale scratch from the first call
is present), and refuses a call whose scratch exceeds the static array on the host."""
import sys

import numpy as np
import pytest
import torch

import synth
from paper_2506_13348_amd import DeviceScene, RenderPlan
from paper_2506_13348_amd import _ffi as F

pytestmark = pytest.mark.gpu


def _outputs(plan, cap):
    dev = plan.scene.device
    i32 = dict(device=dev, dtype=torch.int32)
    return dict(sorted_ids=torch.full((plan.V * max(plan.scene.n, 1),), -7, **i32),
                tile_ranges=torch.full((plan.V * plan.n_tiles * 2,), -7, **i32),
                pair_ids=torch.full((max(cap, 1),), -7, **i32),
                n_pairs=torch.full((1,), -7, device=dev, dtype=torch.int64),
                status=torch.full((1,), -7, **i32))


def _compare(name, n, views, W, H, cap_scale=1.0):
    print(f"no-alloc case {name}: n={n} views={views} {W}x{H}", flush=True)
    sc = synth.make_scene("sq100k", n=n, tex_res=2, env_res=16)
    ds = DeviceScene.from_dict(sc, device="cuda:0")
    cams = synth.orbit_cameras(views, W, H, dist=2.8)
    plan = RenderPlan(ds, cams, W, H, shade=False)       # sizes the capacity from a probe run
    cap = int(plan.cap * cap_scale)
    plan.preprocess()
    a, b = _outputs(plan, cap), _outputs(plan, cap)
    F.ts_bin_sort(plan.V, W, H, ds.n, plan.rect, plan.depth_key, plan.ws, cap, a["sorted_ids"],
                  a["tile_ranges"], a["pair_ids"], a["n_pairs"], a["status"])
    F.ts_bin_sort_noalloc(plan.V, W, H, ds.n, plan.rect, plan.depth_key, cap, b["sorted_ids"],
                          b["tile_ranges"], b["pair_ids"], b["n_pairs"], b["status"])
    torch.cuda.synchronize()
    npairs = int(a["n_pairs"].item())
    assert npairs == int(b["n_pairs"].item()) and npairs > 0
    assert int(a["status"].item()) == int(b["status"].item())
    for k in ("sorted_ids", "tile_ranges"):
        assert torch.equal(a[k], b[k]), k
    m = min(npairs, cap)
    assert torch.equal(a["pair_ids"][:m], b["pair_ids"][:m])
    return npairs, int(b["status"].item())


def test_noalloc_matches_workspace_call_twice_second_smaller():
    big = _compare("first", 40000, 3, 320, 240)
    small = _compare("second", 5000, 1, 96, 80)
    assert big[0] > small[0]
    assert big[1] == 0 and small[1] == 0


def test_noalloc_reports_overflow_like_the_workspace_call():
    npairs, status = _compare("overflow", 8000, 2, 160, 128, cap_scale=0.5)
    assert status == 1


def test_noalloc_refuses_scratch_above_the_static_array():
    one = torch.zeros(16, device="cuda:0", dtype=torch.int32)
    # 64 views of 1M splats at 1920x1080 need far more than the static array
    need = F.ts_workspace_size(F.TS_OP_BIN_SORT, 64, 1_000_000, 1920, 1080)
    assert need > F.ts_bin_sort_noalloc_max_bytes()
    with pytest.raises(RuntimeError, match="static array"):
        F.ts_bin_sort_noalloc(64, 1920, 1080, 1_000_000, one, one, 16, one, one, one,
                              one.view(torch.int64), one)


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-v"]))
