"""nx_render_forward_noalloc (the forward whose intermediates live in the
library's fixed scratch array) against nx_render_forward_async with a
caller-allocated workspace, through the C ABI (needs an MI355X).

Two calls in a row, the second on a smaller input (fewer surfels, fewer and
smaller cameras), each compared bit for bit with the workspace entry point on
the same inputs: the scratch keeps the first call's contents, so the second
call checks that nothing depends on it being cleared. A size beyond the
scratch is rejected with NX_ERR_UNSUPPORTED before anything is launched.
"""
from __future__ import annotations

import pytest
import torch

import scenes
from tests.gpu_helpers import device_inputs, log

pytestmark = pytest.mark.gpu

FWD_FIELDS = ("image", "plain", "ids", "weights", "depths", "t_final", "tex", "n_iter")


@pytest.fixture(scope="module")
def nx():
    import paper_2512_13796_amd as m
    return m


def _compare(nx, wl, cams, label):
    surf, table, weights = device_inputs(wl)
    ctx = nx.Context(wl.K, table.dtype, weights[0].dtype)
    ref = nx.render_forward(ctx, surf, cams, table, wl.grid.level_scales, weights)
    cap = max(ref.n_instances_cam) + 64
    asy = nx.render_forward(ctx, surf, cams, table, wl.grid.level_scales, weights, max_instances=cap)
    res = nx.render_forward_noalloc(ctx, surf, cams, table, wl.grid.level_scales, weights, max_instances=cap)
    torch.cuda.synchronize()
    log(f"{label}: {wl.scene.n} surfels, {len(cams)} cameras, instances {ref.n_instances_cam}, bound {cap}")
    assert res.n_instances_cam == [cap] * len(cams)
    for nm in FWD_FIELDS:
        assert torch.equal(getattr(res, nm), getattr(asy, nm)), f"{label}: {nm} differs from the async forward"
        assert torch.equal(getattr(res, nm), getattr(ref, nm)), f"{label}: {nm} differs from the synced forward"
    return ctx, surf, table, weights


def test_noalloc_forward_equals_workspace_forward_twice(nx):
    big = scenes.make_workload(4, seed=3, n_surfels=10_000)
    _compare(nx, big, big.cameras[:2], "first call")
    small = scenes.make_workload(1, seed=4, width=75, height=53)
    _compare(nx, small, small.cameras[:1], "second call (smaller)")


def test_noalloc_rejects_sizes_beyond_the_scratch(nx):
    from paper_2512_13796_amd import _lib as L
    wl = scenes.make_workload(1, seed=0, width=64, height=64)
    surf, table, weights = device_inputs(wl)
    ctx = nx.Context(wl.K, table.dtype, weights[0].dtype)
    with pytest.raises(L.NexelsError) as err:
        nx.render_forward_noalloc(ctx, surf, wl.cameras[0], table, wl.grid.level_scales, weights,
                                  max_instances=1 << 26)
    assert err.value.code == L.NX_ERR_UNSUPPORTED
    assert "scratch" in str(err.value)
