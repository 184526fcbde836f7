"""Spherical-harmonics appearance through the C ABI against the FP64 oracle (needs an MI355X).

Representation, Appearance and Results (degree-3 SH, 48 coefficients per
surfel and 48 MLP outputs): the plain colour is decoded along the direction
from the camera centre to the surfel centre, the texture along the pixel's
ray (both max(0, sum_k Y_k a_k + 0.5)). Same acceptance as the RGB form:
ids bit-exact on decisive pixels, image / textures within 1e-5 (FP32 form),
gradients (including the 48 coefficients per surfel, the centre's gradient
through the view direction and the 48-row head) within relative L2 1e-3 and
the per-element rule; the BF16 form against the BF16 bar. Covered: K = 0
(colours only), K = 4, hidden width 64 and 128, FP32 and BF16 forms (both at
hidden width 128).
"""
from __future__ import annotations

import pytest
import torch

import scenes
from tests.test_gpu_parity import BF16_VIOL, _forward_case, _grad_case, _sample_pixels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nx():
    import paper_2512_13796_amd as m
    return m


def test_sh_forward_small_full_frame(nx):
    _forward_case(nx, scenes.with_sh(scenes.make_workload(1)), label="sh c1 fwd")


@pytest.mark.parametrize("K", [0, 4])
def test_sh_backward_small(nx, K):
    wl = scenes.with_sh(scenes.make_workload(1, seed=3, width=64, height=64))
    _grad_case(nx, wl, K=K, label=f"sh K={K}")


def test_sh_backward_hidden128_fp32(nx):
    wl = scenes.make_workload(5, seed=9, n_surfels=40_000, width=160, height=90, feat_dtype=torch.float32,
                              mlp_dtype=torch.float32)
    wl = scenes.with_sh(wl, seed=9)
    pix = _sample_pixels(wl.cameras[0], 3, per_block=16, full_tiles=2)
    _grad_case(nx, wl, label="sh h128 fp32", pixels=pix)


def test_sh_backward_hidden128_bf16(nx):
    """The 48-output head at hidden width 128 in the BF16 form (BF16 grid and MLP): the texture backward runs
    8-wave workgroups there. BF16 bars as for the RGB head at this width."""
    wl = scenes.make_workload(5, seed=11, n_surfels=40_000, width=160, height=90)
    wl = scenes.with_sh(wl, seed=11)
    pix = _sample_pixels(wl.cameras[0], 5, per_block=16, full_tiles=2)
    _grad_case(nx, wl, label="sh h128 bf16", pixels=pix, rel_tol=5e-2, bf16_bound=BF16_VIOL, tol_fwd=1e-3)


def test_sh_bf16_form_sampled(nx):
    """FP16 grid + BF16 MLP with the 48-output head at 1080p on a pixel sample: the BF16 bar for the table and
    MLP gradients; the surfel gradients (SH coefficients included) stay near FP32 accuracy."""
    wl = scenes.with_sh(scenes.make_workload(3))
    pix = _sample_pixels(wl.cameras[0], 11, per_block=64, full_tiles=2)
    rep = _grad_case(nx, wl, label="sh c3 bf16", pixels=pix, rel_tol=5e-2, bf16_bound=BF16_VIOL, tol_fwd=1e-3,
                     max_nd=3e-3)
    for nm in ("means", "quats", "scales", "opacities", "gammas", "colors"):
        assert rep[nm]["rel_l2"] <= 1e-3, f"{nm}: {rep[nm]['rel_l2']:.2e}"


def test_sh_joint_cameras_equal_single_calls(nx):
    """Several cameras in one call with the SH appearance: each camera's plain colours are decoded along its
    own view directions, so the joint forward must equal the single-camera calls bit for bit, and the joint
    backward (SH coefficients included) their summed gradients up to float32 atomic order."""
    from tests.gpu_helpers import device_inputs
    wl = scenes.with_sh(scenes.make_workload(4, seed=2, n_surfels=20_000))
    cams = wl.cameras[:3]
    surf, table, weights = device_inputs(wl)
    ctx = nx.Context(wl.K, table.dtype, weights[0].dtype, sh_degree=3)
    res = nx.render_forward(ctx, surf, cams, table, wl.grid.level_scales, weights)
    P = res.image.shape[0]
    gi = torch.randn(P, 3, device="cuda", generator=torch.Generator(device="cuda").manual_seed(4))
    z = lambda t: torch.zeros(t.shape, device=t.device, dtype=torch.float32)
    joint = {"means": z(surf[0]), "colors": z(surf[5]), "table": z(table)}
    nx.render_backward(ctx, surf, res, table, wl.grid.level_scales, weights, gi, None, None, joint)
    single = {k: z(v) for k, v in joint.items()}
    off = 0
    for cam in cams:
        n = cam.width * cam.height
        one = nx.render_forward(ctx, surf, cam, table, wl.grid.level_scales, weights)
        torch.cuda.synchronize()
        for nm in ("image", "plain", "tex"):
            assert torch.equal(getattr(res, nm)[off:off + n], getattr(one, nm)), nm
        nx.render_backward(ctx, surf, one, table, wl.grid.level_scales, weights, gi[off:off + n].contiguous(), None,
                           None, single)
        off += n
    torch.cuda.synchronize()
    for k in joint:
        a, b = joint[k].double(), single[k].double()
        rel = float((a - b).norm() / max(float(b.norm()), 1e-30))
        assert rel <= 1e-4, f"{k}: joint vs summed single-camera gradients rel {rel:.2e}"
