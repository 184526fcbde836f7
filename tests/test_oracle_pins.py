"""Pins of the FP64 oracle against closed forms, invariants, limits, brute
force and finite differences (CPU only).

Each test names the part of the paper it checks. None re-types the oracle's
own expression and compares it with itself: the expected values come from an
independent special case, a property the mathematics fixes, or a separate
evaluation route.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest
import torch
from scipy.special import erf

import oracle
import scenes
from oracle.binning import bin_surfels
from oracle.constants import ALPHA_MIN, PRIMES
from oracle.geometry import kernel
from oracle.hashgrid import downweight, encode, map_positive, spatial_hash
from oracle.mlp import mlp_forward
from tests.oracle_cases import (constant_grid, facing_scene, identity_camera, random_grid, random_mlp,
                                scene_from)

HERE = os.path.dirname(os.path.abspath(__file__))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _np_mlp(z, ws):
    h = z
    for i, w in enumerate(ws):
        h = h @ np.asarray(w, dtype=np.float64).T
        h = _sigmoid(h) if i == len(ws) - 1 else np.maximum(h, 0.0)
    return h


# ---------------------------------------------------------------- single surfel

def _single_surfel_expect(cam, mu, sig, opac):
    """Closed form for an axis-aligned surfel facing an identity camera.

    The plane is z = mu_z, so t* = mu_z for every pixel; the hit point is
    (mu_z dx, mu_z dy) and u, v are its offsets from the centre in units of
    the scales (Preliminaries: (u, v) in primitive space; Geometry: alpha).
    """
    W, H = cam.width, cam.height
    py, px = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    dx = (px + 0.5 - cam.cx) / cam.fx
    dy = (py + 0.5 - cam.cy) / cam.fy
    u = (mu[2] * dx - mu[0]) / sig[0]
    v = (mu[2] * dy - mu[1]) / sig[1]
    G = np.exp(-0.5 * (u * u + v * v))
    a = opac * G
    ok = (np.abs(u) <= 3) & (np.abs(v) <= 3) & (a >= ALPHA_MIN)
    return np.where(ok, a, 0.0).reshape(-1), np.where(ok, G, 0.0).reshape(-1), dx.reshape(-1), dy.reshape(-1)


def test_single_surfel_plain_closed_form():
    """K=0: C = alpha c, T_final = 1 - alpha (eq. composite with one surfel)."""
    cam = identity_camera(32, 32, 40.0)
    mu, sig, opac, col = [0.05, -0.03, 2.0], [0.2, 0.3], 0.8, [0.2, 0.5, 0.7]
    sc = scene_from([mu], [[1, 0, 0, 0]], [sig], [opac], [[1, 1]], [col])
    rng = np.random.default_rng(1)
    grid = random_grid(rng)
    mlp = random_mlp(rng, [4, 8, 8, 3])
    out = oracle.render(sc, cam, grid, mlp, K=0)
    a, _, _, _ = _single_surfel_expect(cam, mu, sig, opac)
    assert (a > 0).sum() > 50
    np.testing.assert_allclose(out.image, a[:, None] * np.array(col)[None], atol=1e-14)
    np.testing.assert_allclose(out.t_final, 1.0 - a, atol=1e-14)


def test_single_surfel_textured_closed_form():
    """K=1: C = alpha Tex(x*), W = alpha, D = t* = mu_z, N = 0 (eq. final).

    A constant grid makes every level's interpolated feature equal that
    constant (trilinear weights sum to one), so the texture is the MLP of
    Delta_l(t*) * constant_l, evaluated here with numpy.
    """
    cam = identity_camera(32, 32, 40.0)
    mu, sig, opac, col = [0.05, -0.03, 2.0], [0.2, 0.3], 0.8, [0.2, 0.5, 0.7]
    sc = scene_from([mu], [[1, 0, 0, 0]], [sig], [opac], [[1, 1]], [col])
    lvl = [[0.3, -0.2], [0.1, 0.4]]
    grid = constant_grid(lvl)
    rng = np.random.default_rng(2)
    mlp = random_mlp(rng, [4, 8, 8, 3])
    out = oracle.render(sc, cam, grid, mlp, K=1)
    a, _, _, _ = _single_surfel_expect(cam, mu, sig, opac)
    s = grid.level_scales.double().numpy()
    delta = 1.0 - np.exp(-((cam.fx / (s * mu[2])) ** 2) / (2.0 * math.pi))
    z = np.concatenate([delta[l] * np.array(lvl[l]) for l in range(2)])
    tex = _np_mlp(z[None], [w.numpy() for w in mlp.weights])[0]
    hit = a > 0
    np.testing.assert_allclose(out.image, a[:, None] * tex[None], atol=1e-13)
    np.testing.assert_allclose(out.weights[:, 0], a, atol=1e-14)
    np.testing.assert_allclose(out.depths[hit, 0], mu[2], rtol=1e-14)
    assert np.all(out.ids[hit, 0] == 0) and np.all(out.ids[~hit, 0] == -1)
    np.testing.assert_allclose(out.plain, 0.0, atol=1e-15)


def test_single_surfel_gradients_closed_form():
    """dC/dc = alpha and dC/do = G c for a lone surfel (K=0)."""
    cam = identity_camera(32, 32, 40.0)
    mu, sig, opac, col = [0.05, -0.03, 2.0], [0.2, 0.3], 0.8, [0.2, 0.5, 0.7]
    sc = scene_from([mu], [[1, 0, 0, 0]], [sig], [opac], [[1, 1]], [col])
    rng = np.random.default_rng(3)
    grid = random_grid(rng)
    mlp = random_mlp(rng, [4, 8, 8, 3])
    g = rng.standard_normal((32 * 32, 3))
    out = oracle.render_and_grad(sc, cam, grid, mlp, K=0, grad_image=g)
    a, G, _, _ = _single_surfel_expect(cam, mu, sig, opac)
    np.testing.assert_allclose(out.grads["colors"][0], (a[:, None] * g).sum(0), rtol=1e-12)
    np.testing.assert_allclose(out.grads["opacities"][0], (G * (g @ np.array(col))).sum(), rtol=1e-12)


def test_two_surfels_front_to_back():
    """w1 = alpha1, w2 = alpha2 (1 - alpha1); slots in compositing order."""
    cam = identity_camera(8, 8, 10.0)
    sc = scene_from([[0, 0, 2.0], [0, 0, 3.0]], [[1, 0, 0, 0]] * 2, [[1.0, 1.0], [1.5, 1.5]], [0.6, 0.7],
                    [[1, 1]] * 2, [[1, 0, 0], [0, 1, 0]])
    rng = np.random.default_rng(4)
    out0 = oracle.render(sc, cam, random_grid(rng), random_mlp(rng, [4, 8, 8, 3]), K=0)
    rng = np.random.default_rng(4)
    out2 = oracle.render(sc, cam, random_grid(rng), random_mlp(rng, [4, 8, 8, 3]), K=2)
    W, H = 8, 8
    py, px = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    dx = ((px + 0.5 - 4) / 10.0).reshape(-1)
    dy = ((py + 0.5 - 4) / 10.0).reshape(-1)
    a1 = 0.6 * np.exp(-0.5 * ((2 * dx) ** 2 + (2 * dy) ** 2))
    a2 = 0.7 * np.exp(-0.5 * ((3 * dx / 1.5) ** 2 + (3 * dy / 1.5) ** 2))
    np.testing.assert_allclose(out0.image[:, 0], a1, atol=1e-14)
    np.testing.assert_allclose(out0.image[:, 1], a2 * (1 - a1), atol=1e-14)
    np.testing.assert_allclose(out0.t_final, (1 - a1) * (1 - a2), atol=1e-14)
    np.testing.assert_allclose(out2.weights[:, 0], a1, atol=1e-14)
    np.testing.assert_allclose(out2.weights[:, 1], a2 * (1 - a1), atol=1e-14)
    assert np.all(out2.ids[:, 0] == 0) and np.all(out2.ids[:, 1] == 1)


def _on_axis_stack(cam, px, py, depths, opac, scale=0.3):
    """Facing surfels centred on the ray through the centre of pixel (px, py)."""
    dx = (px + 0.5 - cam.cx) / cam.fx
    dy = (py + 0.5 - cam.cy) / cam.fy
    n = len(depths)
    means = [[z * dx, z * dy, z] for z in depths]
    cols = [[0.1 * (i + 1), 1.0 - 0.1 * i, 0.5] for i in range(n)]
    return scene_from(means, [[1, 0, 0, 0]] * n, [[scale, scale]] * n, [opac] * n, [[1, 1]] * n, cols), cols


def test_stop_rule_stack_of_opaque_surfels():
    """Compositing stops before the surfel that would take T below 1e-4
    (eq. composite with the 3DGS termination; reading 3). Five facing surfels
    of alpha = 0.95 on one pixel's ray: T after three is 0.05^3 = 1.25e-4,
    the fourth would give 6.25e-6, so exactly three are composited and
    C = sum_{i<3} 0.95 * 0.05^i * c_i."""
    cam = identity_camera(9, 9, 10.0)
    sc, cols = _on_axis_stack(cam, 4, 4, [2.0, 2.5, 3.0, 3.5, 4.0], 0.95)
    rng = np.random.default_rng(30)
    out = oracle.render(sc, cam, random_grid(rng), random_mlp(rng, [4, 8, 8, 3]), K=0)
    p = 4 * 9 + 4
    assert out.n_comp[p] == 3
    t = [1.0, 1.0 - 0.95, (1.0 - 0.95) ** 2, (1.0 - 0.95) ** 3]
    np.testing.assert_allclose(out.t_final[p], t[3], rtol=1e-13)
    assert out.t_final[p] > 1e-4 > out.t_final[p] * (1.0 - 0.95)
    expect = sum(0.95 * t[i] * np.array(cols[i]) for i in range(3))
    np.testing.assert_allclose(out.image[p], expect, rtol=1e-13)
    # K = 4 sees the same three: the top-K slots hold them and a fourth slot stays empty
    out4 = oracle.render(sc, cam, random_grid(rng), random_mlp(rng, [4, 8, 8, 3]), K=4)
    assert list(out4.ids[p]) == [0, 1, 2, -1]
    np.testing.assert_allclose(out4.weights[p, :3], [0.95 * t[i] for i in range(3)], rtol=1e-13)


def test_alpha_clamp_at_full_opacity():
    """alpha = min(0.99, o G) (reading 3): an opacity-1 surfel seen through its
    centre has G = 1, so alpha = 0.99 and T_final = 0.01; away from the centre
    the kernel is below the clamp and alpha = G."""
    cam = identity_camera(9, 9, 10.0)
    sc, cols = _on_axis_stack(cam, 4, 4, [2.0], 1.0, scale=0.2)
    rng = np.random.default_rng(31)
    out = oracle.render(sc, cam, random_grid(rng), random_mlp(rng, [4, 8, 8, 3]), K=0)
    p = 4 * 9 + 4
    np.testing.assert_allclose(out.t_final[p], 0.01, rtol=1e-13)
    np.testing.assert_allclose(out.image[p], 0.99 * np.array(cols[0]), rtol=1e-13)
    # one pixel to the right: u = 2 * 0.1 / 0.2 = 1, G = exp(-1/2) < 0.99
    np.testing.assert_allclose(out.t_final[p + 1], 1.0 - math.exp(-0.5), rtol=1e-13)


def _rodrigues(axis, angle):
    """Rotation matrix of `angle` about the unit `axis`: cos I + sin [a]x + (1 - cos) a a^T."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K_ = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return math.cos(angle) * np.eye(3) + math.sin(angle) * K_ + (1.0 - math.cos(angle)) * np.outer(a, a)


def _axis_angle_quat(axis, angle):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    return np.concatenate([[math.cos(angle / 2.0)], math.sin(angle / 2.0) * a])


def _quat_mul(p, q):
    """Hamilton product p q of (w, x, y, z) quaternions (rotation by q, then p)."""
    w1, x1, y1, z1 = p
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_quaternion_columns_are_rodrigues_axes():
    """R = [v1 v2 v3] (Representation, Geometry) is the rotation the quaternion
    stands for: its columns equal Rodrigues' matrix of the same axis and angle,
    in both the rendering and the binning code."""
    from oracle.binning import quat_columns_f64
    from oracle.geometry import quat_columns
    rng = np.random.default_rng(32)
    for _ in range(20):
        axis = rng.standard_normal(3)
        angle = rng.uniform(0.2, 3.0)
        R = _rodrigues(axis, angle)
        q = _axis_angle_quat(axis, angle)
        v = quat_columns(torch.from_numpy(q))
        np.testing.assert_allclose(np.stack([c.numpy() for c in v], axis=1), R, atol=1e-14)
        vb = quat_columns_f64(q[None])
        np.testing.assert_allclose(np.stack([c[0] for c in vb], axis=1), R, atol=1e-14)


def test_quarter_turn_swaps_the_surfel_axes():
    """A +90 degree turn about the normal maps v1 to the camera's y axis: with
    scales (s1, s2) it renders and bins like the unrotated surfel with
    (s2, s1); on the tilted plane u and v follow the closed form
    u = ((X - mu) . v1) / s1 with the hit point X of the ray-plane
    intersection and v1, v2 from Rodrigues' formula."""
    cam = identity_camera(24, 24, 30.0)
    mu = [0.02, -0.01, 2.0]
    qz = _axis_angle_quat([0, 0, 1], math.pi / 2)
    a = scene_from([mu], [qz], [[0.3, 0.12]], [0.8], [[1, 1]], [[0.2, 0.4, 0.6]])
    b = scene_from([mu], [[1, 0, 0, 0]], [[0.12, 0.3]], [0.8], [[1, 1]], [[0.2, 0.4, 0.6]])
    rng = np.random.default_rng(33)
    grid, mlp = random_grid(rng), random_mlp(rng, [4, 8, 8, 3])
    oa, ob = oracle.render(a, cam, grid, mlp, K=0), oracle.render(b, cam, grid, mlp, K=0)
    np.testing.assert_allclose(oa.image, ob.image, atol=1e-14)
    ba, bb = bin_surfels(a, cam), bin_surfels(b, cam)
    np.testing.assert_array_equal(ba["rect"], bb["rect"])
    # tilted about the x axis by 35 degrees, then turned by 70 degrees about the new normal
    q = _quat_mul(_axis_angle_quat([1, 0, 0], math.radians(35.0)), _axis_angle_quat([0, 0, 1], math.radians(70.0)))
    R = _rodrigues([1, 0, 0], math.radians(35.0)) @ _rodrigues([0, 0, 1], math.radians(70.0))
    sig = [0.4, 0.25]
    c = scene_from([mu], [q], [sig], [0.9], [[1, 1]], [[1.0, 1.0, 1.0]])
    oc = oracle.render(c, cam, grid, mlp, K=1)
    py, px = np.meshgrid(np.arange(24), np.arange(24), indexing="ij")
    d = np.stack([(px + 0.5 - 12) / 30.0, (py + 0.5 - 12) / 30.0, np.ones_like(px, dtype=float)], -1).reshape(-1, 3)
    t = (np.asarray(mu) @ R[:, 2]) / (d @ R[:, 2])
    X = t[:, None] * d - np.asarray(mu)[None]
    u = X @ R[:, 0] / sig[0]
    v = X @ R[:, 1] / sig[1]
    alpha = 0.9 * np.exp(-0.5 * (u * u + v * v))
    inside = (np.abs(u) <= 3) & (np.abs(v) <= 3) & (alpha >= ALPHA_MIN)
    assert inside.sum() > 100
    np.testing.assert_allclose(oc.t_final, np.where(inside, 1.0 - alpha, 1.0), atol=1e-13)
    np.testing.assert_allclose(oc.depths[inside, 0], t[inside], rtol=1e-13)


def test_camera_looks_along_its_axis():
    """Pinhole rays (reading 7): the ray through the principal point of a
    look-at camera starts at the eye and points at the target, and the target
    projects to the principal point."""
    from oracle.binning import to_camera_f64
    from oracle.geometry import camera_origin_and_rays
    eye, target = np.array([0.7, -1.2, 2.5]), np.array([-0.3, 0.4, -0.8])
    cam = scenes.look_at(eye, target, (0.0, -1.0, 0.0), 33, 21)
    o, d = camera_origin_and_rays(cam, np.array([16]), np.array([10]))
    np.testing.assert_allclose(o.numpy(), eye, atol=1e-14)
    dirn = (target - eye) / np.linalg.norm(target - eye)
    dd = d.numpy()[0]
    np.testing.assert_allclose(dd / np.linalg.norm(dd), dirn, atol=1e-14)
    assert abs(dd @ (target - eye) / np.linalg.norm(target - eye) - 1.0) < 1e-14  # unit camera-z component
    pc = to_camera_f64(np.asarray(cam.world_to_cam), target[None])[0]
    np.testing.assert_allclose([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy], [16.5, 10.5],
                               atol=1e-12)


def test_rigid_motion_of_scene_and_camera_changes_nothing():
    """Moving the surfels and the camera by one rigid motion (x -> Q x + b,
    q -> q_Q q, camera [R | t] -> [R Q^T | t - R Q^T b]) leaves every
    camera-frame quantity unchanged, so the collection pass (ids, W, D,
    T_final, N) and the K = 0 image are identical up to rounding."""
    wl = scenes.make_workload(1, seed=3, width=40, height=32, n_surfels=400)
    cam = scenes.look_at((0.4, -0.5, -2.8), (0.1, 0.0, 0.2), (0.0, -1.0, 0.0), 40, 32)
    rng = np.random.default_rng(34)
    axis, angle, b = rng.standard_normal(3), 1.1, np.array([0.7, -2.0, 1.3])
    Q = _rodrigues(axis, angle)
    qQ = _axis_angle_quat(axis, angle)
    sc = wl.scene
    mu = sc.means.double().numpy()
    quats = sc.quats.double().numpy()
    # unit to double precision: the textbook matrix is a rotation (and composes) only for |q| = 1
    quats = quats / np.linalg.norm(quats, axis=1, keepdims=True)
    moved = scenes.Scene(torch.from_numpy(mu @ Q.T + b), torch.from_numpy(np.stack([_quat_mul(qQ, q) for q in quats])),
                         sc.scales.double(), sc.opacities.double(), sc.gammas.double(), sc.colors.double())
    m = np.asarray(cam.world_to_cam)
    Rn = m[:, :3] @ Q.T
    cam2 = scenes.Camera(np.concatenate([Rn, (m[:, 3] - Rn @ b)[:, None]], axis=1), cam.fx, cam.fy, cam.cx, cam.cy,
                         cam.width, cam.height)
    base = scenes.Scene(sc.means.double(), torch.from_numpy(quats), *[t.double() for t in sc.tensors()[2:]])
    for K in (0, 4):
        a = oracle.render(base, cam, wl.grid, wl.mlp, K)
        c = oracle.render(moved, cam2, wl.grid, wl.mlp, K)
        assert (a.n_comp > 0).mean() > 0.3
        np.testing.assert_array_equal(a.ids, c.ids)
        np.testing.assert_array_equal(a.n_comp, c.n_comp)
        for nm in ("weights", "t_final", "plain"):
            np.testing.assert_allclose(getattr(a, nm), getattr(c, nm), atol=1e-11)
        np.testing.assert_allclose(a.depths, c.depths, rtol=1e-11, atol=1e-11)
        if K == 0:
            np.testing.assert_allclose(a.image, c.image, atol=1e-11)


def test_blended_error_closed_forms():
    """Blended errors (supplementary, Densification): per surfel the sum over
    pixels of its blending weight times the pixel's error. For two facing
    surfels w1 = alpha1 and w2 = alpha2 (1 - alpha1) per pixel; with a unit
    error everywhere the surfels' errors and the pixels' final transmittance
    add up to the number of pixels (sum_i w_i + T_final = 1)."""
    cam = identity_camera(8, 8, 10.0)
    sc = scene_from([[0, 0, 2.0], [0, 0, 3.0]], [[1, 0, 0, 0]] * 2, [[1.0, 1.0], [1.5, 1.5]], [0.6, 0.7],
                    [[1, 1]] * 2, [[1, 0, 0], [0, 1, 0]])
    rng = np.random.default_rng(35)
    E = rng.uniform(0.0, 2.0, 64)
    out = oracle.render(sc, cam, random_grid(rng), random_mlp(rng, [4, 8, 8, 3]), K=1, pixel_error=E)
    py, px = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    dx = ((px + 0.5 - 4) / 10.0).reshape(-1)
    dy = ((py + 0.5 - 4) / 10.0).reshape(-1)
    a1 = 0.6 * np.exp(-0.5 * ((2 * dx) ** 2 + (2 * dy) ** 2))
    a2 = 0.7 * np.exp(-0.5 * ((3 * dx / 1.5) ** 2 + (3 * dy / 1.5) ** 2))
    np.testing.assert_allclose(out.blended_error, [(a1 * E).sum(), (a2 * (1 - a1) * E).sum()], rtol=1e-13)
    wl = scenes.make_workload(1, seed=4, width=40, height=30)
    ones = oracle.render(wl.scene, wl.cameras[0], wl.grid, wl.mlp, 4, pixel_error=np.ones(1200))
    assert (ones.blended_error > 0).sum() > 50
    np.testing.assert_allclose(ones.blended_error.sum() + ones.t_final.sum(), 1200.0, rtol=1e-12)


# ---------------------------------------------------------------- kernel limits

def test_kernel_gamma_one_is_gaussian():
    """gamma = 1 gives the 2DGS Gaussian exp(-(u^2 + v^2)/2) (Geometry)."""
    u = torch.linspace(-3, 3, 61, dtype=torch.float64)
    v = torch.linspace(-2, 2, 61, dtype=torch.float64)
    G = kernel(u, v, torch.ones(61, 2, dtype=torch.float64))
    np.testing.assert_allclose(G.numpy(), np.exp(-0.5 * (u.numpy() ** 2 + v.numpy() ** 2)), rtol=1e-14)


def test_kernel_large_gamma_is_quad_indicator():
    """gamma -> infinity approaches the indicator of the unit quad (Geometry)."""
    u = torch.tensor([0.0, 0.5, 0.9, 1.1, 2.0], dtype=torch.float64)
    v = torch.tensor([0.0, 0.2, 0.85, 0.3, 0.1], dtype=torch.float64)
    G = kernel(u, v, torch.full((5, 2), 50.0, dtype=torch.float64)).numpy()
    np.testing.assert_allclose(G[:3], 1.0, atol=2e-3)
    np.testing.assert_allclose(G[3:], 0.0, atol=1e-300)


# ---------------------------------------------------------------- invariants on a scene

@pytest.fixture(scope="module")
def c1_small():
    wl = scenes.make_workload(1, seed=0, width=64, height=48)
    return wl


def test_weights_plus_transmittance_is_one(c1_small):
    """sum_i w_i + T_final = 1 (eq. composite, telescoping product)."""
    wl = c1_small
    sc = scenes.Scene(*[t.clone() for t in wl.scene.tensors()])
    sc.colors = torch.ones_like(sc.colors)
    out = oracle.render(sc, wl.cameras[0], wl.grid, wl.mlp, K=4)
    total = out.weights.sum(1) + out.plain[:, 0] + out.t_final
    np.testing.assert_allclose(total, 1.0, atol=1e-12)
    assert out.weights.min() >= 0 and out.weights.max() <= 1
    assert out.t_final.min() >= 0 and out.t_final.max() <= 1


def test_final_versus_notexture(c1_small):
    """C(K=0) = N(K) + sum_j W_j c_{I_j} (eq. notexture against eq. composite)."""
    wl = c1_small
    cam = wl.cameras[0]
    out0 = oracle.render(wl.scene, cam, wl.grid, wl.mlp, K=0)
    out4 = oracle.render(wl.scene, cam, wl.grid, wl.mlp, K=4)
    col = wl.scene.colors.double().numpy()
    sel = np.where(out4.ids[..., None] >= 0, col[np.maximum(out4.ids, 0)], 0.0)
    recon = out4.plain + (out4.weights[..., None] * sel).sum(1)
    np.testing.assert_allclose(recon, out0.image, atol=1e-13)
    np.testing.assert_allclose(out0.t_final, out4.t_final, atol=0)


def test_topk_is_prefix_of_full_sort(c1_small):
    """The K slots are the K largest weights under (w desc, id asc) (Collection Pass)."""
    wl = c1_small
    cam = wl.cameras[0]
    full = oracle.render(wl.scene, cam, wl.grid, wl.mlp, K=64)
    assert full.n_comp.max() < 64
    np.testing.assert_allclose(full.plain, 0.0, atol=1e-15)  # everything selected: N = 0
    out = oracle.render(wl.scene, cam, wl.grid, wl.mlp, K=4)
    for p in range(full.pixels.shape[0]):
        entries = [(full.weights[p, j], full.ids[p, j], j) for j in range(64) if full.ids[p, j] >= 0]
        best = sorted(entries, key=lambda e: (-e[0], e[1]))[:4]
        best = sorted(best, key=lambda e: e[2])  # compositing order
        ids = [e[1] for e in best] + [-1] * (4 - len(best))
        assert list(out.ids[p]) == ids


def test_tiled_equals_untiled(c1_small):
    """Binning is conservative: restricting candidates to tile lists changes nothing."""
    wl = c1_small
    cam = wl.cameras[0]
    a = oracle.render(wl.scene, cam, wl.grid, wl.mlp, K=4)
    b = oracle.render(wl.scene, cam, wl.grid, wl.mlp, K=4, tiled=True)
    np.testing.assert_array_equal(a.ids, b.ids)
    np.testing.assert_allclose(a.image, b.image, atol=1e-13)
    np.testing.assert_allclose(a.t_final, b.t_final, atol=1e-13)


def test_tiled_equals_untiled_near_plane_crossing():
    """Camera inside the cloud: many surfels cross the near plane and get clipped."""
    wl = scenes.make_workload(1, seed=5, width=48, height=48, n_surfels=3000)
    cam = scenes.look_at((0.0, 0.0, -0.3), (0.0, 0.0, 1.0), (0.0, -1.0, 0.0), 48, 48)
    info = bin_surfels(wl.scene, cam)
    a = oracle.render(wl.scene, cam, wl.grid, wl.mlp, K=4, bins=info)
    b = oracle.render(wl.scene, cam, wl.grid, wl.mlp, K=4, tiled=True, bins=info)
    assert (a.n_comp > 0).mean() > 0.5
    np.testing.assert_array_equal(a.ids, b.ids)
    np.testing.assert_allclose(a.image, b.image, atol=1e-13)


def test_binning_matches_brute_force_lists(c1_small):
    """Each tile's list is exactly the surfels whose rectangle covers it, by (key, id)."""
    wl = c1_small
    info = bin_surfels(wl.scene, wl.cameras[0])
    rect, count, key = info["rect"], info["count"], info["key"]
    for t in range(info["ntx"] * info["nty"]):
        tx, ty = t % info["ntx"], t // info["ntx"]
        members = [i for i in range(rect.shape[0]) if count[i] > 0 and rect[i, 0] <= tx <= rect[i, 2]
                   and rect[i, 1] <= ty <= rect[i, 3]]
        members.sort(key=lambda i: (float(key[i]), i))
        s, e = info["ranges"][t]
        assert list(info["ids"][s:e]) == members


# ---------------------------------------------------------------- hash grid

def test_map_positive_is_bijection():
    """MapPositive maps Z one-to-one onto N (supplementary, Architecture)."""
    z = np.arange(-10**6, 10**6 + 1)
    m = map_positive(z)
    assert m.min() == 0 and m.max() == 2 * 10**6
    assert np.unique(m).shape[0] == z.shape[0]
    assert list(map_positive(np.array([0, 1, -1, 2, -2]))) == [0, 1, 2, 3, 4]


def test_spatial_hash_matches_big_integer_arithmetic():
    rng = np.random.default_rng(7)
    k = rng.integers(0, 2**31, (1000, 3))
    got = spatial_hash(k[:, 0], k[:, 1], k[:, 2], 19)
    for i in range(1000):
        h = ((int(k[i, 0]) * PRIMES[0]) ^ (int(k[i, 1]) * PRIMES[1]) ^ (int(k[i, 2]) * PRIMES[2])) % (1 << 32)
        assert got[i] == h & ((1 << 19) - 1)


def test_constant_table_partition_of_unity():
    """Trilinear weights sum to one: a constant table yields Delta * constant."""
    grid = constant_grid([[0.25, -0.5], [1.5, 0.125]])
    rng = np.random.default_rng(8)
    x = torch.from_numpy(rng.uniform(-30, 30, (500, 3)))
    D = torch.from_numpy(rng.uniform(0.3, 40, 500))
    z = encode(x, D, grid.table.double(), grid.level_scales.double(), 500.0).numpy()
    for l, vals in enumerate([[0.25, -0.5], [1.5, 0.125]]):
        dl = downweight(D, float(grid.level_scales[l]), 500.0).numpy()
        np.testing.assert_allclose(z[:, 2 * l:2 * l + 2], dl[:, None] * np.array(vals)[None], rtol=1e-13)


def test_lattice_points_read_single_entry():
    """At a lattice point the interpolation returns the entry of that corner."""
    rng = np.random.default_rng(9)
    grid = random_grid(rng, levels=1, log2_size=10)
    s = float(grid.level_scales[0])
    k = rng.integers(-5000, 5000, (200, 3))
    x = torch.from_numpy(k / s)
    D = torch.full((200,), 1e-6, dtype=torch.float64)  # Delta = 1 to double precision
    z = encode(x, D, grid.table.double(), grid.level_scales.double(), 1.0).numpy()
    mp = map_positive(k)
    h = spatial_hash(mp[:, 0], mp[:, 1], mp[:, 2], 10)
    np.testing.assert_array_equal(z, grid.table.numpy()[0, h])


def test_interpolation_is_linear_inside_a_cell():
    rng = np.random.default_rng(10)
    grid = random_grid(rng, levels=1, log2_size=8)
    s = float(grid.level_scales[0])
    base = np.array([[3.25, -7.5, 11.75]]) / s
    e = np.array([[1.0, 0.0, 0.0]]) / s
    pts = torch.from_numpy(np.concatenate([base, base + 0.25 * e, base + 0.5 * e]))
    D = torch.full((3,), 1e-6, dtype=torch.float64)
    z = encode(pts, D, grid.table.double(), grid.level_scales.double(), 1.0).numpy()
    np.testing.assert_allclose(z[1], 0.5 * (z[0] + z[2]), rtol=1e-13)


def test_forced_cells_match_natural_cells_and_faces_are_continuous():
    """Forcing the natural lattice cell changes nothing; at a cell face the
    two neighbouring cells' trilinear polynomials agree (continuity), which
    is what makes evaluating a sample in another implementation's cell a
    rounding-sized change of the value."""
    rng = np.random.default_rng(12)
    grid = random_grid(rng, levels=2, log2_size=8)
    s = grid.level_scales.double().numpy()
    x = torch.from_numpy(rng.uniform(-3, 3, (50, 3)))
    D = torch.from_numpy(rng.uniform(0.5, 5, 50))
    cells = np.stack([np.floor(s[l] * x.numpy()) for l in range(2)], axis=1).astype(np.int64)
    a = encode(x, D, grid.table.double(), grid.level_scales.double(), 100.0).numpy()
    b = encode(x, D, grid.table.double(), grid.level_scales.double(), 100.0, cells=cells).numpy()
    np.testing.assert_array_equal(a, b)
    # points exactly on an x-face of level 0: cell k and cell k-1 give the same features
    k = rng.integers(-50, 50, (20, 3)).astype(np.float64)
    frac = rng.uniform(0.1, 0.9, (20, 3))
    frac[:, 0] = 0.0
    xf = torch.from_numpy((k + frac) / s[0])
    Df = torch.full((20,), 1.0, dtype=torch.float64)
    c_hi = np.stack([np.floor(s[l] * xf.numpy()) for l in range(2)], axis=1).astype(np.int64)
    c_lo = c_hi.copy()
    c_lo[:, 0, 0] -= 1
    za = encode(xf, Df, grid.table.double(), grid.level_scales.double(), 100.0, cells=c_hi).numpy()
    zb = encode(xf, Df, grid.table.double(), grid.level_scales.double(), 100.0, cells=c_lo).numpy()
    np.testing.assert_allclose(za[:, :2], zb[:, :2], rtol=1e-12, atol=1e-15)


def test_downweight_matches_erf_squared_and_limits():
    """Delta approximates erf(f / (2 sqrt2 s t))^2 (supplementary, Anti-aliasing)."""
    f = 1662.77
    s = torch.tensor(16.0 * 1.5 ** np.arange(16), dtype=torch.float64)
    t = torch.logspace(-2, 3, 400, dtype=torch.float64)
    D = downweight(t[:, None], s[None, :], f).numpy()
    ref = erf(f / (2 * np.sqrt(2) * s.numpy()[None] * t.numpy()[:, None])) ** 2
    assert np.max(np.abs(D - ref)) <= 0.0116
    assert np.all(np.diff(D, axis=0) <= 0) and np.all(np.diff(D, axis=1) <= 0)  # decreasing in t and s
    assert downweight(torch.tensor(1e-9, dtype=torch.float64), 7000.0, f).item() == 1.0
    assert downweight(torch.tensor(1e9, dtype=torch.float64), 16.0, f).item() < 1e-12


def test_forced_relu_masks():
    """Natural masks reproduce the ReLU network; a flipped unit with a zero
    pre-activation leaves the output unchanged (continuity at the kink)."""
    from oracle.mlp import unpack_masks
    rng = np.random.default_rng(13)
    mlp = random_mlp(rng, [32, 64, 64, 3])
    z = torch.from_numpy(rng.standard_normal((20, 32)))
    h1 = z @ mlp.weights[0].t()
    h2 = torch.relu(h1) @ mlp.weights[1].t()
    def pack(b):
        b = b.numpy().astype(np.uint64).reshape(20, 2, 32)
        return (b << np.arange(32, dtype=np.uint64)).sum(-1).astype(np.uint32)
    words = np.concatenate([pack(h1 > 0), pack(h2 > 0)], axis=1)
    masks = unpack_masks(words, 64, 2)
    np.testing.assert_array_equal(masks[0].numpy(), (h1 > 0).numpy().astype(float))
    a = mlp_forward(z, mlp.weights).numpy()
    b = mlp_forward(z, mlp.weights, relu_masks=masks).numpy()
    np.testing.assert_allclose(a, b, rtol=1e-14)


def test_mlp_matches_numpy_chain_and_zero_input():
    rng = np.random.default_rng(11)
    mlp = random_mlp(rng, [32, 64, 64, 3])
    z = rng.standard_normal((100, 32))
    got = mlp_forward(torch.from_numpy(z), mlp.weights).numpy()
    np.testing.assert_allclose(got, _np_mlp(z, [w.numpy() for w in mlp.weights]), rtol=1e-12)
    # bias-free: G(0) is the head's activation at zero
    z0 = mlp_forward(torch.zeros(1, 32, dtype=torch.float64), mlp.weights).numpy()
    np.testing.assert_allclose(z0, 0.5)


# ---------------------------------------------------------------- finite differences

def _fd_setup(seed, gamma_range=None):
    rng = np.random.default_rng(seed)
    cam = identity_camera(32, 32, 40.0)
    sc = facing_scene(rng, 14, tilt=0.35)
    if gamma_range is not None:
        sc.gammas = torch.from_numpy(rng.uniform(*gamma_range, (14, 2)))
    grid = random_grid(rng, levels=2, log2_size=8, scale=0.5)
    mlp = random_mlp(rng, [4, 16, 16, 3])
    gi = rng.standard_normal((32 * 32, 3))
    gw = rng.standard_normal((32 * 32, 2))
    gt = rng.standard_normal((32 * 32, 2, 3))
    return rng, cam, sc, grid, mlp, gi, gw, gt


def _loss(out, gi, gw, gt):
    return float((out.image * gi).sum() + (out.weights * gw).sum() + (out.tex * gt).sum())


@pytest.mark.parametrize("seed,gamma_range", [(20, None), (21, (1.0, 4.0))])
def test_gradients_match_central_differences(seed, gamma_range):
    """Autograd gradients of the oracle equal central differences of its forward."""
    rng, cam, sc, grid, mlp, gi, gw, gt = _fd_setup(seed, gamma_range)
    K = 2
    out = oracle.render_and_grad(sc, cam, grid, mlp, K, grad_image=gi, grad_weights=gw, grad_tex=gt)
    assert (out.n_comp > 0).mean() > 0.4
    h = 1e-8  # small enough that no hash-cell face or ReLU kink is crossed

    def run(scn, grd, mp):
        return oracle.render(scn, cam, grd, mp, K)

    names = ["means", "quats", "scales", "opacities", "gammas", "colors"]
    for nm in names + ["table", "mlp0", "mlp1", "mlp2"]:
        for trial in range(2):
            if nm in names:
                base = getattr(sc, nm)
                vdir = torch.from_numpy(rng.standard_normal(tuple(base.shape)))
                g = out.grads[nm]

                def make(sign):
                    s2 = scenes.Scene(*[t.clone() for t in sc.tensors()])
                    setattr(s2, nm, base + sign * h * vdir)
                    return run(s2, grid, mlp)
            elif nm == "table":
                base = grid.table
                vdir = torch.from_numpy(rng.standard_normal(tuple(base.shape)))
                g = out.grads["table"]

                def make(sign):
                    return run(sc, scenes.HashGrid(base + sign * h * vdir, grid.level_scales), mlp)
            else:
                li = int(nm[-1])
                base = mlp.weights[li]
                vdir = torch.from_numpy(rng.standard_normal(tuple(base.shape)))
                g = out.grads["mlp"][li]

                def make(sign):
                    ws = list(mlp.weights)
                    ws[li] = base + sign * h * vdir
                    return run(sc, grid, scenes.MLP(ws))
            op, om = make(+1), make(-1)
            assert np.array_equal(op.ids, out.ids) and np.array_equal(om.ids, out.ids), nm
            assert np.array_equal(op.n_comp, out.n_comp) and np.array_equal(om.n_comp, out.n_comp), nm
            fd = (_loss(op, gi, gw, gt) - _loss(om, gi, gw, gt)) / (2 * h)
            an = float((np.asarray(g) * vdir.numpy()).sum())
            assert abs(fd - an) <= 2e-6 * max(1.0, abs(an)), (nm, fd, an)


# ---------------------------------------------------------------- parameter layout

def test_storage_count_matches_paper_figures():
    """Two bytes per Instant-NGP parameter, four per other parameter
    (supplementary, Other details) reproduce the printed 160/100/90 MB.
    60 floats per surfel: mean 3, quaternion 4, scale 2, opacity 1, gamma 2, SH 48."""
    g = json.load(open(os.path.join(HERE, "golden", "paper_storage.json")))
    n = g["n_primitives"]
    per_surfel = 3 + 4 + 2 + 1 + 2 + g["sh_values_per_primitive"]
    dims = g["mlp_dims"]
    ngp = g["levels"] * (1 << g["log2_table"]) * g["feat"] + sum(dims[i] * dims[i + 1] for i in range(3))
    full = (n * per_surfel * 4 + ngp * 2) / 1e6
    no_tex = n * per_surfel * 4 / 1e6
    no_sh = (n * (per_surfel - 45) * 4 + ngp * 2) / 1e6
    tol = g["printed_rounding_mb"]
    assert abs(full - g["printed_mb"]["full"]) <= tol
    assert abs(no_tex - g["printed_mb"]["no_texture"]) <= tol
    assert abs(no_sh - g["printed_mb"]["no_prim_sh"]) <= tol
