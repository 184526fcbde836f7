"""Pins of the oracle's spherical-harmonics colour (CPU).

Representation, Appearance (degree-3 SH, 16 coefficients per channel).
  * Orthonormality: a product Gauss-Legendre x uniform-azimuth quadrature,
    exact for polynomials of this degree, gives the integral of Y_i Y_j over
    the sphere = delta_ij (fixes every constant).
  * Addition theorem: sum over m of Y_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a.b)
    for each degree l (fixes each degree's functions up to a rotation of
    the basis, whatever the sign convention).
  * Colour: zero coefficients give grey 0.5; the DC coefficient alone gives
    C0 a + 0.5 in every direction; negative results clamp to 0.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle.sh import C0, basis, colour


def _sphere_quadrature(n_theta=12, n_phi=24):
    x, w = np.polynomial.legendre.leggauss(n_theta)  # nodes in cos(theta)
    phi = (np.arange(n_phi) + 0.5) * 2 * np.pi / n_phi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wt = (w[:, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, :]).reshape(-1)
    return torch.tensor(d), torch.tensor(wt)


def test_orthonormal_over_the_sphere():
    d, w = _sphere_quadrature()
    Y = basis(d)
    gram = (Y * w[:, None]).T @ Y
    assert torch.allclose(gram, torch.eye(16, dtype=torch.float64), atol=1e-12)


def test_addition_theorem_per_degree():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(50, 3))
    b = rng.normal(size=(50, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya, Yb = basis(torch.tensor(a)), basis(torch.tensor(b))
    c = (a * b).sum(1)
    legendre = [np.ones_like(c), c, 0.5 * (3 * c ** 2 - 1), 0.5 * (5 * c ** 3 - 3 * c)]
    for l in range(4):
        sl = slice(l * l, (l + 1) ** 2)
        lhs = (Ya[:, sl] * Yb[:, sl]).sum(1).numpy()
        rhs = (2 * l + 1) / (4 * math.pi) * legendre[l]
        assert np.allclose(lhs, rhs, atol=1e-13), l


def test_colour_special_cases():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(20, 3))
    d = torch.tensor(d / np.linalg.norm(d, axis=1, keepdims=True))
    assert torch.all(colour(torch.zeros(20, 48, dtype=torch.float64), d) == 0.5)
    a = torch.zeros(20, 48, dtype=torch.float64)
    a[:, 0:3] = torch.tensor([0.3, -0.2, -5.0], dtype=torch.float64)
    col = colour(a, d)
    assert torch.allclose(col[:, 0], torch.full((20,), C0 * 0.3 + 0.5, dtype=torch.float64))
    assert torch.allclose(col[:, 1], torch.full((20,), C0 * -0.2 + 0.5, dtype=torch.float64))
    assert torch.all(col[:, 2] == 0.0)


# ---------------------------------------------------------------- the renderer's SH mode

from tests.oracle_cases import constant_grid, facing_scene, identity_camera, random_grid, random_mlp, scene_from  # noqa: E402
from tests.test_oracle_pins import _single_surfel_expect  # noqa: E402

import oracle  # noqa: E402
import scenes  # noqa: E402


def test_single_surfel_sh_colour_closed_form():
    """K=0: C = alpha colour(a, mu / |mu|) (identity camera at the origin)."""
    cam = identity_camera(32, 32, 40.0)
    mu, sig, opac = [0.05, -0.03, 2.0], [0.2, 0.3], 0.8
    rng = np.random.default_rng(4)
    a = rng.normal(scale=0.3, size=48)
    sc = scene_from([mu], [[1, 0, 0, 0]], [sig], [opac], [[1, 1]], [a])
    out = oracle.render(sc, cam, random_grid(rng), random_mlp(rng, [4, 8, 8, 48]), K=0, sh_degree=3)
    al, _, _, _ = _single_surfel_expect(cam, mu, sig, opac)
    m = torch.tensor(mu, dtype=torch.float64)
    c = colour(torch.tensor(a)[None], (m / m.norm())[None])[0].numpy()
    assert (al > 0).sum() > 50
    np.testing.assert_allclose(out.image, al[:, None] * c[None], atol=1e-14)


def test_single_surfel_sh_texture_closed_form():
    """K=1: Tex = colour(G(Delta const), unit ray) with a linear 48-value head (numpy)."""
    cam = identity_camera(32, 32, 40.0)
    mu, sig, opac = [0.05, -0.03, 2.0], [0.2, 0.3], 0.8
    sc = scene_from([mu], [[1, 0, 0, 0]], [sig], [opac], [[1, 1]], [np.zeros(48)])
    lvl = [[0.3, -0.2], [0.1, 0.4]]
    grid = constant_grid(lvl)
    rng = np.random.default_rng(5)
    mlp = random_mlp(rng, [4, 8, 8, 48])
    out = oracle.render(sc, cam, grid, mlp, K=1, sh_degree=3)
    al, _, dx, dy = _single_surfel_expect(cam, mu, sig, opac)
    s = grid.level_scales.double().numpy()
    delta = 1.0 - np.exp(-((cam.fx / (s * mu[2])) ** 2) / (2.0 * math.pi))
    z = np.concatenate([delta[l] * np.array(lvl[l]) for l in range(2)])
    h = z[None]
    ws = [w.numpy() for w in mlp.weights]
    for i, w in enumerate(ws):
        h = h @ w.T
        if i < len(ws) - 1:
            h = np.maximum(h, 0.0)
    ray = np.stack([dx, dy, np.ones_like(dx)], 1)
    ray /= np.linalg.norm(ray, axis=1, keepdims=True)
    tex = colour(torch.tensor(np.repeat(h, ray.shape[0], 0)), torch.tensor(ray)).numpy()
    np.testing.assert_allclose(out.image, al[:, None] * tex, atol=1e-13)


def test_sh_mode_gradients_match_central_differences():
    rng = np.random.default_rng(30)
    cam = identity_camera(32, 32, 40.0)
    sc = facing_scene(rng, 12, tilt=0.35)
    sc.colors = torch.from_numpy(rng.normal(scale=0.3, size=(12, 48)))
    grid = random_grid(rng, levels=2, log2_size=8, scale=0.5)
    mlp = random_mlp(rng, [4, 16, 16, 48])
    gi = rng.standard_normal((32 * 32, 3))
    gt = rng.standard_normal((32 * 32, 2, 3))
    K = 2
    out = oracle.render_and_grad(sc, cam, grid, mlp, K, grad_image=gi, grad_tex=gt, sh_degree=3)
    h = 1e-8

    def loss(o):
        return float((o.image * gi).sum() + (o.tex * gt).sum())

    for nm in ("colors", "means", "mlp2", "table"):
        if nm == "mlp2":
            base = mlp.weights[2]
            vdir = torch.from_numpy(rng.standard_normal(tuple(base.shape)))
            g = out.grads["mlp"][2]
            run = lambda sg: oracle.render(sc, cam, grid, scenes.MLP([mlp.weights[0], mlp.weights[1],
                                                                      base + sg * h * vdir]), K, sh_degree=3)
        elif nm == "table":
            base = grid.table
            vdir = torch.from_numpy(rng.standard_normal(tuple(base.shape)))
            g = out.grads["table"]
            run = lambda sg: oracle.render(sc, cam, scenes.HashGrid(base + sg * h * vdir, grid.level_scales), mlp, K,
                                           sh_degree=3)
        else:
            base = getattr(sc, nm)
            vdir = torch.from_numpy(rng.standard_normal(tuple(base.shape)))
            g = out.grads[nm]

            def run(sg, nm=nm, base=base, vdir=vdir):
                s2 = scenes.Scene(*[t.clone() for t in sc.tensors()])
                setattr(s2, nm, base + sg * h * vdir)
                return oracle.render(s2, cam, grid, mlp, K, sh_degree=3)
        fd = (loss(run(+1)) - loss(run(-1))) / (2 * h)
        an = float((np.asarray(g) * vdir.numpy()).sum())
        assert abs(fd - an) <= 2e-6 * max(1.0, abs(an)), (nm, fd, an)
