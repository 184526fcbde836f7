"""Seeded synthetic workloads for the surfel renderer.

This module only draws random numbers and builds pinhole cameras. It holds
none of the rendering arithmetic, so both the FP64 oracle and the HIP path
take their inputs from here without sharing any method code.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` and draws in the
order written below, so a (config, seed) pair always yields the same scene.

Parameter conventions (activated values, as the renderer consumes them):
  means   [N,3] float32   world-space centres
  quats   [N,4] float32   unit quaternions (w, x, y, z); R = [v1 v2 v3]
  scales  [N,2] float32   > 0, extent along v1 and v2
  opac    [N]   float32   in (0, 1)
  gammas  [N,2] float32   >= 1 (generalised-Gaussian exponents)
  colors  [N,3] float32   RGB
Cameras use the OpenCV convention (x right, y down, z forward) and carry a
world-to-camera matrix [R | t] in float64, focal lengths fx = fy and the
principal point at the image centre.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

__all__ = [
    "Camera",
    "Scene",
    "HashGrid",
    "MLP",
    "Workload",
    "look_at",
    "make_workload",
    "TrainWorkload",
    "make_train_workload",
    "CONFIG_NAMES",
]


@dataclasses.dataclass
class Camera:
    world_to_cam: np.ndarray  # [3,4] float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Scene:
    means: torch.Tensor
    quats: torch.Tensor
    scales: torch.Tensor
    opacities: torch.Tensor
    gammas: torch.Tensor
    colors: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def tensors(self):
        return (self.means, self.quats, self.scales, self.opacities, self.gammas, self.colors)


@dataclasses.dataclass
class HashGrid:
    table: torch.Tensor        # [L, T, F] in its storage dtype
    level_scales: torch.Tensor  # [L] float32

    @property
    def levels(self) -> int:
        return int(self.table.shape[0])

    @property
    def log2_size(self) -> int:
        return int(self.table.shape[1]).bit_length() - 1

    @property
    def feat(self) -> int:
        return int(self.table.shape[2])


@dataclasses.dataclass
class MLP:
    weights: list  # list of [out, in] tensors in their storage dtype (no biases)


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    cameras: list
    grid: HashGrid
    mlp: MLP
    K: int
    target: list  # per camera: [H, W, 3] float32 target image (or None)
    sh_degree: int = None  # 3: colours are [N,48] SH coefficients and the MLP head has 48 outputs


CONFIG_NAMES = {
    1: "c1_2k_128px_K4_fp32",
    2: "c2_100k_1024x768_K4_fp32",
    3: "c3_400k_1920x1080_K4",
    4: "c4_300k_16views_uneven",
    5: "c5_1M_2560x1440_K8_bf16",
}


def look_at(eye, target, up, width, height, fov_y_deg=None, fov_x_deg=60.0):
    """OpenCV pinhole camera at ``eye`` looking at ``target``.

    The focal length puts a field of view of ``fov_x_deg`` across the image
    width (fx = fy = (W/2)/tan(fov/2)); the principal point is the image centre.
    """
    eye = np.asarray(eye, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    up = np.asarray(up, dtype=np.float64)
    z = target - eye
    z = z / np.linalg.norm(z)
    y = -up + np.dot(up, z) * z
    y = y / np.linalg.norm(y)
    x = np.cross(y, z)
    c2w = np.stack([x, y, z], axis=1)  # columns are the camera axes in world
    r = c2w.T
    t = -r @ eye
    w2c = np.concatenate([r, t[:, None]], axis=1)
    half = math.radians(fov_x_deg) / 2.0
    f = (width / 2.0) / math.tan(half)
    return Camera(w2c, f, f, width / 2.0, height / 2.0, int(width), int(height))


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _rot_to_quat_fast(m):
    """Vectorised rotation-to-quaternion (branch by largest diagonal term)."""
    n = m.shape[0]
    q = np.zeros((n, 4))
    tr = m[:, 0, 0] + m[:, 1, 1] + m[:, 2, 2]
    d = np.stack([tr, m[:, 0, 0], m[:, 1, 1], m[:, 2, 2]], axis=1)
    case = np.argmax(d, axis=1)
    r = m
    for c in range(4):
        sel = case == c
        if not np.any(sel):
            continue
        rs = r[sel]
        if c == 0:
            s = np.sqrt(tr[sel] + 1.0) * 2
            q[sel] = np.stack([0.25 * s, (rs[:, 2, 1] - rs[:, 1, 2]) / s, (rs[:, 0, 2] - rs[:, 2, 0]) / s,
                               (rs[:, 1, 0] - rs[:, 0, 1]) / s], 1)
        elif c == 1:
            s = np.sqrt(1.0 + rs[:, 0, 0] - rs[:, 1, 1] - rs[:, 2, 2]) * 2
            q[sel] = np.stack([(rs[:, 2, 1] - rs[:, 1, 2]) / s, 0.25 * s, (rs[:, 0, 1] + rs[:, 1, 0]) / s,
                               (rs[:, 0, 2] + rs[:, 2, 0]) / s], 1)
        elif c == 2:
            s = np.sqrt(1.0 + rs[:, 1, 1] - rs[:, 0, 0] - rs[:, 2, 2]) * 2
            q[sel] = np.stack([(rs[:, 0, 2] - rs[:, 2, 0]) / s, (rs[:, 0, 1] + rs[:, 1, 0]) / s, 0.25 * s,
                               (rs[:, 1, 2] + rs[:, 2, 1]) / s], 1)
        else:
            s = np.sqrt(1.0 + rs[:, 2, 2] - rs[:, 0, 0] - rs[:, 1, 1]) * 2
            q[sel] = np.stack([(rs[:, 1, 0] - rs[:, 0, 1]) / s, (rs[:, 0, 2] + rs[:, 2, 0]) / s,
                               (rs[:, 1, 2] + rs[:, 2, 1]) / s, 0.25 * s], 1)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _plane_quats(rng, normals):
    """Quaternions with v3 = +-normal and a uniform in-plane angle."""
    n = normals.shape[0]
    flip = rng.random(n) < 0.5
    nrm = np.where(flip[:, None], -normals, normals)
    angle = rng.uniform(0.0, 2.0 * math.pi, n)
    nn = nrm / np.linalg.norm(nrm, axis=1, keepdims=True)
    helper = np.where(np.abs(nn[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    a = np.cross(nn, helper)
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = np.cross(nn, a)
    ca, sa = np.cos(angle)[:, None], np.sin(angle)[:, None]
    v1 = ca * a + sa * b
    v2 = np.cross(nn, v1)
    rot = np.stack([v1, v2, nn], axis=2)
    return _rot_to_quat_fast(rot)


def _scales(rng, n, log_sd, clip=None, mean=0.03):
    s = np.exp(rng.normal(math.log(mean), log_sd, (n, 2)))
    if clip is not None:
        s = np.clip(s, clip[0], clip[1])
    return s


def _grid(rng, levels, log2_size, feat, dtype, amp=1e-2, base=16.0):
    table = rng.uniform(-amp, amp, (levels, 1 << log2_size, feat)).astype(np.float32)
    scales = (base * 1.5 ** np.arange(levels)).astype(np.float32)
    return HashGrid(torch.from_numpy(table).to(dtype), torch.from_numpy(scales))


def _mlp(rng, dims, dtype):
    ws = []
    for i in range(len(dims) - 1):
        fan_in, fan_out = dims[i], dims[i + 1]
        bound = math.sqrt(6.0 / (fan_in + fan_out))
        w = rng.uniform(-bound, bound, (fan_out, fan_in)).astype(np.float32)
        ws.append(torch.from_numpy(w).to(dtype))
    return MLP(ws)


def _pack_scene(means, quats, scales, opac, gammas, colors):
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    return Scene(f(means), f(quats), f(scales), f(opac), f(gammas), f(colors))


def _uniform_scene(rng, n):
    means = rng.uniform(-1.0, 1.0, (n, 3))
    scales = _scales(rng, n, 0.5)
    quats = _unit_quats(rng, n)
    opac = rng.uniform(0.1, 0.99, n)
    colors = rng.uniform(0.0, 1.0, (n, 3))
    gammas = np.ones((n, 2))
    return _pack_scene(means, quats, scales, opac, gammas, colors)


def _planes_scene(rng, n_planar, n_clutter, n_planes=20, half=2.0, scale_mean=0.03):
    """Surfels on random planes through the box [-half, half]^3 plus clutter."""
    normals = rng.standard_normal((n_planes, 3))
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    points = rng.uniform(-1.5, 1.5, (n_planes, 3))
    per = n_planar // n_planes
    means_l, norm_l = [], []
    radius = half * math.sqrt(3.0) + 1.5 * math.sqrt(3.0)
    for p in range(n_planes):
        nrm = normals[p]
        helper = np.array([1.0, 0.0, 0.0]) if abs(nrm[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        a = np.cross(nrm, helper)
        a /= np.linalg.norm(a)
        b = np.cross(nrm, a)
        got = []
        have = 0
        while have < per:
            uv = rng.uniform(-radius, radius, (4 * per, 2))
            cand = points[p] + uv[:, :1] * a + uv[:, 1:] * b
            keep = np.all(np.abs(cand) <= half, axis=1)
            cand = cand[keep]
            got.append(cand)
            have += cand.shape[0]
        cand = np.concatenate(got)[:per]
        cand = cand + rng.normal(0.0, 0.01, (per, 1)) * nrm
        means_l.append(cand)
        norm_l.append(np.repeat(nrm[None], per, axis=0))
    planar_means = np.concatenate(means_l)
    planar_normals = np.concatenate(norm_l)
    planar_quats = _plane_quats(rng, planar_normals)
    clutter_means = rng.uniform(-half, half, (n_clutter, 3))
    clutter_quats = _unit_quats(rng, n_clutter)
    means = np.concatenate([planar_means, clutter_means])
    quats = np.concatenate([planar_quats, clutter_quats])
    n = means.shape[0]
    scales = _scales(rng, n, 0.5, mean=scale_mean)
    opac = rng.uniform(0.1, 0.99, n)
    colors = rng.uniform(0.0, 1.0, (n, 3))
    gammas = np.ones((n, 2))
    return _pack_scene(means, quats, scales, opac, gammas, colors)


def _outdoor_scene(rng, n_ground, n_boxes_total, n_boxes=50, cam_eye=(0.0, 1.0, 0.0)):
    """Ground plane y=0 (x in [-50,50], z in [0,50]) plus surfels on box faces."""
    g_means = np.stack([rng.uniform(-50.0, 50.0, n_ground), np.zeros(n_ground), rng.uniform(0.0, 50.0, n_ground)], 1)
    g_normals = np.repeat(np.array([[0.0, 1.0, 0.0]]), n_ground, axis=0)
    eye = np.asarray(cam_eye)
    centres, sizes = [], []
    while len(centres) < n_boxes:
        size = rng.uniform(0.5, 5.0, 3)
        dist = rng.uniform(1.0, 45.0)
        phi = rng.uniform(-math.radians(40.0), math.radians(40.0))
        c = np.array([dist * math.sin(phi), size[1] / 2.0, dist * math.cos(phi)])
        # keep the camera at least 0.5 m outside every box
        gap = np.maximum(np.abs(eye - c) - size / 2.0, 0.0)
        if np.linalg.norm(gap) < 0.5:
            continue
        centres.append(c)
        sizes.append(size)
    centres = np.array(centres)
    sizes = np.array(sizes)
    per_box = n_boxes_total // n_boxes
    b_means, b_normals = [], []
    for i in range(n_boxes):
        c, s = centres[i], sizes[i]
        areas = np.array([s[1] * s[2], s[1] * s[2], s[0] * s[2], s[0] * s[2], s[0] * s[1], s[0] * s[1]])
        face = rng.choice(6, size=per_box, p=areas / areas.sum())
        uv = rng.uniform(-0.5, 0.5, (per_box, 3)) * s
        axis = face // 2
        sign = np.where(face % 2 == 0, 1.0, -1.0)
        pts = uv.copy()
        pts[np.arange(per_box), axis] = sign * s[axis] / 2.0
        nrm = np.zeros((per_box, 3))
        nrm[np.arange(per_box), axis] = sign
        b_means.append(c + pts)
        b_normals.append(nrm)
    means = np.concatenate([g_means] + b_means)
    normals = np.concatenate([g_normals] + b_normals)
    quats = _plane_quats(rng, normals)
    n = means.shape[0]
    scales = _scales(rng, n, 1.0, clip=(9.5e-4, 0.95))
    opac = rng.uniform(0.1, 0.99, n)
    colors = rng.uniform(0.0, 1.0, (n, 3))
    gammas = np.ones((n, 2))
    return _pack_scene(means, quats, scales, opac, gammas, colors)


def _random_look(rng, eye_low, eye_high, width, height):
    eye = rng.uniform(eye_low, eye_high, 3)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    up = np.array([0.0, -1.0, 0.0]) if abs(d[1]) < 0.95 else np.array([1.0, 0.0, 0.0])
    return look_at(eye, eye + d, up, width, height)


def _target_images(rng, cams):
    return [torch.from_numpy(rng.uniform(0.0, 1.0, (c.height, c.width, 3)).astype(np.float32)) for c in cams]


def with_sh(wl: Workload, seed: int = 0, ac_sd: float = 0.2) -> Workload:
    """The same workload with the spherical-harmonics appearance (degree 3): per-surfel coefficients [N,48]
    whose DC term reproduces the RGB colour (a_0 = (c - 0.5) / Y_0, Y_0 = 0.5 / sqrt(pi)) and whose higher
    terms are N(0, ac_sd^2), and a 48-output head (Xavier-uniform) in the MLP's dtype. Drawn from a generator
    of its own (PCG64(seed + 7919)), so the base workload is unchanged."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    rgb = wl.scene.colors.double().numpy()
    n = rgb.shape[0]
    coef = rng.normal(0.0, ac_sd, (n, 16, 3))
    coef[:, 0, :] = (rgb - 0.5) / (0.5 / math.sqrt(math.pi))
    scene = Scene(*wl.scene.tensors()[:5], torch.from_numpy(coef.reshape(n, 48).astype(np.float32)))
    w = wl.mlp.weights
    hid = w[2].shape[1]
    b = math.sqrt(6.0 / (hid + 48))
    head = torch.from_numpy(rng.uniform(-b, b, (48, hid)).astype(np.float32)).to(w[2].dtype)
    return Workload(wl.name + "_sh3", scene, wl.cameras, wl.grid, MLP([w[0], w[1], head]), wl.K, wl.target, 3)


def make_workload(config: int, seed: int = 0, *, n_surfels=None, width=None, height=None,
                  feat_dtype=None, mlp_dtype=None, K=None, grid_amp=1e-2) -> Workload:
    """Build one of the five synthetic workloads.

    1: 2000 surfels uniform in [-1,1]^3, 128x128, K=4, grid 8 x 2^14 x 2 fp32, MLP 16-64-64-3 fp32.
    2: 100k surfels on 20 planes + 10% clutter in [-2,2]^3, indoor camera 1024x768, K=4,
       grid 16 x 2^19 x 2 fp32, MLP 32-64-64-3 fp32, random target image.
    3: 400k surfels on a ground plane plus 50 boxes, 1920x1080, K=4, grid 16 x 2^19 x 2 fp16,
       MLP 32-64-64-3 bf16, random target image.
    4: config-2 generator at 300k, 16 orbit cameras with mixed resolutions, fp32.
    5: config-3 generator at 1M, 2560x1440, K=8, grid 16 x 2^21 x 2 bf16, MLP 32-128-128-3 bf16.

    Keyword overrides shrink a workload for tests (surfel count, image size,
    dtypes, K) or scale the table's initial entries to U(-grid_amp, grid_amp);
    the draw order is unchanged.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if config == 1:
        n = n_surfels or 2000
        scene = _uniform_scene(rng, n)
        w, h = width or 128, height or 128
        cam = look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), (0.0, -1.0, 0.0), w, h)
        grid = _grid(rng, 8, 14, 2, feat_dtype or torch.float32, amp=grid_amp)
        mlp = _mlp(rng, [16, 64, 64, 3], mlp_dtype or torch.float32)
        cams = [cam]
        target = _target_images(rng, cams)
        return Workload(CONFIG_NAMES[1], scene, cams, grid, mlp, K or 4, target)
    if config == 2 or config == 4:
        if config == 2:
            n = n_surfels or 100_000
            scene = _planes_scene(rng, int(n * 0.9), n - int(n * 0.9))
            w, h = width or 1024, height or 768
            cams = [_random_look(rng, -1.0, 1.0, w, h)]
        else:
            n = n_surfels or 300_000
            scene = _planes_scene(rng, int(n * 0.9), n - int(n * 0.9))
            res = [(640, 480), (1024, 768), (1280, 720), (1920, 1080)]
            cams = []
            for _ in range(16):
                ang = rng.uniform(0.0, 2.0 * math.pi)
                hgt = rng.uniform(-0.5, 0.5)
                eye = np.array([math.cos(ang), hgt, math.sin(ang)])
                tgt = rng.normal(0.0, 0.2, 3)
                rw, rh = res[int(rng.integers(0, 4))]
                if width is not None:
                    rw, rh = width, height
                cams.append(look_at(eye, tgt, (0.0, -1.0, 0.0), rw, rh))
        grid = _grid(rng, 16, 19, 2, feat_dtype or torch.float32, amp=grid_amp)
        mlp = _mlp(rng, [32, 64, 64, 3], mlp_dtype or torch.float32)
        target = _target_images(rng, cams)
        return Workload(CONFIG_NAMES[config], scene, cams, grid, mlp, K or 4, target)
    if config == 3 or config == 5:
        n = n_surfels or (400_000 if config == 3 else 1_000_000)
        n_ground = int(round(n * 0.6))
        scene = _outdoor_scene(rng, n_ground, n - n_ground)
        if config == 3:
            w, h = width or 1920, height or 1080
        else:
            w, h = width or 2560, height or 1440
        pitch = math.radians(15.0)
        eye = np.array([0.0, 1.0, 0.0])
        fwd = np.array([0.0, -math.sin(pitch), math.cos(pitch)])
        cam = look_at(eye, eye + fwd, (0.0, 1.0, 0.0), w, h)
        if config == 3:
            grid = _grid(rng, 16, 19, 2, feat_dtype or torch.float16, amp=grid_amp)
            mlp = _mlp(rng, [32, 64, 64, 3], mlp_dtype or torch.bfloat16)
            kk = K or 4
        else:
            grid = _grid(rng, 16, 21, 2, feat_dtype or torch.bfloat16, amp=grid_amp)
            mlp = _mlp(rng, [32, 128, 128, 3], mlp_dtype or torch.bfloat16)
            kk = K or 8
        cams = [cam]
        target = _target_images(rng, cams)
        return Workload(CONFIG_NAMES[config], scene, cams, grid, mlp, kk, target)
    raise ValueError(f"unknown config {config}")


@dataclasses.dataclass
class TrainWorkload:
    scene: Scene          # geometry and the colours the targets were made with
    cameras: list         # training views first, the held-out view last
    teacher_grid: HashGrid
    teacher_mlp: MLP
    init_colors: torch.Tensor
    init_grid: HashGrid
    init_mlp: MLP
    K: int
    init_gammas: torch.Tensor = None  # the students' starting exponents (None: the scene's own)


def make_train_workload(seed: int = 0, n_surfels: int = 3000, n_views: int = 7, width: int = 64,
                        height: int = 64, K: int = 4, teacher_gamma: float = None) -> TrainWorkload:
    """A small textured scene for the training check.

    Surfels on 6 planes through [-2,2]^3 (no clutter) with scales around 0.15;
    a teacher grid (8 levels x 2^14 x 2, entries U(-1,1), level scales
    2 * 1.5^l so that the coarse levels stay above the pixel footprint at this
    resolution) and a teacher MLP 16-64-64-3 give the targets a texture that
    per-surfel colours cannot express (its output layer is scaled by 8 so the
    texture varies by about 0.06 within a surfel). Cameras sit on an arc of radius 6 at
    heights U(0.5, 1.5) looking at the origin; the held-out view lies between
    two training views. The student starts from fresh colours U[0,1], a grid
    U(-1e-2, 1e-2) with the same level scales, and a fresh MLP.

    teacher_gamma: the teacher's surfels use this kernel exponent on both
    axes (flat-topped, near-rectangular footprints) while the students start
    from gamma = 1 (Gaussians); set after every random draw, so the rest of
    the workload is unchanged.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    scene = _planes_scene(rng, n_surfels, 0, n_planes=6, half=2.0, scale_mean=0.15)
    angles = list(np.linspace(-0.7, 0.7, n_views - 1)) + [0.7 / (n_views - 2)]
    cams = []
    for a in angles:
        eye = np.array([6.0 * math.sin(a), rng.uniform(0.5, 1.5), -6.0 * math.cos(a)])
        cams.append(look_at(eye, (0.0, 0.0, 0.0), (0.0, -1.0, 0.0), width, height))
    teacher_grid = _grid(rng, 8, 14, 2, torch.float32, amp=1.0, base=2.0)
    teacher_mlp = _mlp(rng, [16, 64, 64, 3], torch.float32)
    teacher_mlp.weights[2] = teacher_mlp.weights[2] * 8.0  # contrast: texture std ~0.1 within a surfel
    init_colors = torch.from_numpy(rng.uniform(0.0, 1.0, (scene.n, 3)).astype(np.float32))
    init_grid = _grid(rng, 8, 14, 2, torch.float32, amp=1e-2, base=2.0)
    init_mlp = _mlp(rng, [16, 64, 64, 3], torch.float32)
    init_gammas = None
    if teacher_gamma is not None:
        init_gammas = torch.ones_like(scene.gammas)
        scene.gammas = torch.full_like(scene.gammas, float(teacher_gamma))
    return TrainWorkload(scene, cams, teacher_grid, teacher_mlp, init_colors, init_grid, init_mlp, K, init_gammas)
