"""The two rendering passes and their gradients, untiled, in FP64 (oracle).

Paper references:
  * eq. composite: C = sum_i T_i alpha_i c_i with T_i = prod_{j<i} (1 - alpha_j)
    (the printed product index is read as j).
  * Rendering, Collection Pass: blending weights w_i = alpha_i T_i; the K
    primitives with the highest weights are selected per pixel and their
    id, weight and depth are returned as the H x W x K images I, W, D;
    eq. notexture: N_p sums w_i c_i over the surfels not selected.
  * Rendering, Texturing Pass and eq. texture: x = o + D d per selected slot,
    Tex_{p,j} = G(Delta(r) * H(x)).
  * eq. final: C_p = N_p + sum_j W_{p,j} Tex_{p,j}.
  * Results (implementation) and the supplementary: parameter activations are
    done by the caller; gradients flow to every surfel that was composited,
    textured or not (Further Discussion, Texturing Strategy).

Per pixel, every surfel is intersected (no tiling), the surfels that pass are
ordered by (centre-depth key, id), composited front to back, and the top-K
set is found by a full sort under the total order (weight descending, id
ascending). Output slots follow compositing order; empty slots hold id -1,
weight 0, depth 0 and texture 0.

Gradients are reverse-mode autograd through the same FP64 expressions, with
every discrete choice (support test, alpha threshold, stop, top-K, hash
cell) held at the value the forward took; tests pin them to central finite
differences.

Each pixel also reports how robust its discrete decisions are: for every
decision (alpha threshold and clamp, support box and near plane, the stop
test, the K-th versus (K+1)-th weight, the sign of every hidden MLP
pre-activation of its textured samples) the relative distance to the
threshold is divided by an estimate of the relative error an FP32
evaluation makes in that quantity, and the smallest ratio is returned. A
pixel whose ratio is well above 1 has decisions FP32 rounding cannot flip.
Error scales (relative worst-case bounds): u, v and t 3e-7 (a few FP32
roundings of offsets from the projected centre); alpha 3e-7 + 4e-7 g E
(E = |u|^2g1 + |v|^2g2 is the kernel exponent, g the larger gamma: the
exponent inherits the relative error of u and v times 2g, plus the exp2
rounding); transmittance and weights the sum of 1.2e-7 + e_alpha
alpha / (1 - alpha) over the surfels composited so far (1 - alpha inherits
alpha's absolute error); MLP pre-activations `mlp_rel_err` times
sum_j |W_ij x_j| (a 64-term FP32 accumulation plus the feature errors). The ReLU
decisions change gradients only (the forward is continuous in them), so
they are reported separately as `mlp_margin`.

force_cells pins the hash-grid lattice cell of each textured sample to the
one another implementation reports, so that positional gradients are
compared on the same branch of the piecewise-trilinear interpolation.

want_decisions=True also returns the natural (unforced) decisions' inputs
of every textured slot: the lattice positions s_l x (their floors are the
natural cells) and the features z evaluated in the natural cells (the
hidden pre-activations of the natural MLP follow from them), so that a
decision another implementation reports can be checked against the FP64
one.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from .binning import bin_surfels
from .constants import ALPHA_MAX, ALPHA_MIN, NEAR, SUPPORT, T_MIN
from .geometry import camera_origin_and_rays, intersect, kernel, quat_columns
from .hashgrid import encode
from .mlp import mlp_forward, unpack_masks
from .sh import colour as sh_colour


@dataclasses.dataclass
class OracleOutputs:
    pixels: np.ndarray   # [P] flat pixel indices (y * W + x)
    image: np.ndarray    # [P,3]
    plain: np.ndarray    # [P,3] N, the non-textured render without the K selected
    ids: np.ndarray      # [P,K] int64, -1 for empty slots
    weights: np.ndarray  # [P,K]
    depths: np.ndarray   # [P,K]
    t_final: np.ndarray  # [P]
    tex: np.ndarray      # [P,K,3]
    n_comp: np.ndarray   # [P] number of composited surfels
    margin: np.ndarray   # [P] collection-pass decisions: smallest margin / FP32 error scale
    mlp_margin: np.ndarray = None  # [P] MLP ReLU decisions of the textured samples, same units
    lattice: np.ndarray = None     # [P,K,L,3] s_l x per textured slot (NaN for empty slots), want_decisions only
    features: np.ndarray = None    # [P,K,L*F] natural-cell features z per textured slot (0 if empty)
    blended_error: np.ndarray = None  # [N] sum over pixels of w_{i,p} E_p, when pixel_error is given
    grads: dict | None = None


_PARAM_NAMES = ("means", "quats", "scales", "opacities", "gammas", "colors")


def _leaf(t, need_grad):
    x = t.detach().to(torch.float64).clone()
    if need_grad:
        x.requires_grad_(True)
    return x


def render(scene, cam, grid, mlp, K, pixels=None, tiled=False, bins=None, **kw):
    """Forward only. See render_and_grad."""
    return render_and_grad(scene, cam, grid, mlp, K, pixels=pixels, tiled=tiled, bins=bins, **kw)


def render_and_grad(scene, cam, grid, mlp, K, pixels=None, grad_image=None, grad_weights=None,
                    grad_tex=None, tiled=False, bins=None, outer_pixels=2048, pair_budget=3_000_000,
                    force_cells=None, force_relu=None, mlp_rel_err=5e-6, want_decisions=False, pixel_error=None,
                    sh_degree=None):
    """Render the given pixels (all by default) and optionally back-propagate.

    grad_image [P,3], grad_weights [P,K] and grad_tex [P,K,3] are upstream
    gradients for the listed pixels, in the order of ``pixels``. When any is
    given, the returned ``grads`` dict holds d(loss)/d(parameter) for
    means, quats, scales, opacities, gammas, colors, table (float64, the
    table's shape) and mlp (list of [out,in]).
    tiled=True restricts each pixel's candidates to its tile list from the
    binning step (used to check that binning loses no surfel).
    force_cells [P,K,L,3] (int, aligned with ``pixels``) fixes the hash-grid
    cell per textured slot and level; force_relu [P,K,2*hidden/32] (uint32
    bit words, layer 1 then layer 2) fixes the ReLU decisions per slot;
    mlp_rel_err is the relative error scale of the MLP pre-activations used
    for the decision margins. want_decisions fills ``lattice`` and ``features``.
    pixel_error [P] (per listed pixel) fills ``blended_error``: per surfel the
    sum over pixels of its blending weight w = alpha T times the pixel's error
    (supplementary, Densification: the blended errors of Rota Bulo et al.,
    accumulated by adding).
    sh_degree (None: RGB colours [N,3] and a sigmoid head) selects the
    spherical-harmonics appearance (Representation, Appearance): colours
    [N,3 (d+1)^2] are per-surfel coefficients decoded along the unit
    direction from the camera centre to the surfel centre, and the MLP head's
    3 (d+1)^2 outputs are coefficients decoded along the pixel's unit ray
    direction (oracle.sh.colour: max(0, sum_k Y_k a_k + 0.5)).
    """
    need_grad = grad_image is not None or grad_weights is not None or grad_tex is not None
    W, H = cam.width, cam.height
    if pixels is None:
        pixels = np.arange(W * H, dtype=np.int64)
    pixels = np.asarray(pixels, dtype=np.int64)
    P = pixels.shape[0]
    if bins is None:
        bins = bin_surfels(scene, cam)

    prm = {nm: _leaf(t, need_grad) for nm, t in zip(_PARAM_NAMES, scene.tensors())}
    table = _leaf(grid.table, need_grad)
    weights = [_leaf(w, need_grad) for w in mlp.weights]
    level_scales = grid.level_scales.to(torch.float64)
    key_np = bins["key"]
    alive_ids = np.nonzero(bins["alive"])[0]

    with torch.no_grad():
        all_v1, all_v2, all_v3 = quat_columns(prm["quats"].detach())
        all_mu = prm["means"].detach()
        all_sg = prm["scales"].detach()

    out = {
        "image": np.zeros((P, 3)), "plain": np.zeros((P, 3)), "ids": np.full((P, K), -1, dtype=np.int64),
        "weights": np.zeros((P, K)), "depths": np.zeros((P, K)), "t_final": np.ones(P),
        "tex": np.zeros((P, K, 3)), "n_comp": np.zeros(P, dtype=np.int64), "margin": np.full(P, np.inf),
        "mlp_margin": np.full(P, np.inf),
    }
    if want_decisions:
        L_, F_ = grid.table.shape[0], grid.table.shape[2]
        out["lattice"] = np.full((P, K, L_, 3), np.nan)
        out["features"] = np.zeros((P, K, L_ * F_))
    if pixel_error is not None:
        out["blended_error"] = np.zeros(scene.n)
        perr = np.asarray(pixel_error, dtype=np.float64)
    if P == 0:
        return OracleOutputs(pixels=pixels, grads=_collect_grads(prm, table, weights) if need_grad else None, **out)

    gi = None if grad_image is None else torch.as_tensor(np.asarray(grad_image), dtype=torch.float64)
    gw = None if grad_weights is None else torch.as_tensor(np.asarray(grad_weights), dtype=torch.float64)
    gt = None if grad_tex is None else torch.as_tensor(np.asarray(grad_tex), dtype=torch.float64)

    if tiled:
        ntx = bins["ntx"]
        tile_of = (pixels // W // 16) * ntx + (pixels % W) // 16
        order = np.argsort(tile_of, kind="stable")
    else:
        order = np.arange(P)

    for c0 in range(0, P, outer_pixels):
        sel = order[c0:c0 + outer_pixels]
        pix = pixels[sel]
        px = pix % W
        py = pix // W
        o, d = camera_origin_and_rays(cam, px, py)

        # Phase 1: which (pixel, surfel) pairs can contribute (relaxed test, no gradient).
        pair_p, pair_s = [], []
        if tiled:
            tl = (py // 16) * bins["ntx"] + px // 16
            groups = [(np.nonzero(tl == t)[0], bins["ids"][bins["ranges"][t, 0]:bins["ranges"][t, 1]])
                      for t in np.unique(tl)]
        else:
            step = max(1, pair_budget // max(1, alive_ids.shape[0]))
            groups = [(np.arange(i, min(i + step, pix.shape[0])), alive_ids) for i in range(0, pix.shape[0], step)]
        with torch.no_grad():
            for rows, cand in groups:
                if cand.shape[0] == 0 or rows.shape[0] == 0:
                    continue
                ct = torch.from_numpy(cand)
                t, u, v, den = intersect(o, d[rows].unsqueeze(1), all_mu[ct].unsqueeze(0), all_v1[ct].unsqueeze(0),
                                         all_v2[ct].unsqueeze(0), all_v3[ct].unsqueeze(0), all_sg[ct].unsqueeze(0))
                ok = (den != 0) & (t > NEAR * (1.0 - 1e-9)) & (u.abs() <= SUPPORT * (1.0 + 1e-9)) \
                    & (v.abs() <= SUPPORT * (1.0 + 1e-9))
                r, c = torch.nonzero(ok, as_tuple=True)
                pair_p.append(rows[r.numpy()])
                pair_s.append(cand[c.numpy()])
        Pc = pix.shape[0]
        pp = np.concatenate(pair_p) if pair_p else np.zeros(0, dtype=np.int64)
        ss = np.concatenate(pair_s) if pair_s else np.zeros(0, dtype=np.int64)

        fc = None if force_cells is None else np.asarray(force_cells)[sel]
        fr = None if force_relu is None else np.asarray(force_relu)[sel]
        res = _composite_chunk(pp, ss, Pc, o, d, prm, key_np, K, table, level_scales, cam.fx, weights, fc,
                               mlp_rel_err, fr, want_decisions, sh_degree)
        for nm in ("image", "plain", "weights", "depths", "t_final", "tex"):
            out[nm][sel] = res[nm].detach().numpy()
        for nm in ("ids", "n_comp", "margin", "mlp_margin"):
            out[nm][sel] = res[nm]
        if want_decisions:
            out["lattice"][sel] = res["lattice"]
            out["features"][sel] = res["features"]
        if pixel_error is not None:
            rows, cols = np.nonzero(res["comp"])
            np.add.at(out["blended_error"], res["sid"][rows, cols], res["wfull"][rows, cols] * perr[sel][rows])

        if need_grad:
            loss = torch.zeros((), dtype=torch.float64)
            st = torch.from_numpy(sel)
            if gi is not None:
                loss = loss + (gi[st] * res["image"]).sum()
            if gw is not None:
                loss = loss + (gw[st] * res["weights"]).sum()
            if gt is not None:
                loss = loss + (gt[st] * res["tex"]).sum()
            if loss.requires_grad:
                loss.backward()

    grads = _collect_grads(prm, table, weights) if need_grad else None
    return OracleOutputs(pixels=pixels, grads=grads, **out)


def _collect_grads(prm, table, weights):
    g = {}
    for nm, t in prm.items():
        g[nm] = (t.grad if t.grad is not None else torch.zeros_like(t)).numpy()
    g["table"] = (table.grad if table.grad is not None else torch.zeros_like(table)).numpy()
    g["mlp"] = [(w.grad if w.grad is not None else torch.zeros_like(w)).numpy() for w in weights]
    return g


def _unit(v):
    return v / torch.sqrt((v * v).sum(dim=-1, keepdim=True))


def _composite_chunk(pp, ss, Pc, o, d, prm, key_np, K, table, level_scales, focal, weights, force_cells=None,
                     mlp_rel_err=5e-6, force_relu=None, want_decisions=False, sh_degree=None):
    """Phase 2 for one chunk of pixels: exact decisions, compositing, texture."""
    E = pp.shape[0]
    order = np.lexsort((ss, key_np[ss].astype(np.float64), pp))
    pp = pp[order]
    ss = ss[order]
    st = torch.from_numpy(ss)
    ptt = torch.from_numpy(pp)

    mu = prm["means"][st]
    v1, v2, v3 = quat_columns(prm["quats"][st])
    sg = prm["scales"][st]
    t, u, v, den = intersect(o, d[ptt], mu, v1, v2, v3, sg)
    supp = (den != 0) & (t > NEAR) & (u.abs() <= SUPPORT) & (v.abs() <= SUPPORT)
    G = kernel(u, v, prm["gammas"][st])
    a_raw = prm["opacities"][st] * G
    alpha = torch.clamp(a_raw, max=ALPHA_MAX)
    valid = supp & (alpha >= ALPHA_MIN)

    counts = np.bincount(pp, minlength=Pc)
    starts = np.cumsum(counts) - counts
    col = np.arange(E, dtype=np.int64) - starts[pp]
    M = max(1, int(counts.max()) if E else 1)
    colt = torch.from_numpy(col)

    zeros = torch.zeros(Pc, M, dtype=torch.float64)
    A = zeros.index_put((ptt, colt), torch.where(valid, alpha, torch.zeros_like(alpha)))
    Td = zeros.index_put((ptt, colt), t.where(supp, torch.zeros_like(t)))
    vd = torch.zeros(Pc, M, dtype=torch.bool).index_put((ptt, colt), valid)
    sid_d = torch.full((Pc, M), -1, dtype=torch.int64).index_put((ptt, colt), st)
    if sh_degree is None:
        pair_col = prm["colors"][st]
    else:
        pair_col = sh_colour(prm["colors"][st], _unit(mu - o), sh_degree)
    cols_d = torch.zeros(Pc, M, 3, dtype=torch.float64).index_put((ptt, colt), pair_col)

    Ta = torch.cumprod(1.0 - A, dim=1)
    Tb = torch.cat([torch.ones(Pc, 1, dtype=torch.float64), Ta[:, :-1]], dim=1)
    with torch.no_grad():
        stop_hit = vd & (Ta < T_MIN)
        colgrid = torch.arange(M).unsqueeze(0).expand(Pc, M)
        s = torch.where(stop_hit, colgrid, torch.full_like(colgrid, M)).min(dim=1).values
        comp = vd & (colgrid < s.unsqueeze(1))
    w = A * Tb * comp
    Text = torch.cat([torch.ones(Pc, 1, dtype=torch.float64), Ta], dim=1)
    t_final = Text.gather(1, s.unsqueeze(1)).squeeze(1)

    # Top-K by (weight desc, id asc), then slots in compositing order.
    with torch.no_grad():
        wn = w.detach().numpy()
        compn = comp.numpy()
        sidn = sid_d.numpy()
        score = np.where(compn, -wn, np.inf)
        rank = np.lexsort((sidn, score), axis=1)
        kk = min(K, M)
        top = rank[:, :kk]
        top_ok = np.take_along_axis(compn, top, axis=1)
        top = np.where(top_ok, top, M)
        top.sort(axis=1)
        slot_cols = np.full((Pc, K), M, dtype=np.int64)
        slot_cols[:, :kk] = top
        has = slot_cols < M
        selmask = np.zeros((Pc, M + 1), dtype=bool)
        np.put_along_axis(selmask, slot_cols, True, axis=1)
        selmask = selmask[:, :M]
        n_comp = compn.sum(axis=1)

    has_t = torch.from_numpy(has)
    sc = torch.from_numpy(np.where(has, slot_cols, 0))
    Wk = w.gather(1, sc) * has_t
    Dk = Td.gather(1, sc) * has_t
    Ik = np.where(has, np.take_along_axis(sidn, np.where(has, slot_cols, 0), axis=1), -1)

    notsel = comp & ~torch.from_numpy(selmask)
    plain = ((w * notsel).unsqueeze(-1) * cols_d).sum(dim=1)

    # Texturing pass on the selected slots.
    rows, slots = np.nonzero(has)
    tex = torch.zeros(Pc, K, 3, dtype=torch.float64)
    relu_margin = np.full(Pc, np.inf)
    n_lv = table.shape[0]
    lattice = np.full((Pc, K, n_lv, 3), np.nan) if want_decisions else None
    features = np.zeros((Pc, K, n_lv * table.shape[2])) if want_decisions else None
    if rows.shape[0] > 0:
        rt, stt = torch.from_numpy(rows), torch.from_numpy(slots)
        D = Dk[rt, stt]
        x = o + D.unsqueeze(1) * d[rt]
        cells = None if force_cells is None else force_cells[rows, slots]
        z = encode(x, D, table, level_scales, focal, cells=cells)
        if want_decisions:
            with torch.no_grad():
                xd = x.detach()
                lattice[rows, slots] = np.stack([float(level_scales[l]) * xd.numpy() for l in range(n_lv)], axis=1)
                zn = z if cells is None else encode(xd, D.detach(), table.detach(), level_scales, focal)
                features[rows, slots] = zn.detach().numpy()
        masks = None
        if force_relu is not None:
            masks = unpack_masks(force_relu[rows, slots], weights[0].shape[0], len(weights) - 1)
        if sh_degree is None:
            out = mlp_forward(z, weights, relu_masks=masks)
        else:
            out = sh_colour(mlp_forward(z, weights, relu_masks=masks, head="linear"), _unit(d[rt]), sh_degree)
        tex = tex.index_put((rt, stt), out)
        with torch.no_grad():
            sm = _relu_margins(z.detach(), [w.detach() for w in weights]) / mlp_rel_err
        np.minimum.at(relu_margin, rows, sm)
    image = plain + (Wk.unsqueeze(-1) * tex).sum(dim=1)

    E = (-2.0 * torch.log(G.detach().clamp_min(1e-300))).numpy()
    gmax = prm["gammas"][st].detach().max(dim=1).values.numpy()
    margin = _margins(pp, col, Pc, M, s.numpy(), supp.numpy(), alpha.detach().numpy(), a_raw.detach().numpy(),
                      u.detach().numpy(), v.detach().numpy(), t.detach().numpy(), Ta.detach().numpy(),
                      compn, wn, K, E, gmax)
    return {"image": image, "plain": plain, "weights": Wk, "depths": Dk, "t_final": t_final, "tex": tex,
            "ids": Ik, "n_comp": n_comp, "margin": margin, "mlp_margin": relu_margin, "lattice": lattice,
            "features": features, "comp": compn, "sid": sidn, "wfull": wn}


def _relu_margins(z, weights):
    """Per sample: min over hidden units of |h_i| / sum_j |W_ij x_j| (inf if all inputs are 0)."""
    m = torch.full((z.shape[0],), float("inf"), dtype=torch.float64)
    h = z
    for w in weights[:-1]:
        pre = h @ w.t()
        scale = h.abs() @ w.abs().t()
        r = torch.where(scale > 0, pre.abs() / scale, torch.full_like(pre, float("inf")))
        m = torch.minimum(m, r.min(dim=1).values)
        h = torch.relu(pre)
    return m.numpy()


def _margins(pp, col, Pc, M, s, supp, alpha, a_raw, u, v, t, Ta, comp, w, K, E, gmax):
    """Smallest (relative margin / FP32 relative error scale) over every decision of each pixel."""
    m = np.full(Pc, np.inf)
    considered = col < s[pp]
    big = np.inf
    e_alpha = 3e-7 + 4e-7 * gmax * E
    e_geo = 3e-7
    with np.errstate(divide="ignore", invalid="ignore"):
        ma = np.where(considered & supp, np.abs(alpha - ALPHA_MIN) / ALPHA_MIN / e_alpha, big)
        mc = np.where(considered & supp, np.abs(a_raw - ALPHA_MAX) / ALPHA_MAX / e_alpha, big)
        matters = considered & (a_raw >= 0.5 * ALPHA_MIN)
        ms = np.minimum(np.abs(np.abs(u) - SUPPORT), np.abs(np.abs(v) - SUPPORT)) / SUPPORT / e_geo
        mn = np.abs(t - NEAR) / NEAR / e_geo
        msn = np.where(matters, np.minimum(ms, mn), big)
    per_pair = np.minimum(np.minimum(ma, mc), msn)
    np.minimum.at(m, pp, per_pair)
    # Transmittance error accumulated along each pixel's list (composited entries and the stop entry).
    ea = np.zeros((Pc, M))
    ea[pp, col] = np.where(supp, e_alpha, 0.0)
    al = np.zeros((Pc, M))
    al[pp, col] = np.where(supp, alpha, 0.0)
    rows = np.arange(Pc)
    stopped = s < M
    incl = comp.copy()
    incl[rows[stopped], s[stopped]] = True
    step_err = np.where(incl, 1.2e-7 + ea * al / np.maximum(1.0 - al, 1e-12), 0.0)
    e_T = np.cumsum(step_err, axis=1)
    if stopped.any():
        r = rows[stopped]
        m[r] = np.minimum(m[r], (T_MIN - Ta[r, s[r]]) / T_MIN / e_T[r, s[r]])
    lastc = np.where(comp, np.arange(M)[None, :], -1).max(axis=1)
    hasc = lastc >= 0
    if hasc.any():
        r = rows[hasc]
        m[r] = np.minimum(m[r], (Ta[r, lastc[r]] - T_MIN) / T_MIN / e_T[r, lastc[r]])
    # K-th versus (K+1)-th weight
    if M > K:
        ws = np.sort(np.where(comp, w, -np.inf), axis=1)[:, ::-1]
        wk = ws[:, K - 1] if K > 0 else np.full(Pc, np.inf)
        wk1 = ws[:, K]
        e_w = np.where(hasc, e_T[rows, np.maximum(lastc, 0)], 0.0) + np.max(np.where(comp, ea, 0.0), axis=1)
        ok = np.isfinite(wk1) & (wk > 0) & (K > 0)
        with np.errstate(divide="ignore", invalid="ignore"):
            mk = np.where(ok, (wk - wk1) / wk / np.maximum(e_w, 1e-12), np.inf)
        m = np.minimum(m, mk)
    return m
