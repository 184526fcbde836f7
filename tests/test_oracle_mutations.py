"""The oracle pins constrain the parts of the oracle that plausible mistakes
would change (CPU only).

Each case copies the oracle, the scene generator and the tests to a scratch
directory, plants one mistake in the copy of the oracle, and runs the pins
there: at least one pin that names the mutated part must fail, and the
untouched copy must pass them all.

  stop     compositing also the surfel that takes T below 1e-4
           (eq. composite with the 3DGS termination)
  clamp    alpha clamped at 0.999 instead of 0.99
  camera   world ray directions built with R instead of R^T (pinhole rays)
  axes     quaternion matrix rows taken as the surfel axes instead of its
           columns, R = [v1 v2 v3] (Representation, Geometry)

and, for the appearance, loss and density-control parts (each run against
its own pin file):

  sh_constant   the degree-1 SH constant with 2 pi instead of 4 pi
  sh_offset     the SH colour without its +0.5
  sh_clamp      the SH colour without its clamp at 0
  grid_scale    L_grid weighted by s_l^-2 instead of s_l^-3
  texture_norm  L_texture on the premultiplied texture (no division by the
                weights' sum)
  fps_ties      FPS ties broken towards the largest index
  draw_key      the split draw keyed by w / e instead of e / w
  split_axis    a surfel split along its short axis
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PINS = ["test_stop_rule_stack_of_opaque_surfels", "test_alpha_clamp_at_full_opacity",
        "test_quaternion_columns_are_rodrigues_axes", "test_quarter_turn_swaps_the_surfel_axes",
        "test_camera_looks_along_its_axis", "test_rigid_motion_of_scene_and_camera_changes_nothing"]

MUTATIONS = {
    "stop": [("oracle/render.py", "comp = vd & (colgrid < s.unsqueeze(1))", "comp = vd & (colgrid <= s.unsqueeze(1))")],
    "clamp": [("oracle/constants.py", "ALPHA_MAX = 0.99", "ALPHA_MAX = 0.999")],
    "camera": [("oracle/geometry.py",
                "d = torch.stack([(r[0, k] * dcx + r[1, k] * dcy) + r[2, k] * dcz for k in range(3)], dim=-1)",
                "d = torch.stack([(r[k, 0] * dcx + r[k, 1] * dcy) + r[k, 2] * dcz for k in range(3)], dim=-1)")],
    "axes": [(f, f"v{i + 1} = {m}.stack([r0{i}, r1{i}, r2{i}]", f"v{i + 1} = {m}.stack([r{i}0, r{i}1, r{i}2]")
             for f, m in (("oracle/geometry.py", "torch"), ("oracle/binning.py", "np")) for i in range(3)],
}

EXPECTED = {
    "stop": {"test_stop_rule_stack_of_opaque_surfels"},
    "clamp": {"test_alpha_clamp_at_full_opacity"},
    "camera": {"test_camera_looks_along_its_axis", "test_rigid_motion_of_scene_and_camera_changes_nothing"},
    "axes": {"test_quaternion_columns_are_rodrigues_axes", "test_rigid_motion_of_scene_and_camera_changes_nothing"},
}


def _copy(tmp):
    for d in ("oracle", "scenes", "tests"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(tmp, d),
                        ignore=shutil.ignore_patterns("__pycache__", "*.pyc"))


def _run_pins(tmp):
    sel = " or ".join(PINS)
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "-q", "-p", "no:cacheprovider",
                        "-k", sel, "-rf"], cwd=tmp, capture_output=True, text=True, timeout=600)
    failed = {ln.split("::")[1].split(" ")[0] for ln in r.stdout.splitlines() if ln.startswith("FAILED")}
    return r.returncode, failed, r.stdout[-2000:]


def test_unmutated_copy_passes(tmp_path):
    _copy(str(tmp_path))
    rc, failed, out = _run_pins(str(tmp_path))
    assert rc == 0 and not failed, out


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(tmp_path, name):
    tmp = str(tmp_path)
    _copy(tmp)
    for rel, old, new in MUTATIONS[name]:
        p = os.path.join(tmp, rel)
        src = open(p).read()
        assert src.count(old) == 1, f"{rel}: the text to mutate is not there exactly once: {old}"
        open(p, "w").write(src.replace(old, new))
    rc, failed, out = _run_pins(tmp)
    assert rc != 0, f"mutation {name} passed every pin:\n{out}"
    assert EXPECTED[name] <= failed, f"mutation {name}: expected {sorted(EXPECTED[name])} to fail, got {sorted(failed)}"


# (file, old text, new text), the pin file, the pins that must fail
MUTATIONS_2 = {
    "sh_constant": ([("oracle/sh.py", "C1 = math.sqrt(3.0 / (4.0 * math.pi))", "C1 = math.sqrt(3.0 / (2.0 * math.pi))")],
                    "tests/test_oracle_sh.py", {"test_orthonormal_over_the_sphere"}),
    "sh_offset": ([("oracle/sh.py", "(y[..., :, None] * a).sum(dim=-2) + 0.5, min=0.0)",
                    "(y[..., :, None] * a).sum(dim=-2) + 0.0, min=0.0)")],
                  "tests/test_oracle_sh.py", {"test_colour_special_cases"}),
    "sh_clamp": ([("oracle/sh.py", "return torch.clamp((y[..., :, None] * a).sum(dim=-2) + 0.5, min=0.0)",
                   "return (y[..., :, None] * a).sum(dim=-2) + 0.5")],
                 "tests/test_oracle_sh.py", {"test_colour_special_cases"}),
    "grid_scale": ([("oracle/losses.py", "l_grid = (s ** -3.0 *", "l_grid = (s ** -2.0 *")],
                   "tests/test_oracle_losses.py", {"test_closed_forms"}),
    "texture_norm": ([("oracle/losses.py", "r = (W[:, :, None] * X).sum(dim=1) / Sd[:, None]",
                       "r = (W[:, :, None] * X).sum(dim=1)")],
                     "tests/test_oracle_losses.py", {"test_texture_loss_is_scale_invariant_in_the_weights"}),
    "fps_ties": ([("oracle/adc.py", "cur = int(np.argmax(best))", "cur = int(len(best) - 1 - np.argmax(best[::-1]))")],
                 "tests/test_oracle_adc.py", {"test_fps_collinear_closed_form"}),
    "draw_key": ([("oracle/adc.py", "key[ok] = (e[ok] / w[ok]).astype(np.float32)",
                   "key[ok] = (w[ok] / e[ok]).astype(np.float32)")],
                 "tests/test_oracle_adc.py", {"test_selection_weights_and_exclusions"}),
    "split_axis": ([("oracle/adc.py", "        if s1 >= s2:\n            half, axis, which = s1 / 2.0, v1[i], 0",
                     "        if s1 < s2:\n            half, axis, which = s1 / 2.0, v1[i], 0")],
                   "tests/test_oracle_adc.py", {"test_split_closed_forms"}),
}


def _run_file(tmp, test_file):
    r = subprocess.run([sys.executable, "-m", "pytest", test_file, "-q", "-p", "no:cacheprovider", "-rf"], cwd=tmp,
                       capture_output=True, text=True, timeout=600)
    failed = {ln.split("::")[1].split(" ")[0] for ln in r.stdout.splitlines() if ln.startswith("FAILED")}
    return r.returncode, failed, r.stdout[-2000:]


def test_unmutated_copy_passes_the_other_pins(tmp_path):
    tmp = str(tmp_path)
    _copy(tmp)
    for f in sorted({v[1] for v in MUTATIONS_2.values()}):
        rc, failed, out = _run_file(tmp, f)
        assert rc == 0 and not failed, out


@pytest.mark.parametrize("name", sorted(MUTATIONS_2))
def test_other_mutation_is_caught(tmp_path, name):
    tmp = str(tmp_path)
    _copy(tmp)
    edits, test_file, expected = MUTATIONS_2[name]
    for rel, old, new in edits:
        p = os.path.join(tmp, rel)
        src = open(p).read()
        assert src.count(old) == 1, f"{rel}: the text to mutate is not there exactly once: {old}"
        open(p, "w").write(src.replace(old, new))
    rc, failed, out = _run_file(tmp, test_file)
    assert rc != 0, f"mutation {name} passed every pin:\n{out}"
    assert expected <= failed, f"mutation {name}: expected {sorted(expected)} to fail, got {sorted(failed)}"
