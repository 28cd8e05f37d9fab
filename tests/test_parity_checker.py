"""The two-stage comparison used by the GPU parity tests, checked on the CPU: the oracle's own
output rounded to float32 passes, and a planted error of each kind fails at the stage meant to
catch it (G-buffer and alpha at stage 1, shading at stage 2), while the grazing exemption
lifts only the G-buffer bar."""
import numpy as np
import pytest

import oracle
import synth
from parity import e2e_bound, pixel_match


@pytest.fixture(scope="module")
def case():
    sc = synth.make_scene("shell2k", n=300)
    cam = synth.crop_camera(synth.config_cameras("shell2k")[0], 40, 40, 24, 24)
    pix = oracle.all_pixels(24, 24)
    ref = oracle.render(sc, cam, pixels=pix)
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    rgba = ref["rgba"].astype(np.float32).astype(np.float64)
    gbuf = ref["gbuf"].astype(np.float32).astype(np.float64)
    covered = np.nonzero((ref["rgba"][:, 3] > 0.2) & (ref["stat"][:, 2] == 0))[0]
    assert len(covered) > 20
    return cam, pix, ref, tabs, rgba, gbuf, covered


def test_oracle_values_pass(case):
    cam, pix, ref, tabs, rgba, gbuf, _ = case
    ok, info = pixel_match(rgba, gbuf, ref, cam, pix, tabs)
    assert ok.all(), info
    assert info["e2e_over_1e-4"] == 0 and e2e_bound(info)


def test_planted_shading_error_fails_stage_two(case):
    cam, pix, ref, tabs, rgba, gbuf, covered = case
    k = covered[3]
    bad = rgba.copy()
    bad[k, 1] += 2e-4
    ok, info = pixel_match(bad, gbuf, ref, cam, pix, tabs)
    assert info["fail_shade"] == 1 and info["fail_blend"] == 0 and not ok[k]
    assert info["e2e_over_1e-4"] == 1


def test_planted_gbuffer_and_alpha_errors_fail_stage_one(case):
    cam, pix, ref, tabs, rgba, gbuf, covered = case
    k = covered[5]
    for ch in (0, 3, 4, 6):
        bad = gbuf.copy()
        bad[k, ch] += 3e-5
        ok, info = pixel_match(rgba, bad, ref, cam, pix, tabs, check_rgb=False)
        assert info["fail_blend"] == 1 and not ok[k], ch
    bad = rgba.copy()
    bad[k, 3] += 2e-5
    ok, info = pixel_match(bad, gbuf, ref, cam, pix, tabs, check_rgb=False)
    assert info["fail_blend"] == 1 and not ok[k]


def test_grazing_exemption_lifts_only_the_gbuffer_bar(case):
    cam, pix, ref, tabs, rgba, gbuf, covered = case
    k = covered[7]
    r2 = dict(ref)
    r2["stat"] = ref["stat"].copy()
    r2["stat"][k, 3] = 1.0                      # flagged grazing
    bad = gbuf.copy()
    bad[k, 5] += 3e-5
    ok, info = pixel_match(rgba, bad, r2, cam, pix, tabs, check_rgb=False, skip_graze=True)
    assert ok[k] and info["grazing_off_gbuf_bar"] == 1
    bad_a = rgba.copy()
    bad_a[k, 3] += 2e-5
    ok, _ = pixel_match(bad_a, gbuf, r2, cam, pix, tabs, check_rgb=False, skip_graze=True)
    assert not ok[k]
    bad_c = rgba.copy()
    bad_c[k, 0] += 2e-4
    ok, _ = pixel_match(bad_c, gbuf, r2, cam, pix, tabs, skip_graze=True)
    assert not ok[k]


def test_end_to_end_count_bar(case):
    cam, pix, ref, tabs, rgba, gbuf, covered = case
    bad = rgba.copy()
    n = int(0.02 * len(pix)) + 3
    bad[covered[:n], 2] += 5e-4
    _, info = pixel_match(bad, gbuf, ref, cam, pix, tabs)
    assert info["e2e_over_1e-4"] == min(n, len(covered)) and not e2e_bound(info)
