"""CPU tier of the C ABI: the library loads, exports every entry point that include/gs4d.h
declares, and rejects invalid arguments on the host before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2509_17513_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 7
    for nm in names:
        assert hasattr(L, nm), nm


def _settings(n, w=64, h=48, deg=0):
    from paper_2509_17513_amd import RenderSettings
    return RenderSettings(w, h, deg, (n,), (1.0,)).c_struct(n)


def test_workspace_size_and_validation(L):
    sz = ctypes.c_size_t()
    s = _settings(1000)
    assert L.gs_workspace_size(ctypes.byref(s), 1000, 1, 2, 10000, ctypes.byref(sz)) == 0
    assert sz.value > 10000 * 4
    # bigger capacity -> 8 bytes per pair more (tile list 4 B + row list 4 B, after 256-byte alignment)
    sz2 = ctypes.c_size_t()
    assert L.gs_workspace_size(ctypes.byref(s), 1000, 1, 2, 10000 + 64 * 10, ctypes.byref(sz2)) == 0
    assert sz2.value - sz.value == 5120
    bad = [
        (_settings(1000), -1, 1, 1, 10),
        (_settings(1000), 1000, 0, 1, 10),
        (_settings(1000), 999, 1, 1, 10),       # last level count != n
        (_settings(1000, deg=4), 1000, 1, 1, 10),
        (_settings(1000, w=0), 1000, 1, 1, 10),
        (_settings(1000), 1000, 1, 1, -5),
    ]
    for st, n, F, V, cap in bad:
        assert L.gs_workspace_size(ctypes.byref(st), n, F, V, cap, ctypes.byref(sz)) == -1
    st = _settings(1000)
    st.level_counts[0] = 5
    st.n_levels = 2
    st.level_counts[1] = 4  # not ascending
    assert L.gs_workspace_size(ctypes.byref(st), 1000, 1, 1, 10, ctypes.byref(sz)) == -1
    st = _settings(1000)
    st.res_channels = 9
    assert L.gs_workspace_size(ctypes.byref(st), 1000, 1, 1, 10, ctypes.byref(sz)) == -1
    st = _settings(1000)
    st.tile_w = st.tile_h = 8
    assert L.gs_workspace_size(ctypes.byref(st), 1000, 1, 1, 10, ctypes.byref(sz)) == -6
    # alpha_max = 1 is rejected whatever t_stop is: the backward divides by 1 - alpha
    for t_stop in (0.0, 1e-4):
        st = _settings(1000)
        st.alpha_max, st.t_stop = 1.0, t_stop
        assert L.gs_workspace_size(ctypes.byref(st), 1000, 1, 1, 10, ctypes.byref(sz)) == -1
    st = _settings(1000)
    st.alpha_max = 0.999
    assert L.gs_workspace_size(ctypes.byref(st), 1000, 1, 1, 10, ctypes.byref(sz)) == 0
    assert L.gs_error_string(-3) == b"pair list capacity exceeded"
    # launch shapes: only the listed values, and the workspace does not depend on them
    for field, value in (("bin_chunk", 300), ("bin_chunk", 4096), ("row_seg", 512), ("wave_layout", 3),
                         ("lds_batch", 100), ("lds_batch", 512), ("bwd_pixels", 3)):
        st = _settings(1000)
        setattr(st, field, value)
        assert L.gs_workspace_size(ctypes.byref(st), 1000, 1, 2, 10000, ctypes.byref(sz2)) == -1, (field, value)
    ref = ctypes.c_size_t()
    st = _settings(1000)
    assert L.gs_workspace_size(ctypes.byref(st), 1000, 1, 2, 10000, ctypes.byref(ref)) == 0
    for bc, rs, wl, lb in ((512, 1024, 1, 64), (2048, 4096, 2, 128), (1024, 2048, 0, 256)):
        st = _settings(1000)
        st.bin_chunk, st.row_seg, st.wave_layout, st.lds_batch = bc, rs, wl, lb
        assert L.gs_workspace_size(ctypes.byref(st), 1000, 1, 2, 10000, ctypes.byref(sz2)) == 0
        assert sz2.value == ref.value


def test_render_calls_reject_bad_args_before_launch(L):
    s = _settings(10)
    P = ctypes.c_void_p
    # NULL image
    assert L.gs_render_forward(ctypes.byref(s), 10, P(8), 1, None, 1, P(8), None, P(8), 1 << 20, None) == -1
    # workspace too small
    assert L.gs_render_forward(ctypes.byref(s), 10, P(8), 1, None, 1, P(8), P(8), P(8), 16, None) == -2
    # backward needs exactly one of d_image / target
    assert L.gs_render_backward(ctypes.byref(s), 10, P(8), 1, None, 1, P(8), None, None, None, P(8), None, None,
                                P(8), 1 << 20, None) == -1
    # residuals without res_channels
    assert L.gs_render_forward(ctypes.byref(s), 10, P(8), 1, P(8), 1, P(8), P(8), P(8), 1 << 20, None) == -1


def test_color_loss_workspace_and_validation(L):
    P = ctypes.c_void_p
    sz = ctypes.c_size_t()
    s = _settings(10, w=150, h=70)
    s.n_levels = 3
    for l in range(3):
        s.level_counts[l] = 10
    # three floats per image element, whatever the shapes of the render
    assert L.gs_color_loss_workspace_size(ctypes.byref(s), 2, 3, ctypes.byref(sz)) == 0
    assert sz.value == 3 * 4 * (6 * 3 * 3 * 150 * 70)
    assert L.gs_color_loss_workspace_size(None, 1, 1, ctypes.byref(sz)) == -1
    assert L.gs_color_loss_workspace_size(ctypes.byref(s), 0, 1, ctypes.byref(sz)) == -1
    s0 = _settings(10, w=0)
    assert L.gs_color_loss_workspace_size(ctypes.byref(s0), 1, 1, ctypes.byref(sz)) == -1
    big = 1 << 30
    # NULL image / target, nothing to compute, lambda outside [0, 1], no or too small workspace
    assert L.gs_color_loss(ctypes.byref(s), 1, 1, None, P(8), 0.2, P(8), P(8), P(8), big, None) == -1
    assert L.gs_color_loss(ctypes.byref(s), 1, 1, P(8), None, 0.2, P(8), P(8), P(8), big, None) == -1
    assert L.gs_color_loss(ctypes.byref(s), 1, 1, P(8), P(8), 0.2, None, None, P(8), big, None) == -1
    for lam in (-0.1, 1.5, float("nan")):
        assert L.gs_color_loss(ctypes.byref(s), 1, 1, P(8), P(8), lam, P(8), P(8), P(8), big, None) == -1
    assert L.gs_color_loss(ctypes.byref(s), 1, 1, P(8), P(8), 0.2, P(8), P(8), None, big, None) == -1
    assert L.gs_color_loss(ctypes.byref(s), 1, 1, P(8), P(8), 0.2, P(8), P(8), P(8), 16, None) == -2


def test_workspace_layout_regions_are_disjoint(L):
    from paper_2509_17513_amd._lib import GsWorkspaceLayout
    s = _settings(5000, 200, 120, 3)
    lo = GsWorkspaceLayout()
    assert L.gs_workspace_describe(ctypes.byref(s), 5000, 2, 3, 123456, ctypes.byref(lo)) == 0
    offs = [lo.status, lo.records, lo.rects, lo.keys, lo.vals, lo.ranges, lo.t_final, lo.n_last, lo.grad2d,
            lo.lists]
    assert lo.lists + 4 * 123456 + 8 * (123456 // 2) <= lo.total
    assert offs == sorted(offs) and len(set(offs)) == len(offs)
    assert lo.tiles_x == 13 and lo.tiles_y == 8


def test_maps_describe_matches_the_layout_rule_and_validates(L):
    from oracle import bitstream as BS
    from paper_2509_17513_amd._lib import GsMapsLayout
    lv = [300, 300, 900, 3000]  # an empty second layer
    arr = (ctypes.c_int32 * 8)(*lv)
    lo = GsMapsLayout()
    assert L.gs_maps_describe(14, 4, arr, ctypes.byref(lo)) == 0
    prev = 0
    end = 0
    for l, c in enumerate(lv):
        assert (lo.width[l], lo.height[l]) == BS.map_size(c - prev), l
        assert lo.offset[l] >= end and lo.offset[l] % 256 == 0
        end = lo.offset[l] + lo.width[l] * lo.height[l] * (6 + 11)
        prev = c
    assert lo.total_bytes >= end
    bad = (ctypes.c_int32 * 8)(300, 200, 900)
    assert L.gs_maps_describe(14, 3, bad, ctypes.byref(lo)) == -1
    assert L.gs_maps_describe(10, 3, arr, ctypes.byref(lo)) == -1
    assert L.gs_maps_describe(14, 9, arr, ctypes.byref(lo)) == -1
    # encode re-validates a layout that does not hold its layers, before any device work
    assert L.gs_maps_describe(14, 4, arr, ctypes.byref(lo)) == 0
    lo.width[3] = 16
    sz = ctypes.c_size_t()
    assert L.gs_encode_workspace_size(ctypes.byref(lo), ctypes.byref(sz)) == -1
    P = ctypes.c_void_p
    assert L.gs_significance_order(-1, P(8), 14, 1e5, P(8), None, P(8), 1 << 20, None) == -1
    assert L.gs_significance_order(10, P(8), 14, float("inf"), P(8), None, P(8), 1 << 20, None) == -1
    assert L.gs_significance_order(10, P(8), 14, 1e5, P(8), None, P(8), 16, None) == -2


def test_package_modules_import():
    import importlib
    for m in ("render", "train", "bitstream", "entropy", "motion", "_lib"):
        importlib.import_module(f"paper_2509_17513_amd.{m}")


def test_work_counter_switch_is_host_only_and_returns_previous(L):
    prev = L.gs_set_work_counters(1)
    try:
        assert L.gs_set_work_counters(0) == 1
        assert L.gs_set_work_counters(0) == 0
        assert L.gs_set_work_counters(5) == 0
        assert L.gs_set_work_counters(0) == 1
    finally:
        L.gs_set_work_counters(prev)


def test_deterministic_switch_sizes_the_workspace_for_its_fixed_point_sums(L):
    """The deterministic backward's switch is host-only, returns the previous setting, and while it
    is on the workspace holds 144 more bytes (nine 128-bit sums) per (view, Gaussian)."""
    from paper_2509_17513_amd import RenderSettings
    st = RenderSettings(64, 48, 1, (100,), (1.0,)).c_struct(100)
    size = ctypes.c_size_t()
    assert L.gs_workspace_size(ctypes.byref(st), 100, 1, 3, 1000, ctypes.byref(size)) == 0
    base = size.value
    prev = L.gs_set_deterministic(1)
    try:
        assert L.gs_set_deterministic(1) == 1
        assert L.gs_workspace_size(ctypes.byref(st), 100, 1, 3, 1000, ctypes.byref(size)) == 0
        assert size.value >= base + 3 * 100 * 144 + 16
        assert size.value <= base + 3 * 100 * 144 + 16 + 512  # two 256-byte alignments
        assert L.gs_set_deterministic(0) == 1
        assert L.gs_workspace_size(ctypes.byref(st), 100, 1, 3, 1000, ctypes.byref(size)) == 0
        assert size.value == base
    finally:
        L.gs_set_deterministic(prev)


def test_render_backward_checks_every_shape_on_the_host():
    """The C ABI cannot see a tensor's extent, so the binding checks the shape of every buffer
    render_backward passes: a d_image shaped like the target, a narrower d_params or a wrong
    residual block would be read or written out of bounds by the kernels."""
    import torch

    from paper_2509_17513_amd import RenderSettings, render_backward
    n, W, H, L, V = 50, 32, 24, 3, 2
    st = RenderSettings(W, H, 0, (10, 30, 50), (0.5, 0.25, 1.0))
    p = torch.zeros((14, n))
    cams = torch.zeros((V, 16))
    good_img = torch.zeros((1, V, L, 3, H, W))
    cases = [
        dict(image=good_img, d_image=torch.zeros((V, 3, H, W))),                  # d_image shaped like the target
        dict(image=torch.zeros((1, V, 1, 3, H, W)), target=torch.zeros((V, 3, H, W))),  # image with one layer
        dict(image=good_img, target=torch.zeros((1, 3, H, W))),                    # target of one view
        dict(image=good_img, target=torch.zeros((V, 3, H, W)), d_params=torch.zeros((14, n - 1))),
        dict(image=good_img, target=torch.zeros((V, 3, H, W)), loss=torch.zeros(0)),
    ]
    for kw in cases:
        with pytest.raises(ValueError, match="shape|elements"):
            render_backward(st, p, cams, None, **kw)
    st8 = RenderSettings(W, H, 0, (10, 30, 50), (0.5, 0.25, 1.0), res_channels=8)
    with pytest.raises(ValueError, match="shape"):
        render_backward(st8, p, cams, None, 1, torch.zeros((1, 8, n)), image=good_img,
                        target=torch.zeros((V, 3, H, W)), d_residuals=torch.zeros((1, 7, n)))
    with pytest.raises(ValueError, match=r"params must be"):
        render_backward(st, torch.zeros((13, n)), cams, None, image=good_img, target=torch.zeros((V, 3, H, W)))
