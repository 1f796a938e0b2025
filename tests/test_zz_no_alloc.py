"""gs_rate_histogram_noalloc (the histogram rate on the library's fixed scratch, for callers that
cannot allocate) against gs_rate_histogram (the same kernels on a caller's workspace), through
the C ABI: bit-identical bits on two calls in a row, the second with a smaller input, so the
scratch left by the first call must not leak into the second."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _with_workspace(L, attrs, step):
    A, n = attrs.shape
    sz = ctypes.c_size_t()
    assert L.gs_rate_histogram_workspace_size(A, ctypes.byref(sz)) == 0
    ws = torch.empty(sz.value, dtype=torch.uint8, device=attrs.device)
    bits = torch.zeros(A, dtype=torch.float64, device=attrs.device)
    assert L.gs_rate_histogram(n, A, _p(attrs), ctypes.c_float(step), _p(bits), _p(ws), sz.value, _stream()) == 0
    torch.cuda.synchronize()
    return bits.cpu().numpy()


def test_noalloc_histogram_matches_workspace_entry_point_on_two_calls():
    from paper_2509_17513_amd import _lib
    L = _lib.lib()
    dev = torch.device("cuda:0")
    step = 1.0 / 64
    cases = [(200_000, 56, 5), (3_001, 20, 6)]  # the second is smaller in both n and attributes
    for n, A, seed in cases:
        print(f"\n[case] noalloc histogram n={n} n_attr={A} seed={seed}", flush=True)
        p = synth.cube_scene(n, seed, 3)
        attrs = torch.from_numpy(np.ascontiguousarray(p[3:3 + A])).to(dev)
        ref = _with_workspace(L, attrs, step)
        bits = torch.full((A,), -1.0, dtype=torch.float64, device=dev)
        assert L.gs_rate_histogram_noalloc(n, A, _p(attrs), ctypes.c_float(step), _p(bits), _stream()) == 0
        torch.cuda.synchronize()
        got = bits.cpu().numpy()
        assert np.array_equal(got, ref), np.abs(got - ref).max()
        assert np.all(got > 0)


def test_noalloc_histogram_rejects_too_many_attributes_and_bad_args():
    from paper_2509_17513_amd import _lib
    L = _lib.lib()
    P = ctypes.c_void_p
    s = ctypes.c_float(1.0 / 64)
    assert L.gs_rate_histogram_noalloc(10, 65, P(8), s, P(8), None) == -1   # beyond the scratch's 64 attributes
    assert L.gs_rate_histogram_noalloc(10, 0, P(8), s, P(8), None) == -1
    assert L.gs_rate_histogram_noalloc(-1, 4, P(8), s, P(8), None) == -1
    assert L.gs_rate_histogram_noalloc(10, 4, None, s, P(8), None) == -1
    assert L.gs_rate_histogram_noalloc(10, 4, P(8), ctypes.c_float(0.0), P(8), None) == -1
