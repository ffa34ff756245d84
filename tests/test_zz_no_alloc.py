"""The allocation-free maxabs entry point against the scratch-buffer one.

hgs_nn_maxabs_noalloc keeps its per-chunk partials in a static device array
of the library instead of a caller's scratch buffer.  It is called through
the C ABI twice in a row, the second time with a smaller input, so that the
second call runs over partials the first one left behind; max is exact, so
both calls must equal hgs_nn_maxabs bit for bit.  Sizes beyond the array are
refused on the host before anything is launched.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _maxabs_pair(hgs, x):
    import torch

    L = hgs.library()
    B = x.shape[0]
    nvox = x[0].numel()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ref = torch.full((B,), -1.0, dtype=torch.float32, device=x.device)
    got = torch.full((B,), -2.0, dtype=torch.float32, device=x.device)
    scratch = torch.empty(B * hgs.NN_MAXABS_CHUNKS, dtype=torch.float32, device=x.device)
    assert L.hgs_nn_maxabs(x.data_ptr(), B, nvox, ref.data_ptr(), scratch.data_ptr(), st) == hgs.HGS_OK
    assert L.hgs_nn_maxabs_noalloc(x.data_ptr(), B, nvox, got.data_ptr(), st) == hgs.HGS_OK, \
        L.hgs_nn_last_error()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_maxabs_matches_scratch_version_twice(gpu_lib):
    import torch

    rng = np.random.default_rng(71)
    # first call: many samples with a ragged voxel count; second: fewer and
    # smaller samples, so most partials of the array still hold the first
    # call's (larger) values
    for B, shape in ((37, (13, 11, 29)), (5, (3, 7, 9))):
        a = rng.normal(0.0, 1.0, (B,) + shape).astype(np.float32)
        a[0, 1, 2, 3] = 40.0 if B == 37 else 0.5  # a peak in one sample
        x = torch.from_numpy(a).to("cuda")
        ref, got = _maxabs_pair(gpu_lib, x)
        want = np.max(np.abs(a.reshape(B, -1)), axis=1)
        assert np.array_equal(ref, want)
        assert np.array_equal(got, ref), (got, ref)


def test_noalloc_maxabs_at_the_size_limit_and_beyond(gpu_lib):
    import torch

    L = gpu_lib.library()
    B = gpu_lib.NN_MAXABS_NOALLOC_MAX_B
    x = torch.randn(B, 70, dtype=torch.float32, device="cuda")
    ref, got = _maxabs_pair(gpu_lib, x)
    assert np.array_equal(got, ref)
    out = torch.empty(B + 1, dtype=torch.float32, device="cuda")
    big = torch.zeros(B + 1, 4, dtype=torch.float32, device="cuda")
    assert L.hgs_nn_maxabs_noalloc(big.data_ptr(), B + 1, 4, out.data_ptr(), None) == gpu_lib.HGS_ERR_ARG
    assert b"static scratch" in L.hgs_nn_last_error()
    assert L.hgs_nn_maxabs_noalloc(None, 1, 4, out.data_ptr(), None) == gpu_lib.HGS_ERR_ARG
