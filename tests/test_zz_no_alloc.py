"""The allocation-free variant of the relative L1 sample error
(mclbm_sample_error_noalloc), called through the C ABI, against the variant
with a caller-provided work buffer (mclbm_sample_error): bit-equal results
on two calls in a row, the second with fewer samples (the scratch array of
the library keeps the first call's contents), and its size limit."""
import ctypes

import numpy as np
import pytest
import torch

import mc_inputs

pytestmark = pytest.mark.gpu
mc = pytest.importorskip("paper_2608_23786_amd")
from paper_2608_23786_amd import _lib  # noqa: E402


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(a, b, q, stream):
    m = a.shape[0]
    L = _lib.lib()
    ref = torch.empty(4, dtype=torch.float64, device="cuda")
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    wb = int(L.mclbm_sample_error_work_bytes(m))
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    s = ctypes.c_void_p(stream.cuda_stream)
    _lib.check(L.mclbm_sample_error(_p(a), _p(b), m, q, _p(ref), _p(work), wb, s))
    _lib.check(L.mclbm_sample_error_noalloc(_p(a), _p(b), m, q, _p(out), s))
    stream.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_sample_error_matches_the_work_buffer_variant():
    stream = torch.cuda.Stream()
    q = 8
    for m, seed in ((1000, 5), (37, 6)):
        a = torch.from_numpy(mc_inputs.random_populations(seed, (m, 3, q ** 3), 1.0)).cuda()
        b = torch.from_numpy(mc_inputs.random_populations(seed + 100, (m, 3, q ** 3), 1.0)).cuda()
        torch.cuda.synchronize()
        ref, out = _both(a, b, q, stream)
        print(m, ref, out)
        assert np.all(np.isfinite(ref)) and np.array_equal(ref, out)


def test_noalloc_sample_error_limits():
    L = _lib.lib()
    a = torch.zeros((2, 3, 8), dtype=torch.float64, device="cuda")
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    st = L.mclbm_sample_error_noalloc(_p(a), _p(a), 65537, 2, _p(out), None)
    assert st == _lib.ERR_ARG and b"65536" in L.mclbm_last_error()
    assert L.mclbm_sample_error_noalloc(None, _p(a), 2, 2, _p(out), None) == _lib.ERR_ARG
