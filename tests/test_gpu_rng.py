"""The walk's momentum-noise stream on the GPU against the oracle's own
implementation of the same stream: the integer words bit for bit, the FP32
Box-Muller normals within the hardware transcendentals' error."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TAG_EPS = 4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.mark.parametrize("seed,it", [(7, 0), (0xDEADBEEF12345678, 93)])
def test_noise_stream_matches_oracle(torch, orc, seed, it):
    from paper_2312_03911_amd import _lib
    L = _lib.load()
    W, B, T = 5, 3, 9
    n = T * W * B * 4
    z = torch.zeros(n, dtype=torch.float32, device="cuda")
    w = torch.zeros(n, dtype=torch.int32, device="cuda")
    cs = torch.zeros(W * B, dtype=torch.float32, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(L.ggns_noise_normals(seed, it, W, B, T, z.data_ptr(), w.data_ptr(), cs.data_ptr(), s),
               "ggns_noise_normals")
    torch.cuda.synchronize()
    z = z.cpu().numpy().reshape(T, W, B, 4)
    w = w.cpu().numpy().view(np.uint32).reshape(T, W, B, 4)
    cs = cs.cpu().numpy().reshape(W, B)
    for m in range(W):
        for b in range(B):
            state = orc.stream_words(seed, b, m, it, TAG_EPS, 0)
            words = orc.xoshiro_stream(state, 4 * T).reshape(T, 4)
            np.testing.assert_array_equal(w[:, m, b], words)
            ref = np.array([orc.box_muller4(words[t]) for t in range(T)])
            assert np.all(np.abs(z[:, m, b] - ref) <= 2e-5 * (1.0 + np.abs(ref)))
            assert abs(cs[m, b] - ref.sum()) < 1e-3


def test_noise_stream_rejects_bad_sizes(torch):
    from paper_2312_03911_amd import _lib
    L = _lib.load()
    assert L.ggns_noise_normals(1, 0, -1, 1, 1, None, None, None, None) == _lib.GGNS_EINVAL
    assert L.ggns_noise_normals(1, 0, 1 << 20, 1 << 11, 1, None, None, None, None) == _lib.GGNS_EINVAL
    assert L.ggns_noise_normals(1, 0, 0, 4, 10, None, None, None, None) == _lib.GGNS_OK
