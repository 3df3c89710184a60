"""The device-rate probes compute what they are declared to compute: the FMA
chains bitwise against their FP32 recurrence, the MFMA accumulations against
their closed form (each entry gains 32 a b per round)."""
import numpy as np
import pytest

from paper_2312_03911_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _run(torch, fn, blocks, iters, a, b):
    import ctypes as C
    out = torch.full((blocks * 256,), float("nan"), dtype=torch.float32, device="cuda:0")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert fn(blocks, iters, a, b, out.data_ptr(), s) == 0
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("iters", [0, 1, 37, 300])
def test_valu_probe_matches_its_recurrence(torch, iters):
    """v <- fma(v, 1/2, 1/4) from v = (lane mod 64)/64 + chain: v/2 is exact in
    FP32, so the fused and the two-step forms round alike."""
    L = _lib.load()
    got = _run(torch, L.ggns_probe_valu, 3, iters, 0.5, 0.25)
    lane = (np.arange(3 * 256) % 256) % 64
    v = [np.float32(lane * 0.015625 + k).astype(np.float32) for k in range(8)]
    half, quarter = np.float32(0.5), np.float32(0.25)
    for _ in range(iters):
        v = [(x * half + quarter).astype(np.float32) for x in v]
    want = np.zeros(3 * 256, dtype=np.float32)
    for x in v:
        want = (want + x).astype(np.float32)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("a,b,iters", [(1.0, 1.0, 0), (1.0, 1.0, 1000), (0.5, 3.0, 200)])
def test_mfma_probe_matches_closed_form(torch, a, b, iters):
    """Four accumulators of four entries per lane, each gaining 32 a b per
    round: every thread's sum is 512 a b iters (exact at these sizes)."""
    L = _lib.load()
    got = _run(torch, L.ggns_probe_mfma, 2, iters, a, b)
    np.testing.assert_array_equal(got, np.full(2 * 256, 512.0 * a * b * iters, dtype=np.float32))
