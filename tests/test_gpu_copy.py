"""The streaming copy the bench uses as its bandwidth ceiling: bit-exact on
aligned and unaligned pointers, odd lengths and empty input."""
import numpy as np
import pytest

from gpu_util import announce, bits, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,offset", [(1, 0), (2, 0), (1023, 0), (1 << 20, 0), ((1 << 20) + 3, 1), (4097, 1)])
def test_copy_exact(n, offset):
    torch = need_gpu()
    import paper_2402_01816_amd as gs
    announce("copy", n, offset)
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n + offset)
    x[::97] = np.nan
    src = torch.from_numpy(x).to("cuda")[offset:]
    dst = torch.full((n + offset,), 7.0, dtype=torch.float64, device="cuda")[offset:]
    gs.gs_copy_f64(src, dst)
    torch.cuda.synchronize()
    assert np.array_equal(bits(dst), bits(src))


def test_copy_empty():
    torch = need_gpu()
    import paper_2402_01816_amd as gs
    a = torch.empty(0, dtype=torch.float64, device="cuda")
    gs.gs_copy_f64(a, a)
