"""adr_dot_noalloc (include/adr.h): the inner product for callers that cannot
allocate, called through the C ABI, against adr_dot on the same inputs --
bit for bit (the same kernels and the same double-double reduction) -- on
two calls in a row, the second with a smaller input, plus its size limits."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    import paper_1308_5215_amd  # noqa: F401
    from paper_1308_5215_amd import _lib
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return _lib


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def dot_noalloc(lib, x, y, n=None):
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.load().adr_dot_noalloc(ptr(x), ptr(y), x.numel() if n is None else n, stream, ptr(out))
    torch.cuda.synchronize()
    return st, out.item()


def dot_ref(lib, x, y):
    res = ctypes.c_double(0.0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.load().adr_dot(ptr(x), ptr(y), x.numel(), stream, ctypes.byref(res)) == lib.OK
    return res.value


def test_dot_noalloc_equals_dot_on_two_calls(lib):
    rng = np.random.default_rng(11)
    for n in ((1 << 22) + 13, 1000):      # the second call is smaller: no stale partial sums
        x = torch.from_numpy(rng.standard_normal(n) * 10.0 ** rng.integers(-5, 5, n)).cuda()
        y = torch.from_numpy(rng.standard_normal(n)).cuda()
        st, got = dot_noalloc(lib, x, y)
        print("n %d: %r vs %r" % (n, got, dot_ref(lib, x, y)), flush=True)
        assert st == lib.OK
        assert got == dot_ref(lib, x, y)


def test_dot_noalloc_limits(lib):
    x = torch.ones(8, dtype=torch.float64, device="cuda")
    st, got = dot_noalloc(lib, x, x, n=0)
    assert st == lib.OK and got == 0.0
    st, got = dot_noalloc(lib, x, x, n=1)
    assert st == lib.OK and got == 1.0
    st, _ = dot_noalloc(lib, x, x, n=1 << 31)
    assert st == lib.ERR_ARG and b"2^31" in lib.load().adr_last_error()
    st, _ = dot_noalloc(lib, x, x, n=-1)
    assert st == lib.ERR_ARG
