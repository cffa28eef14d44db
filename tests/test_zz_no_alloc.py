"""kpm_dot_noalloc (partials in the library's static per-GPU array) against kpm_dot
(partials in a buffer allocated per stream), both called through the C ABI."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_1410_5242_amd import kpm

pytestmark = pytest.mark.gpu

DT = {"c128": (0, np.complex128), "c64": (1, np.complex64)}


def say(*a):
    print("[no-alloc]", *a, flush=True)


def _vec(n, seed, dtype):
    rng = np.random.default_rng(seed)
    v = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(max(n, 1))
    return v.astype(dtype)


def _call(fn, code, x, y, out):
    st = fn(code, x.numel(), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, kpm.lib().kpm_last_error().decode()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("same", [False, True])
def test_dot_noalloc_matches_dot_on_two_calls(dtype, same):
    L = kpm.lib()
    L.kpm_last_error.restype = ctypes.c_char_p
    code, npdt = DT[dtype]
    # first call: more 16-byte units than 2048 workgroups of 256 lanes cover (every
    # partial slot written); second call: a smaller, odd length (scalar tail)
    for n, seed in ((3_000_001, 1), (1_001, 2)):
        say(dtype, "same" if same else "x,y", "n", n)
        xh = _vec(n, seed, npdt)
        yh = xh if same else _vec(n, seed + 10, npdt)
        x = torch.from_numpy(xh).cuda()
        y = x if same else torch.from_numpy(yh).cuda()
        got = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
        ref = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
        _call(L.kpm_dot_noalloc, code, x, y, got)
        _call(L.kpm_dot, code, x, y, ref)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        # same kernels, same grid, same order: equal bit for bit
        assert np.array_equal(g, r), (g, r)
        # and the sum itself against the oracle's pairwise FP64 sum of the same elements
        o = O.block_dot(xh.astype(np.complex128), yh.astype(np.complex128))[0]
        assert abs(complex(g[0], g[1]) - o) <= 1e-13, (g, o)
        if same:
            assert g[1] == 0.0


def test_dot_noalloc_empty_and_errors():
    L = kpm.lib()
    x = torch.zeros(4, dtype=torch.complex128, device="cuda")
    out = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
    st = L.kpm_dot_noalloc(0, 0, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                           ctypes.c_void_p(out.data_ptr()), None)
    assert st == 0
    torch.cuda.synchronize()
    assert out.cpu().numpy().tolist() == [0.0, 0.0]
    assert L.kpm_dot_noalloc(2, 4, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                             ctypes.c_void_p(out.data_ptr()), None) == kpm.KPM_EINVAL
    assert L.kpm_dot_noalloc(0, 4, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                             None, None) == kpm.KPM_EINVAL
