"""The allocation-free Gram entry point (pase_gram_noalloc) against the handle-based
pase_gram, both called through the C ABI: two calls in a row, the second on a smaller input,
so a result that depended on what the first call left in the library's scratch array would
show.  Bitwise equal where both use the same row blocks (k <= 64), to rounding otherwise."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("k, N1, N2", [(50, 250047, 3375), (64, 100000, 777), (100, 250047, 12345),
                                       (128, 70000, 5000)])
def test_gram_noalloc_matches_pase_gram(k, N1, N2):
    _gpu()
    from paper_2502_04589_amd import Solver
    from paper_2502_04589_amd import _native as nat

    lib = nat.load()
    s = Solver(3, [64, 32, 16, 8], nev_max=max(k, 4))
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = torch.Generator().manual_seed(7)
    for N in (N1, N2):
        print(f"gram_noalloc k={k} N={N}", flush=True)
        X = torch.rand((N, k), generator=g, dtype=torch.float64).mul_(2).sub_(1).cuda()
        Y = torch.rand((N, k), generator=g, dtype=torch.float64).mul_(2).sub_(1).cuda()
        G = torch.full((k, k), np.nan, dtype=torch.float64, device="cuda")
        st = lib.pase_gram_noalloc(N, k, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                                   C.c_void_p(G.data_ptr()), stream)
        assert st == 0, lib.pase_last_error(None)
        torch.cuda.synchronize()
        ref = s.gram(X, Y).cpu().numpy()
        got = G.cpu().numpy()
        if k <= 64:
            assert np.array_equal(got, ref)
        else:
            scale = np.abs(X.cpu().numpy()).T @ np.abs(Y.cpu().numpy())
            assert np.max(np.abs(got - ref) / scale) < 1e-14
        # and against the plain definition
        exact = X.cpu().numpy().T @ Y.cpu().numpy()
        assert np.max(np.abs(got - exact)) < 1e-12 * np.max(np.abs(exact)) + 1e-12


def test_gram_noalloc_rejects_bad_sizes():
    _gpu()
    from paper_2502_04589_amd import _native as nat

    lib = nat.load()
    X = torch.zeros((10, 129), dtype=torch.float64, device="cuda")
    G = torch.zeros((129, 129), dtype=torch.float64, device="cuda")
    p = C.c_void_p(X.data_ptr())
    assert lib.pase_gram_noalloc(10, 129, p, p, C.c_void_p(G.data_ptr()), None) == 1
    assert b"k must be" in lib.pase_last_error(None)
    assert lib.pase_gram_noalloc(0, 8, p, p, C.c_void_p(G.data_ptr()), None) == 1
    assert lib.pase_gram_noalloc(10, 8, None, p, C.c_void_p(G.data_ptr()), None) == 1
