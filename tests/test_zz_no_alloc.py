"""dmrg_block_gemm_noalloc (descriptors in the library's fixed device array)
against dmrg_block_gemm (descriptors in memory allocated per call): identical
results on two calls in a row, the second smaller than the first, so stale
descriptors of the first call would show; sizes beyond the array are refused."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run(pk, fn, prec, mode, A, B, M, N, K, coef, stream):
    import torch
    dt = torch.float64 if prec == 0 else torch.float32
    dA = torch.from_numpy(A).to(dt).cuda()
    dB = torch.from_numpy(B).to(dt).cuda()
    dC = torch.full((M, N), float("nan"), dtype=dt, device="cuda")
    code = fn(prec, mode, M, N, K, ctypes.c_void_p(dA.data_ptr()), A.shape[1], ctypes.c_void_p(dB.data_ptr()),
              B.shape[1], ctypes.c_void_p(dC.data_ptr()), N, coef, ctypes.c_void_p(stream))
    assert code == 0, pk.dmrg_last_error()
    torch.cuda.current_stream().synchronize()
    return dC.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_noalloc_matches_allocating_entry_two_calls(prec, mode):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_09990_amd as pk
    stream = torch.cuda.current_stream().cuda_stream
    # first call covers 3 x 4 tiles, the second 1 x 2: it must not pick up the
    # first call's extra tile descriptors
    for call, (M, N, K) in enumerate([(150, 230, 77), (37, 70, 23)]):
        rng = np.random.default_rng(100 * call + 10 * mode + prec)
        A = rng.standard_normal((K, M) if mode == 2 else (M, K))
        B = rng.standard_normal((N, K) if mode == 1 else (K, N))
        coef = -0.5 - call
        ref = _run(pk, pk.dmrg_block_gemm, prec, mode, A, B, M, N, K, coef, stream)
        got = _run(pk, pk.dmrg_block_gemm_noalloc, prec, mode, A, B, M, N, K, coef, stream)
        assert np.all(np.isfinite(got)), f"call {call}: unwritten output elements"
        # the same kernel on the same tile table: bitwise equal
        assert np.array_equal(got, ref), f"call {call}: max diff {np.max(np.abs(got - ref))}"
        # and both against numpy (as the allocating entry's own test does)
        Ar = A.T if mode == 2 else A
        Br = B.T if mode == 1 else B
        exact = coef * (Ar @ Br)
        tol = 1e-13 if prec == 0 else 1e-5
        assert np.max(np.abs(got - exact)) / max(1.0, np.max(np.abs(exact))) < tol * np.sqrt(K)


def test_noalloc_refuses_oversized_output():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_09990_amd as pk
    d = torch.zeros(8, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(d.data_ptr())
    # 4097 x 4097 needs 65 x 65 tiles > 4096: refused on the host before any launch
    code = pk.dmrg_block_gemm_noalloc(0, 0, 4097, 4097, 1, p, 1, p, 4097, p, 4097, 1.0,
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code == -1
    assert b"allocation-free" in pk.dmrg_last_error()
