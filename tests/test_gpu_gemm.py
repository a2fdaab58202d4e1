"""The block-GEMM engine (MFMA fp64 / fp32 / bf16) against numpy, ragged sizes."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _bf16_bits(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16  # round to nearest even
    return u.astype(np.uint16)


def _bf16_val(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 4), (37, 70, 23), (100, 3, 129), (64, 64, 16),
                                   (130, 65, 2), (5, 200, 64)])
def test_block_gemm(prec, mode, M, N, K):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if prec == 2 and mode == 2:
        pytest.skip("bf16 has no transposed-A mode")
    import paper_2609_09990_amd as pk
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = rng.standard_normal((K, M) if mode == 2 else (M, K))
    B = rng.standard_normal((N, K) if mode == 1 else (K, N))
    coef = -0.75
    if prec == 2:
        Ab, Bb = _bf16_bits(A), _bf16_bits(B)
        Aref, Bref = _bf16_val(_bf16_bits(coef * _bf16_val(Ab))), _bf16_val(Bb)
        dA = torch.from_numpy(Ab.view(np.int16)).cuda()
        dB = torch.from_numpy(Bb.view(np.int16)).cuda()
        ref = (Aref.T if mode == 2 else Aref) @ (Bref.T if mode == 1 else Bref)
        dC = torch.zeros((M, N), dtype=torch.float32, device="cuda")
        tol = 1e-5
    else:
        dt = torch.float64 if prec == 0 else torch.float32
        dA = torch.from_numpy(A).to(dt).cuda()
        dB = torch.from_numpy(B).to(dt).cuda()
        Ar = dA.double().cpu().numpy()
        Br = dB.double().cpu().numpy()
        ref = coef * ((Ar.T if mode == 2 else Ar) @ (Br.T if mode == 1 else Br))
        dC = torch.zeros((M, N), dtype=dt, device="cuda")
        tol = 1e-13 if prec == 0 else 1e-5
    lda = A.shape[1]
    ldb = B.shape[1]
    code = pk.dmrg_block_gemm(prec, mode, M, N, K, ctypes.c_void_p(dA.data_ptr()), lda,
                              ctypes.c_void_p(dB.data_ptr()), ldb, ctypes.c_void_p(dC.data_ptr()), N,
                              coef, None)
    assert code == 0, pk.dmrg_last_error()
    got = dC.double().cpu().numpy()
    err = np.max(np.abs(got - ref)) / max(1.0, np.max(np.abs(ref)))
    assert err < tol * np.sqrt(K), err
