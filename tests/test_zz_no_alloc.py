"""The allocation-free weight-gradient product against the allocating entry
point it mirrors (lts_nn_gemm_tn_bf16), through the C ABI.

Both run the same matrix-core product and the same ordered reduction over the
same row partition, so the bar is bitwise equality; the exact FP64 product
bounds both (K 2^-24 sum |a d| per entry, held at 4x).  Two calls in a row
share the library's fixed partial buffer, the second with fewer rows, so
stale partials of the first call would show up in the second.
"""
import math
import sys

import numpy as np
import pytest

from paper_2106_07154_amd import lts

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def bf16_bits(x):
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)


def bf16_round(x):
    return (bf16_bits(x).astype(np.uint32) << 16).view(np.float32)


@pytest.fixture(scope="module", autouse=True)
def gpu_lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lts.load_library()


def _case(rng, N, K):
    A = bf16_round(rng.standard_normal((N, K)))
    D = bf16_round(rng.standard_normal((N, 64)))
    return A, D


@pytest.mark.parametrize("K,sizes", [(128, (70001, 1100)), (16, (4097, 37)), (64, (1024, 0))])
def test_noalloc_matches_allocating_entry_point(K, sizes):
    import torch
    rng = np.random.default_rng(K)
    s = torch.cuda.Stream()
    for N in sizes:
        say("gemm_tn noalloc", N, K)
        A, D = _case(rng, N, K)
        dA = torch.from_numpy(bf16_bits(A).view(np.int16)).cuda()
        dD = torch.from_numpy(bf16_bits(D).view(np.int16)).cuda()
        P = torch.full((K, 64), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        lts.nn_gemm_tn_bf16_device_noalloc(dA, dD, P, stream=s)
        s.synchronize()
        got = P.cpu().numpy()
        if N == 0:
            assert np.array_equal(got, np.zeros((K, 64), np.float32))
            continue
        want = lts.nn_gemm_tn_bf16(bf16_bits(A), bf16_bits(D))
        assert np.array_equal(got, want)
        ref = A.astype(np.float64).T @ D.astype(np.float64)
        bound = 4 * N * 2.0 ** -24 * (np.abs(A).astype(np.float64).T @ np.abs(D)) + 1e-30
        assert np.all(np.abs(got - ref) <= bound)


def test_noalloc_rejects_sizes_beyond_its_buffer():
    import torch
    K = 128
    nmax = lts.nn_gemm_tn_noalloc_max_rows(K)
    assert nmax == 512 * ((1 << 24) // (256 * K))
    assert lts.nn_gemm_tn_noalloc_max_rows(24) == 0
    say("gemm_tn noalloc reject", nmax + 1, K)
    A = torch.zeros((nmax + 1, K), dtype=torch.int16, device="cuda")
    D = torch.zeros((nmax + 1, 64), dtype=torch.int16, device="cuda")
    P = torch.full((K, 64), 3.0, dtype=torch.float32, device="cuda")
    with pytest.raises(lts.LTSError) as ei:
        lts.nn_gemm_tn_bf16_device_noalloc(A, D, P)
    assert ei.value.status == lts.LTS_EINVAL
    torch.cuda.synchronize()
    assert bool((P == 3.0).all())
