"""mp_gemm_noalloc: the product of mp_gemm with every device buffer in the
library's fixed scratch array (for callers that cannot allocate).

Through the C ABI, two calls in a row (the second smaller, with another
shape and algorithm, so the array holds the first call's plan and
temporaries when the second starts) must give the bits of mp_gemm for the
same arguments; one of them is also checked against the CPU oracle.  A
product whose temporaries exceed the array is refused before anything is
launched (checked on the CPU and on the GPU: C is left untouched).
"""

import ctypes

import numpy as np
import pytest

from helpers import planes_equal
from oracle import cref
from paper_1410_1599_amd import inputs as I

torch = pytest.importorskip("torch")
from paper_1410_1599_amd import mp  # noqa: E402


def test_noalloc_refuses_oversized_product_without_device():
    lib = mp.lib
    n, p = 1024, 256
    words = (p // 32 + 2) * n * n
    base = 1 << 40
    A, B, C = base, base + 4 * words + 4096, base + 8 * words + 8192
    rc = lib.mp_gemm_noalloc(n, n, n, p, mp.WINOGRAD, 64, ctypes.c_void_p(A), n, n * n, ctypes.c_void_p(B), n,
                             n * n, ctypes.c_void_p(C), n, n * n)
    assert rc == -6, rc
    assert "scratch" in mp.last_error()
    # argument errors are those of mp_gemm
    assert lib.mp_gemm_noalloc(4, 4, 4, 100, 0, 0, ctypes.c_void_p(A), 4, 16, ctypes.c_void_p(B), 4, 16,
                               ctypes.c_void_p(C), 4, 16) == -2
    assert lib.mp_gemm_noalloc(4, 4, 4, 256, 0, 0, ctypes.c_void_p(A), 4, 16, ctypes.c_void_p(B), 4, 16,
                               ctypes.c_void_p(A), 4, 16) == -3


def product_pair(m, l, n, p, algo, cutoff, seed):
    A = mp.to_device(I.uniform_pm1(m, l, p, seed))
    B = mp.to_device(I.uniform_pm1(l, n, p, seed + 1))
    C_ref = mp.empty(m, n, p)
    C_na = mp.empty(m, n, p)
    mp.mp_gemm(m, l, n, p, algo, cutoff, A, B, C_ref)
    mp.mp_gemm_noalloc(m, l, n, p, algo, cutoff, A, B, C_na)
    return A, B, C_ref, C_na


@pytest.mark.gpu
def test_noalloc_equals_mp_gemm_on_two_calls():
    p = 256
    # first call: Winograd, three levels (300 -> 150 -> 75 -> 37), odd sizes peeled
    _, _, R1, N1 = product_pair(300, 277, 290, p, mp.WINOGRAD, 64, 41)
    torch.cuda.synchronize()
    assert torch.equal(R1, N1)
    # second call, smaller: Strassen with another cutoff, then Simple
    A2, B2, R2, N2 = product_pair(150, 131, 97, p, mp.STRASSEN, 32, 43)
    torch.cuda.synchronize()
    assert torch.equal(R2, N2)
    want = cref.gemm(mp.to_host(A2), mp.to_host(B2), p, algo="strassen", cutoff=32)
    assert planes_equal(mp.to_host(N2), want)
    _, _, R3, N3 = product_pair(70, 65, 33, 512, mp.SIMPLE, 0, 45)
    torch.cuda.synchronize()
    assert torch.equal(R3, N3)


@pytest.mark.gpu
def test_noalloc_refuses_oversized_product_on_device():
    n, p = 1024, 256
    A = mp.empty(n, n, p)
    B = mp.empty(n, n, p)
    C = torch.full((p // 32 + 2, n, n), 7, dtype=torch.int32, device="cuda")
    with pytest.raises(mp.MPError) as e:
        mp.mp_gemm_noalloc(n, n, n, p, mp.WINOGRAD, 64, A, B, C)
    assert e.value.code == -6
    torch.cuda.synchronize()
    assert bool((C == 7).all())
    # Simple needs no temporaries: any size fits
    m2 = 257
    A2 = mp.to_device(I.uniform_pm1(m2, 64, p, 47))
    B2 = mp.to_device(I.uniform_pm1(64, m2, p, 48))
    R, N = mp.empty(m2, m2, p), mp.empty(m2, m2, p)
    mp.mp_gemm(m2, 64, m2, p, mp.SIMPLE, 0, A2, B2, R)
    mp.mp_gemm_noalloc(m2, 64, m2, p, mp.SIMPLE, 0, A2, B2, N)
    torch.cuda.synchronize()
    assert torch.equal(R, N)
