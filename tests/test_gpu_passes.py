"""GPU parity of each pass and of the full transforms against the FP64 oracle.

Element-by-element comparison on seeded inputs; sizes span several tiles and
a ragged tail (K = N/2 + 1 is odd, so the last column tile of every y pass
is partial).  Tolerance: relative L2 <= 1e-13 (FP64), <= 5e-6 (FP32).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import TOL, cplx_input, host, real_input, rel_l2
from paper_2202_12756_amd import Plan

pytestmark = pytest.mark.gpu

SIZES = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096]
DTYPES = [torch.float64, torch.float32]


def planes_for(n):
    """A few planes at large N keep the oracle within seconds."""
    return max(1, min(n, 2 ** 21 // (n * n)))


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("n", SIZES)
def test_z_r2c(n, dtype):
    x = planes_for(n)
    p = Plan(n, dtype, slab_x=x) if x < n else Plan(n, dtype)
    xin, xref = real_input(p.real_shape, 1000 + n, dtype)
    out = p.z_r2c(xin)
    torch.cuda.synchronize()
    assert rel_l2(host(out), oracle.r2c_last(xref)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("n", SIZES)
def test_z_c2r_nonhermitian(n, dtype):
    x = planes_for(n)
    p = Plan(n, dtype, slab_x=x) if x < n else Plan(n, dtype)
    g, gref = cplx_input(p.spectrum_shape, 2000 + n, dtype)
    out = p.z_c2r(g, scale=0.5)
    torch.cuda.synchronize()
    assert rel_l2(host(out), 0.5 * oracle.c2r_last(gref, n)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("sign", [-1, 1])
def test_y_c2c(n, dtype, sign):
    x = planes_for(n)
    p = Plan(n, dtype, slab_x=x) if x < n else Plan(n, dtype)
    g, gref = cplx_input(p.spectrum_shape, 3000 + n, dtype)
    p.y_c2c(g, sign)
    torch.cuda.synchronize()
    assert rel_l2(host(g), oracle.c2c_axis(gref, -2, sign)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("sign", [-1, 1])
def test_x_c2c(n, dtype, sign):
    # pencil [N][N/p][K] with N/p a power of two small enough for the oracle
    y = max(1, min(n, 2 ** 21 // (n * (n // 2 + 1))))
    y = 1 << (y.bit_length() - 1)
    p = Plan(n, dtype, slab_x=y)
    g, gref = cplx_input(p.pencil_shape, 4000 + n, dtype)
    p.x_c2c(g, sign)
    torch.cuda.synchronize()
    assert rel_l2(host(g), oracle.c2c_axis(gref, -3, sign)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_full_r2c_c2r(n, dtype):
    p = Plan(n, dtype)
    xin, xref = real_input(p.real_shape, 5000 + n, dtype)
    F = p.r2c(xin)
    torch.cuda.synchronize()
    Fref = oracle.r2c3d(xref)
    assert rel_l2(host(F), Fref) <= TOL[dtype]
    back = p.c2r(F, scale=1.0 / n ** 3)
    torch.cuda.synchronize()
    assert rel_l2(host(back), xref) <= TOL[dtype]


@pytest.mark.parametrize("n", [16, 64])
def test_full_c2r_nonhermitian(n):
    p = Plan(n, torch.float64)
    g, gref = cplx_input(p.spectrum_shape, 6000 + n, torch.float64)
    out = p.c2r(g)
    torch.cuda.synchronize()
    assert rel_l2(host(out), oracle.c2r3d(gref, n)) <= 1e-13


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_batch(dtype):
    n, b = 32, 3
    p = Plan(n, dtype, batch=b)
    xin, xref = real_input(p.real_shape, 7000, dtype)
    F = p.r2c(xin)
    torch.cuda.synchronize()
    assert rel_l2(host(F), oracle.r2c3d(xref)) <= TOL[dtype]


@pytest.mark.parametrize("n", [16, 64, 128, 256])
def test_paper_field_round_trip(n):
    """Section 4 test field: a DP pair recovers it within 1e-14 (relative to
    max|f|), and the spectrum has only the eight analytic bins."""
    f = synth.paper_test_field(n)
    p = Plan(n, torch.float64)
    F = p.r2c(torch.from_numpy(f).cuda().reshape(p.real_shape))
    Fh = host(F)[0] / n ** 3
    back = p.c2r(F, scale=1.0 / n ** 3)
    torch.cuda.synchronize()
    assert np.max(np.abs(host(back).reshape(f.shape) - f)) <= 1e-14 * np.max(np.abs(f))
    ref = np.zeros_like(Fh)
    for (a, b, c) in ((1, 2, 3), (4, 5, 6)):
        for sx in (1, -1):
            for sy in (1, -1):
                ref[(sx * a) % n, (sy * b) % n, c] = 1j * sx * sy
    assert np.max(np.abs(Fh - ref)) <= 1e-15 * n


@pytest.mark.parametrize("terms,bound", [(2, 1e-4), (3, 5e-6)])
@pytest.mark.parametrize("n", [32, 64, 256, 1024, 2048, 4096])
@pytest.mark.parametrize("sign", [-1, 1])
def test_mfma_split_bf16_strided(n, terms, bound, sign):
    """First radix-16 stage on the matrix cores: error against the FP64
    oracle (2 BF16 terms: about 2^-16 per product; 3 terms: FP32 level)."""
    x = planes_for(n)
    p = Plan(n, torch.float32, slab_x=x if x < n else None, mfma_terms=terms)
    g, gref = cplx_input(p.spectrum_shape, 8000 + n, torch.float32)
    p.y_c2c(g, sign)
    torch.cuda.synchronize()
    err = rel_l2(host(g), oracle.c2c_axis(gref, -2, sign))
    print(f"mfma bf16x{terms} y pass n={n} sign={sign}: rel-L2 {err:.3e}")
    assert err <= bound
    y = max(1, min(n, 2 ** 21 // (n * (n // 2 + 1))))
    y = 1 << (y.bit_length() - 1)
    q = Plan(n, torch.float32, slab_x=y, mfma_terms=terms)
    pen, pref = cplx_input(q.pencil_shape, 8100 + n, torch.float32)
    q.x_c2c(pen, sign)
    torch.cuda.synchronize()
    err = rel_l2(host(pen), oracle.c2c_axis(pref, -3, sign))
    print(f"mfma bf16x{terms} x pass n={n} sign={sign}: rel-L2 {err:.3e}")
    assert err <= bound


@pytest.mark.parametrize("terms", [2, 3])
def test_mfma_full_round_trip(terms):
    n = 64
    p = Plan(n, torch.float32, mfma_terms=terms)
    xin, xref = real_input(p.real_shape, 8200, torch.float32)
    F = p.r2c(xin)
    torch.cuda.synchronize()
    err = rel_l2(host(F), oracle.r2c3d(xref))
    back = p.c2r(F, scale=1.0 / n ** 3)
    torch.cuda.synchronize()
    rt = rel_l2(host(back), xref)
    print(f"mfma bf16x{terms} 64^3: forward rel-L2 {err:.3e}, round trip {rt:.3e}")
    assert err <= (1e-4 if terms == 2 else 5e-6)
    assert rt <= (1e-4 if terms == 2 else 5e-6)
