"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against the definition evaluated by brute force,
a closed form, an identity of the DFT, the paper's own test field and
accuracy claim, or an independent library; together they are chosen so that
a dropped term, a wrong sign, a wrong index or a transposed operand anywhere
in the oracle fails at least one of them.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rand_real(shape, seed):
    return synth.uniform(shape, seed).numpy()


def rand_cplx(shape, seed):
    return rand_real(shape, seed) + 1j * rand_real(shape, seed + 1000)


# ---------------------------------------------------------------- brute force

def brute_r2c(f):
    """Forward equation of section 2 as one sum per output bin."""
    n = f.shape[0]
    j = np.indices((n, n, n)).reshape(3, -1)
    k = np.indices((n, n, n // 2 + 1)).reshape(3, -1)
    phase = (k.T @ j) % n
    e = np.exp(-2j * np.pi * phase / n)
    return (e @ f.reshape(-1)).reshape(n, n, n // 2 + 1)


def brute_c2r(g, n):
    """w-weighted real part over the stored half, one sum per output point."""
    j = np.indices((n, n, n)).reshape(3, -1)
    k = np.indices((n, n, n // 2 + 1)).reshape(3, -1)
    phase = (j.T @ k) % n
    e = np.exp(2j * np.pi * phase / n)
    w = oracle.half_weights(n)[k[2]]
    return (np.real(e * g.reshape(-1)[None, :]) @ w).reshape(n, n, n)


def brute_c2c_1d(x, sign):
    n = x.shape[-1]
    jk = np.outer(np.arange(n), np.arange(n)) % n
    return x @ np.exp(sign * 2j * np.pi * jk / n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8])
def test_p1_bruteforce_r2c(n):
    f = rand_real((n, n, n), 11 + n)
    ref = brute_r2c(f)
    assert rel_l2(oracle.r2c3d(f, oracle.DIRECT), ref) <= 1e-14
    if n & (n - 1) == 0:
        assert rel_l2(oracle.r2c3d(f, oracle.RADIX2), ref) <= 1e-14


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8])
def test_p1_bruteforce_c2r_nonhermitian(n):
    g = rand_cplx((n, n, n // 2 + 1), 21 + n)   # deliberately not Hermitian
    ref = brute_c2r(g, n)
    assert rel_l2(oracle.c2r3d(g, n, method=oracle.DIRECT), ref) <= 1e-14
    if n & (n - 1) == 0:
        assert rel_l2(oracle.c2r3d(g, n, method=oracle.RADIX2), ref) <= 1e-14


@pytest.mark.parametrize("n", [1, 7, 16, 64])
@pytest.mark.parametrize("sign", [-1, 1])
def test_p1_bruteforce_c2c_axis(n, sign):
    a = rand_cplx((3, n, 5), 31 + n)
    for axis in (0, 1, 2):
        ref = np.moveaxis(brute_c2c_1d(np.moveaxis(a, axis, -1), sign), -1, axis)
        got = oracle.c2c_axis(a, axis, sign, oracle.DIRECT)
        assert rel_l2(got, ref) <= 1e-13
        if a.shape[axis] & (a.shape[axis] - 1) == 0:
            got = oracle.c2c_axis(a, axis, sign, oracle.RADIX2)
            assert rel_l2(got, ref) <= 1e-13


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [8, 16])
def test_p2_delta(n):
    f = np.zeros((n, n, n))
    f[0, 0, 0] = 1.0
    assert np.max(np.abs(oracle.r2c3d(f) - 1.0)) <= 1e-15
    j0 = (1, 3, 5)
    f = np.zeros((n, n, n))
    f[j0] = 1.0
    kx, ky, kz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n // 2 + 1),
                             indexing="ij")
    ref = np.exp(-2j * np.pi * (kx * j0[0] + ky * j0[1] + kz * j0[2]) / n)
    for m in (oracle.DIRECT, oracle.RADIX2):
        assert np.max(np.abs(oracle.r2c3d(f, m) - ref)) <= 1e-14


@pytest.mark.parametrize("k0", [(1, 2, 3), (0, 5, 0), (3, 0, 8), (8, 8, 8),
                                (15, 1, 2)])
def test_p3_plane_wave(k0):
    n = 16
    j = np.indices((n, n, n))
    f = np.cos(2 * np.pi * (k0[0] * j[0] + k0[1] * j[1] + k0[2] * j[2]) / n)
    ref = np.zeros((n, n, n // 2 + 1), dtype=complex)
    for s in (1, -1):
        k = tuple((s * c) % n for c in k0)
        if k[2] <= n // 2:
            ref[k] += n ** 3 / 2
    got = oracle.r2c3d(f)
    assert np.max(np.abs(got - ref)) <= 1e-11


def _eq5_golden(n):
    bins, tol = [], None
    with open(os.path.join(HERE, "golden", "eq5_spectrum.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            parts = line.split()
            if parts[0] == "roundtrip_maxrel_fp64":
                tol = float(parts[1])
                continue
            idx = tuple(n - int(p[2:]) if p.startswith("N-") else int(p)
                        for p in parts[:3])
            bins.append((idx, complex(float(parts[3]), float(parts[4]))))
    return bins, tol


@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_p4_paper_test_field(n):
    f = synth.paper_test_field(n)
    bins, tol = _eq5_golden(n)
    ref = np.zeros((n, n, n // 2 + 1), dtype=complex)
    for idx, v in bins:
        ref[idx] = v
    got = oracle.r2c3d(f) / n ** 3
    assert np.max(np.abs(got - ref)) <= 1e-15 * n
    back = oracle.c2r3d(oracle.r2c3d(f), n, 1.0 / n ** 3)
    assert np.max(np.abs(back - f)) <= tol * np.max(np.abs(f))


# ---------------------------------------------------------------- identities

@pytest.mark.parametrize("n", [6, 16, 32])
def test_p5_parseval(n):
    f = rand_real((n, n, n), 51)
    F = oracle.r2c3d(f)
    lhs = np.sum(f ** 2)
    rhs = np.sum(oracle.half_weights(n) * np.abs(F) ** 2) / n ** 3
    assert abs(lhs - rhs) / lhs <= 1e-14


@pytest.mark.parametrize("n", [8, 16])
def test_p6_hermitian(n):
    f = rand_real((n, n, n), 61)
    full = f.astype(complex)
    for ax in (2, 1, 0):
        full = oracle.c2c_axis(full, ax, -1)
    neg = full[(-np.arange(n)) % n][:, (-np.arange(n)) % n][:, :, (-np.arange(n)) % n]
    assert np.max(np.abs(neg - np.conj(full))) <= 1e-12
    half = oracle.r2c3d(f)
    assert np.max(np.abs(half - full[:, :, : n // 2 + 1])) <= 1e-12
    for kz in (0, n // 2):
        plane = half[:, :, kz]
        negp = plane[(-np.arange(n)) % n][:, (-np.arange(n)) % n]
        assert np.max(np.abs(negp - np.conj(plane))) <= 1e-12
    for kx in (0, n // 2):
        for ky in (0, n // 2):
            for kz in (0, n // 2):
                assert abs(half[kx, ky, kz].imag) <= 1e-12


@pytest.mark.parametrize("n", [5, 16, 32])
def test_p7_round_trip(n):
    f = rand_real((n, n, n), 71)
    back = oracle.c2r3d(oracle.r2c3d(f), n)
    assert rel_l2(back, n ** 3 * f) <= 1e-14


@pytest.mark.parametrize("n", [4, 7, 16, 64])
def test_p8_numpy_pocketfft(n):
    f = rand_real((n, n, n), 81)
    assert rel_l2(oracle.r2c3d(f), np.fft.rfftn(f)) <= 1e-13
    g = rand_cplx((n, n, n // 2 + 1), 82)
    ref = np.fft.irfftn(g, s=(n, n, n), axes=(0, 1, 2), norm="forward")
    assert rel_l2(oracle.c2r3d(g, n), ref) <= 1e-13


@pytest.mark.parametrize("n", [16, 32])
def test_p9_direct_vs_radix2(n):
    f = rand_real((n, n, n), 91)
    a = oracle.r2c3d(f, oracle.DIRECT)
    b = oracle.r2c3d(f, oracle.RADIX2)
    assert rel_l2(a, b) <= 1e-13
    g = rand_cplx((n, n, n // 2 + 1), 92)
    assert rel_l2(oracle.c2r3d(g, n, method=oracle.DIRECT),
                  oracle.c2r3d(g, n, method=oracle.RADIX2)) <= 1e-13


def test_p9_direct_vs_radix2_long_lines():
    a = rand_cplx((4, 256, 3), 93)
    for s in (-1, 1):
        assert rel_l2(oracle.c2c_axis(a, 1, s, oracle.DIRECT),
                      oracle.c2c_axis(a, 1, s, oracle.RADIX2)) <= 1e-13


def test_oracle_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.c2c_axis(np.zeros((2, 6, 2), complex), 1, -1, oracle.RADIX2)
    with pytest.raises(ValueError):
        oracle.c2r_last(np.zeros((2, 4), complex), 8)
