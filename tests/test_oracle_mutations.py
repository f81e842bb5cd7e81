"""The pins catch plausible mistakes planted in the oracle.

Each case copies oracle.c, plants one mistake (a flipped sign, a dropped
factor or term, a wrong index, a transposed operand), builds the copy, swaps
it in for the real library and runs a compact battery of the pins; at least
one pin must fail.  The real library is restored afterwards.  CPU only.
(Dropping the zeroing of Im at kz = 0 and N/2 in the radix-2 C2R is not a
mistake: those imaginary parts only reach the imaginary part of the inverse
DFT, which that path discards.)
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTATIONS = {
    "conjugated roots": ("    *im = -s;", "    *im = s;"),
    "no octant swap": ("    if (swap) { double u = c; c = s; s = u; }", "    (void)swap;"),
    "butterfly sign": ("v[0] = ur - vr; v[1] = ui - vi;", "v[0] = ur - vr; v[1] = ui + vi;"),
    "wrong product index": ("            int64_t m = (j * k) % n;", "            int64_t m = (j * k + k) % n;"),
    "dropped C2R weight": ("double wk = (k == 0 || 2 * k == N) ? 1.0 : 2.0;",
                           "double wk = (k == 0 || 2 * k == N) ? 1.0 : 1.0;"),
    "wrong mirror index": ("                        xl[2 * k] = g[2 * (N - k)];",
                           "                        xl[2 * k] = g[2 * (N - k - 1)];"),
    "missing conjugate": ("xl[2 * k + 1] = -g[2 * (N - k) + 1];", "xl[2 * k + 1] = g[2 * (N - k) + 1];"),
    "transposed gather": ("                xl[2 * j] = src[2 * j * M];\n                xl[2 * j + 1] = src[2 * j * M + 1];",
                          "                xl[2 * j] = src[2 * j];\n                xl[2 * j + 1] = src[2 * j + 1];"),
    "off-by-one bins": ("memcpy(out + 2 * r * K, yl, sizeof(double) * 2 * (size_t)K);",
                        "memcpy(out + 2 * r * K, yl + 2, sizeof(double) * 2 * (size_t)K);"),
    "z-sum sign": ("                si += f[z] * w[2 * m + 1];", "                si -= f[z] * w[2 * m + 1];"),
    "radix-2 twiddle step": ("        int64_t half = len / 2, step = n / len;",
                             "        int64_t half = len / 2, step = n / half;"),
}


def _rand(shape, seed):
    return synth.uniform(shape, seed).numpy()


def _brute_r2c(f):
    n = f.shape[0]
    j = np.indices((n, n, n)).reshape(3, -1)
    k = np.indices((n, n, n // 2 + 1)).reshape(3, -1)
    e = np.exp(-2j * np.pi * ((k.T @ j) % n) / n)
    return (e @ f.reshape(-1)).reshape(n, n, n // 2 + 1)


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def battery():
    """A compact subset of the pins; returns the names of those that fail."""
    failed = []
    checks = []
    for n in (5, 8):
        f = _rand((n, n, n), 7 + n)
        ref = _brute_r2c(f)
        checks.append((f"brute r2c direct n={n}", lambda f=f, ref=ref: _rel(oracle.r2c3d(f, oracle.DIRECT), ref) < 1e-13))
        if n == 8:
            checks.append(("brute r2c radix2", lambda f=f, ref=ref: _rel(oracle.r2c3d(f, oracle.RADIX2), ref) < 1e-13))
    for n, m in ((6, oracle.DIRECT), (16, oracle.RADIX2)):
        g = _rand((n, n, n // 2 + 1), 30 + n) + 1j * _rand((n, n, n // 2 + 1), 40 + n)
        checks.append((f"pocketfft c2r n={n}", lambda g=g, n=n, m=m: _rel(
            oracle.c2r3d(g, n, method=m),
            np.fft.irfftn(g, s=(n, n, n), axes=(0, 1, 2), norm="forward")) < 1e-13))
        f = _rand((n, n, n), 50 + n)
        checks.append((f"round trip n={n}", lambda f=f, n=n, m=m: _rel(
            oracle.c2r3d(oracle.r2c3d(f, m), n, method=m), n ** 3 * f) < 1e-13))
    f = _rand((16, 16, 16), 61)
    checks.append(("kz planes", lambda f=f: _rel(oracle.r2c3d_kz_planes(f, [0, 3, 8]),
                                                 np.fft.rfftn(f)[:, :, [0, 3, 8]]) < 1e-13))
    a = _rand((3, 12, 5), 71) + 1j * _rand((3, 12, 5), 72)
    checks.append(("c2c axis", lambda a=a: _rel(oracle.c2c_axis(a, 1, -1),
                                                np.fft.fft(a, axis=1)) < 1e-13))
    for name, fn in checks:
        try:
            ok = bool(fn())
        except Exception:
            ok = False
        if not ok:
            failed.append(name)
    return failed


def _build_mutant(tmp_path, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not unique: {old!r}"
    src = tmp_path / "oracle_mutant.c"
    src.write_text(text.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                    str(src), "-o", str(lib), "-lm"], check=True)
    return str(lib)


def _swap_in(path):
    """Point the oracle module at another build of oracle.c."""
    real = oracle._load()
    mutant = ctypes.CDLL(path)
    for name in ("oracle_c2c_axis", "oracle_r2c_rows", "oracle_c2r_rows",
                 "oracle_zsum_rows", "oracle_num_threads", "oracle_set_num_threads"):
        f, g = getattr(real, name), getattr(mutant, name)
        g.argtypes, g.restype = f.argtypes, f.restype
    oracle._lib = mutant
    return real


def test_battery_passes_on_the_real_oracle():
    assert battery() == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(tmp_path, name):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    old, new = MUTATIONS[name]
    path = _build_mutant(tmp_path, old, new)
    real = _swap_in(path)
    try:
        failed = battery()
    finally:
        oracle._lib = real
    assert failed, f"no pin caught the planted mistake '{name}'"


def test_pins_catch_python_level_mistakes(monkeypatch):
    """Mistakes in the composition layer: weights and axis order."""
    n = 8
    f = _rand((n, n, n), 91)
    g = _rand((n, n, n // 2 + 1), 92) + 1j * _rand((n, n, n // 2 + 1), 93)
    # adjoint with all-ones weights fails the dot-product test
    monkeypatch.setattr(oracle, "half_weights", lambda m: np.ones(m // 2 + 1))
    lhs = np.sum(np.real(np.conj(oracle.r2c3d(f)) * g))
    rhs = np.sum(f * oracle.r2c3d_adjoint(g, n))
    assert abs(lhs - rhs) > 1e-6 * abs(lhs)
    monkeypatch.undo()
    # transforming x before y before z (wrong axis roles) fails brute force
    wrong = oracle.c2c_axis(oracle.c2c_axis(oracle.r2c_last(f.transpose(2, 1, 0)), -2, -1), -3, -1)
    assert _rel(wrong, _brute_r2c(f)) > 1e-3
