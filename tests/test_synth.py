"""The seeded generators: published SplitMix64 values, ranges, exactness."""
import numpy as np
import torch

import synth


def _splitmix_ref(state, count):
    """SplitMix64 next() loop in Python integers (Steele, Lea, Flood 2014)."""
    mask = (1 << 64) - 1
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & mask
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        out.append(z ^ (z >> 31))
    return out


def test_splitmix_matches_sequential_generator():
    for seed in (0, 1, 7):
        ref = _splitmix_ref(seed << 40, 50)
        got = synth.splitmix_bits(seed, 0, 50).tolist()
        assert [g & ((1 << 64) - 1) for g in got] == ref
        mid = synth.splitmix_bits(seed, 20, 5).tolist()
        assert [g & ((1 << 64) - 1) for g in mid] == ref[20:25]


def test_splitmix_known_value():
    # first output of SplitMix64 from state 0 (widely published test value)
    assert synth.splitmix_bits(0, 0, 1).item() & ((1 << 64) - 1) == 0xE220A8397B1DCDAF


def test_uniform_range_and_exactness():
    a = synth.uniform((1000,), 3, torch.float64)
    assert float(a.min()) >= -1.0 and float(a.max()) < 1.0
    b = synth.uniform((1000,), 3, torch.float32)
    assert b.dtype == torch.float32
    # FP32 values are the 24 most significant bits: exact in FP32
    assert torch.equal(b.double().float(), b)
    # offset reproduces a sub-block of the same stream
    c = synth.uniform((10,), 3, torch.float64, offset=500)
    assert torch.equal(c, a[500:510])
    # chunking does not change values
    d = synth.uniform((1000,), 3, torch.float64, chunk=77)
    assert torch.equal(a, d)


def test_kolmogorov_band_and_seed():
    n = 16
    g = synth.kolmogorov_half_spectrum(n, 2)
    assert g.shape == (n, n, n // 2 + 1)
    assert g[0, 0, 0] == 0
    assert np.all(g[:, :, 6:] == 0)         # 9 k^2 > 256 for kz >= 6
    assert np.array_equal(g, synth.kolmogorov_half_spectrum(n, 2))
