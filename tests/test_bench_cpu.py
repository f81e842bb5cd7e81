"""bench.py host logic without a GPU: refusal of several GPUs, the FLOP
convention, the recorded-traffic lookup (valid only for the kernel
sources it was measured on) and the workload groups of --only."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_flop_convention():
    # 5 (N^3/2) log2 N^3 per R2C, two per pair: 161.06 GFLOP at 1024^3
    assert abs(bench.gflop_pair(1024) - 161.061273600) < 1e-6


def test_recorded_traffic_requires_matching_sources(tmp_path):
    got = bench.recorded_traffic(bench.TRAFFIC_FILE, "x_fwd")
    if got is not None:                       # summary taken on these sources
        assert 0.9 < got / (2 * 1024 * 1024 * 513 * 16) < 1.1
    stale = tmp_path / "stale.md"
    text = open(bench.TRAFFIC_FILE).read()
    stale.write_text(text.replace(f"kernel_source_sha256_16: {bench.kernel_source_hash()}",
                                  "kernel_source_sha256_16: 0000000000000000"))
    assert bench.recorded_traffic(str(stale), "x_fwd") is None
    assert bench.recorded_traffic(str(tmp_path / "missing.md"), "x_fwd") is None


def test_only_groups():
    # every group --only offers is one of the variant functions of the full run
    assert set(bench.ONLY) == {"slab_4096", "pencil_4096", "full_2048", "graphs",
                               "kolmogorov_512", "losses_8x256", "slab_pack_p8"}
    assert all(callable(f) for f in bench.ONLY.values())
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--only", "nope"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "invalid choice" in r.stderr


def test_cpu_model_and_hermitian_part():
    import torch

    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
    # H(G) keeps interior bins, and on the kz = 0 and N/2 planes averages
    # each bin with the conjugate of its mirror -k
    n = 8
    g = torch.complex(torch.randn(1, n, n, n // 2 + 1, dtype=torch.float64),
                      torch.randn(1, n, n, n // 2 + 1, dtype=torch.float64))
    h = bench._hermitian_part(g)
    assert torch.equal(h[..., 1:-1], g[..., 1:-1])
    for kz in (0, n // 2):
        for i in range(n):
            for j in range(n):
                want = 0.5 * (g[0, i, j, kz] + g[0, (-i) % n, (-j) % n, kz].conj())
                assert abs(h[0, i, j, kz] - want) < 1e-15
