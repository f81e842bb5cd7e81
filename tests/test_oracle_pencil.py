"""The oracle's pencil layouts (section 2, pencil decomposition), pinned to
the full-grid forward transform (itself pinned to brute force, closed forms
and the paper's Eq. 5) and to the identities of the exchanges."""
import numpy as np
import torch
import pytest

import oracle
import synth

CASES = [(16, 1, 1), (16, 1, 2), (16, 2, 2), (16, 2, 4), (16, 4, 8), (32, 2, 8), (32, 8, 16),
         (16, 4, 2), (16, 16, 8), (32, 32, 16)]


def test_kz_ranges_partition_the_half_spectrum():
    for n in (16, 32, 64, 1024):
        k = n // 2 + 1
        pc = 1
        while pc <= n // 2:
            seen = np.zeros(k, dtype=int)
            for c in range(pc):
                k0, k1 = oracle.pencil_kz_range(n, pc, c)
                assert k1 - k0 == n // (2 * pc) + (c == pc - 1)
                seen[k0:k1] += 1
            assert np.all(seen == 1)
            pc *= 2


@pytest.mark.parametrize("pc", [1, 2, 8])
def test_send_order_round_trip_and_chunk_contents(pc):
    n, x, y = 16, 4, 2
    k = n // 2 + 1
    rows = np.arange(2 * x * y * k).reshape(2, x, y, k).astype(np.complex128)
    flat = oracle.pencil_send(rows, pc)
    assert flat.shape == (2, x * y * k)
    assert np.array_equal(oracle.pencil_unsend(flat, x, y, pc), rows)
    # chunk c' begins at X Y k0 and is the [X][Y][w] block of its bins
    for c in range(pc):
        k0, k1 = oracle.pencil_kz_range(n, pc, c)
        blk = flat[:, x * y * k0:x * y * k1].reshape(2, x, y, k1 - k0)
        assert np.array_equal(blk, rows[..., k0:k1])


def _forward(f, n, pr, pc):
    """The pencil pipeline on the oracle: per rank z R2C, exchange 1, y DFT,
    exchange 2, x DFT.  Returns {(r, c): x-pencil}."""
    x, y = n // pr, n // pc
    xp = {}
    ys = {}
    for r in range(pr):
        sends = [oracle.pencil_send(oracle.r2c_last(f[r * x:(r + 1) * x, c * y:(c + 1) * y]), pc)
                 for c in range(pc)]
        for c, yp in enumerate(oracle.pencil_exchange1(sends, x, y)):
            ys[r, c] = oracle.pencil_y_c2c(yp, -1)
    for c in range(pc):
        for rp, xpen in enumerate(oracle.pencil_exchange2([ys[r, c] for r in range(pr)], pr)):
            if pr <= pc:
                xp[rp, c] = oracle.pencil_x_c2c(xpen, -1)
            else:                              # [pr][X][N/pr][w] = [N][N/pr][w]
                xp[rp, c] = oracle.x_c2c(xpen.reshape(n, n // pr, -1), -1).reshape(xpen.shape)
    return xp, ys


@pytest.mark.parametrize("n,pr,pc", CASES)
def test_pencil_pipeline_equals_full_transform(n, pr, pc):
    """Every x-pencil element equals F(x = r X + x_l, y = r' N/pr + g_l Y +
    y_l, kz = c w0 + kz_l) of the full-grid transform; p = pr pc exceeds N
    in the last cases."""
    assert _pipeline_error(n, pr, pc) <= 1e-12


def _pipeline_error(n, pr, pc):
    """Largest deviation of the pencil pipeline from the full transform,
    relative to max |F|; the expected index of each element is written out
    here from the layout definitions, independently of the oracle's."""
    f = synth.uniform((n, n, n), 900 + n + pr + pc, torch.float64, "cpu").numpy()
    F = oracle.r2c3d(f)
    x, y, w0 = n // pr, n // pc, n // (2 * pc)
    xp, _ = _forward(f, n, pr, pc)
    worst = 0.0
    for (rp, c), got in xp.items():
        k0, k1 = oracle.pencil_kz_range(n, pc, c)
        if pr <= pc:
            g = pc // pr
            r_, g_, x_, y_, k_ = np.meshgrid(np.arange(pr), np.arange(g), np.arange(x),
                                             np.arange(y), np.arange(k1 - k0), indexing="ij")
            want = F[r_ * x + x_, rp * (n // pr) + g_ * y + y_, c * w0 + k_]
            assert got.shape == (pr, g, x, y, k1 - k0)
        else:
            r_, x_, y_, k_ = np.meshgrid(np.arange(pr), np.arange(x), np.arange(n // pr),
                                         np.arange(k1 - k0), indexing="ij")
            want = F[r_ * x + x_, rp * (n // pr) + y_, c * w0 + k_]
            assert got.shape == (pr, x, n // pr, k1 - k0)
        worst = max(worst, np.max(np.abs(got - want)) / np.max(np.abs(F)))
    return worst


def _mutants():
    """Plausible mistakes in the pencil layouts, one per oracle function."""
    orig = {k: getattr(oracle, k) for k in ("pencil_kz_range", "pencil_exchange1",
                                             "pencil_exchange2", "pencil_send", "pencil_y_c2c")}

    def nyquist_first(n, pc, c):
        w0 = n // (2 * pc)
        return c * w0 + (c > 0), (c + 1) * w0 + 1

    def reversed_blocks(sends, x, y):
        return orig["pencil_exchange1"](sends[::-1], x, y)

    def shifted_peers(ypencils, pr):
        out = orig["pencil_exchange2"](ypencils, pr)
        return out[1:] + out[:1]

    def transposed_chunks(rows, pc):
        return orig["pencil_send"](np.ascontiguousarray(np.swapaxes(rows, -2, -3))
                                   .reshape(rows.shape), pc)

    def wrong_axis(ypencil, sign, method=None):
        return oracle.c2c_axis(ypencil, -3, sign, method)

    return {"pencil_kz_range": nyquist_first, "pencil_exchange1": reversed_blocks,
            "pencil_exchange2": shifted_peers, "pencil_send": transposed_chunks,
            "pencil_y_c2c": wrong_axis}


@pytest.mark.parametrize("name", ["pencil_kz_range", "pencil_exchange1", "pencil_exchange2",
                                  "pencil_send", "pencil_y_c2c"])
def test_pencil_pins_catch_planted_mistakes(name, monkeypatch):
    monkeypatch.setattr(oracle, name, _mutants()[name])
    worst = max(_pipeline_error(16, pr, pc) for pr, pc in ((2, 4), (4, 2)))
    assert worst > 1e-6, f"the pencil pins missed the planted mistake in {name}"


@pytest.mark.parametrize("n,pr,pc", CASES[2:])
def test_pencil_round_trip(n, pr, pc):
    """Backwards through x^-1, exchange 2 back, y^-1, exchange 1 back and
    the z C2R gives N^3 f."""
    f = synth.uniform((n, n, n), 950 + n, torch.float64, "cpu").numpy()
    x, y = n // pr, n // pc
    xp, _ = _forward(f, n, pr, pc)
    out = np.empty_like(f)
    for c in range(pc):
        inv = []
        for rp in range(pr):
            if pr <= pc:
                inv.append(oracle.pencil_x_c2c(xp[rp, c], +1))
            else:
                a = xp[rp, c]
                inv.append(oracle.x_c2c(a.reshape(n, n // pr, -1), +1).reshape(a.shape))
        back = oracle.pencil_exchange2_back(inv, pc)
        for r in range(pr):
            xp[r, c] = oracle.pencil_y_c2c(back[r], +1)          # reuse as y-pencils
    for r in range(pr):
        sends = oracle.pencil_exchange1_back([xp[r, c] for c in range(pc)])
        for c in range(pc):
            rows = oracle.pencil_unsend(sends[c], x, y, pc)
            out[r * x:(r + 1) * x, c * y:(c + 1) * y] = oracle.c2r_last(rows, n)
    assert np.max(np.abs(out / n ** 3 - f)) <= 1e-13


def test_exchange_back_inverts_exchange():
    rng = np.random.default_rng(5)
    x, y, pc, pr = 2, 4, 4, 2
    k = 9
    sends = [rng.standard_normal((x * y * k,)) + 0j for _ in range(pc)]
    ys = oracle.pencil_exchange1(sends, x, y)
    for a, b in zip(oracle.pencil_exchange1_back(ys), sends):
        assert np.array_equal(a, b)
    for pr_ in (2, 8):           # pr <= pc and pr > pc
        ypens = [rng.standard_normal((pc, x, y, 3)) for _ in range(pr_)]
        back = oracle.pencil_exchange2_back(oracle.pencil_exchange2(ypens, pr_), pc)
        for a, b in zip(back, ypens):
            assert np.array_equal(a, b)


def test_pack2_runs_are_the_second_exchange_blocks():
    """pr > pc: run (c', s) of the packed y-pencil is exactly what
    exchange 2 delivers to rank c' h + s."""
    rng = np.random.default_rng(6)
    pc, pr, x, y, w = 2, 8, 2, 8, 3
    h = pr // pc
    ypens = [rng.standard_normal((pc, x, y, w)) for _ in range(pr)]
    recv = oracle.pencil_exchange2(ypens, pr)
    for r, yp in enumerate(ypens):
        packed = oracle.pencil_pack2(yp, h)
        assert packed.shape == (pc, h, x, y // h, w)
        for cp in range(pc):
            for s in range(h):
                assert np.array_equal(packed[cp, s], recv[cp * h + s][r])
