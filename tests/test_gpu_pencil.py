"""GPU parity of pencil plans (section 2, pencil decomposition): every rank
of a pr x pc grid runs on one GPU in turn, the two exchanges are device
copies between the ranks' buffers, and each stage is compared with the
oracle's pencil pipeline; p = pr pc exceeds N in several cases."""
import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, cplx_input, host, real_input, rel_l2
from paper_2202_12756_amd import GfftError, PencilPlan, _lib

pytestmark = pytest.mark.gpu

CASES = [(16, 2, 4), (32, 4, 8), (32, 8, 16), (64, 2, 2), (64, 4, 16), (128, 4, 4),
         (32, 8, 2), (32, 32, 16), (128, 16, 4), (256, 4, 8)]


def _plans(n, pr, pc, dtype, batch=1, mfma_terms=0):
    return [PencilPlan(n, dtype, (pr, pc), c, batch, mfma_terms=mfma_terms) for c in range(pc)]


@pytest.mark.parametrize("dtype,mfma", [(torch.float64, 0), (torch.float32, 0)],
                         ids=["f64", "f32"])
@pytest.mark.parametrize("n,pr,pc", CASES)
def test_pencil_forward_and_inverse(n, pr, pc, dtype, mfma):
    _pipeline(n, pr, pc, dtype, mfma)


def test_pencil_matrix_core_stage():
    """FP32 with the radix-16 stage of the y and x passes on the matrix
    cores (3 BF16 terms, FP32-level accuracy)."""
    _pipeline(64, 2, 4, torch.float32, 3)


def _pipeline(n, pr, pc, dtype, mfma):
    f, fref = real_input((n, n, n), 1200 + n + pr + pc, dtype)
    plans = _plans(n, pr, pc, dtype, mfma_terms=mfma)
    x, y = n // pr, n // pc
    g, h = max(pc // pr, 1), max(pr // pc, 1)
    F = oracle.r2c3d(fref)
    # step 1: z R2C into first-exchange order, per rank
    sends = {}
    for r in range(pr):
        for c in range(pc):
            part = f[r * x:(r + 1) * x, c * y:(c + 1) * y].contiguous().view(plans[c].real_shape)
            sends[r, c] = plans[c].z_r2c(part)
    torch.cuda.synchronize()
    zref = oracle.pencil_send(oracle.r2c_last(fref[:x, :y]), pc)
    assert rel_l2(host(sends[0, 0])[0], zref) <= TOL[dtype]
    # exchange 1 and the y pass
    ypen = {}
    for r in range(pr):
        for c in range(pc):
            yp = torch.empty(plans[c].ypencil_shape, dtype=plans[c].cdtype, device="cuda")
            for cp in range(pc):
                yp[:, cp].copy_(plans[cp].chunk(sends[r, cp], c))
            ypen[r, c] = plans[c].y_c2c(yp, -1)
    torch.cuda.synchronize()
    yref = oracle.pencil_y_c2c(oracle.pencil_exchange1(
        [oracle.pencil_send(oracle.r2c_last(fref[:x, c * y:(c + 1) * y]), pc) for c in range(pc)],
        x, y)[pc - 1], -1)
    assert rel_l2(host(ypen[0, pc - 1])[0], yref) <= TOL[dtype]
    # exchange 2 (through the pack when pr > pc) and the x pass
    xpen, send2 = {}, {}
    if h > 1:
        for key in ypen:
            send2[key] = plans[key[1]].pack2(ypen[key])
    for c in range(pc):
        for rp in range(pr):
            xp = torch.empty(plans[c].xpencil_shape, dtype=plans[c].cdtype, device="cuda")
            for r in range(pr):
                if h > 1:
                    xp[:, r].copy_(send2[r, c][:, rp // h, rp % h])
                else:
                    xp[:, r].copy_(ypen[r, c][:, rp * g:(rp + 1) * g])
            xpen[rp, c] = plans[c].x_c2c(xp, -1)
    torch.cuda.synchronize()
    for (rp, c), got in xpen.items():
        k0, k1 = oracle.pencil_kz_range(n, pc, c)
        if h > 1:
            r_, x_, y_, k_ = np.meshgrid(np.arange(pr), np.arange(x), np.arange(n // pr),
                                         np.arange(k1 - k0), indexing="ij")
            want = F[r_ * x + x_, rp * (n // pr) + y_, k0 + k_]
        else:
            r_, g_, x_, y_, k_ = np.meshgrid(np.arange(pr), np.arange(g), np.arange(x),
                                             np.arange(y), np.arange(k1 - k0), indexing="ij")
            want = F[r_ * x + x_, rp * (n // pr) + g_ * y + y_, k0 + k_]
        assert rel_l2(host(got)[0], want) <= TOL[dtype], (rp, c)
    # inverse: x^-1, exchange 2 back, y^-1, exchange 1 back, z C2R
    for key in xpen:
        plans[key[1]].x_c2c(xpen[key], +1)
    for c in range(pc):
        for r in range(pr):
            for rp in range(pr):
                if h > 1:
                    send2[r, c][:, rp // h, rp % h].copy_(xpen[rp, c][:, r])
                else:
                    ypen[r, c][:, rp * g:(rp + 1) * g].copy_(xpen[rp, c][:, r])
            if h > 1:
                plans[c].unpack2(send2[r, c], ypen[r, c])
            plans[c].y_c2c(ypen[r, c], +1)
    out = torch.empty_like(f)
    for r in range(pr):
        for cp in range(pc):
            back = torch.empty(plans[cp].send_shape, dtype=plans[cp].cdtype, device="cuda")
            for c in range(pc):
                plans[cp].chunk(back, c).copy_(ypen[r, c][:, cp])
            real = plans[cp].z_c2r(back, scale=1.0 / n ** 3)
            out[r * x:(r + 1) * x, cp * y:(cp + 1) * y] = real[0]
    torch.cuda.synchronize()
    assert rel_l2(host(out), fref) <= TOL[dtype]


def test_pencil_batch_and_weighted_z_pass():
    """batch = 2 grids back to back; the adjoint's bin weights on the z pass."""
    n, pr, pc = 32, 2, 4
    p = PencilPlan(n, torch.float64, (pr, pc), 1, batch=2)
    h, href = real_input(p.real_shape, 1300, torch.float64)
    out = p.z_r2c(h, scale=0.5, weighted=True)
    torch.cuda.synchronize()
    w = oracle.half_weights(n)
    want = oracle.pencil_send(0.5 * w * oracle.r2c_last(href), pc)
    assert rel_l2(host(out), want) <= 1e-13
    back = p.z_c2r(out.clone(), scale=1.0, weighted=True)
    torch.cuda.synchronize()
    # C2R(G / w) of w R2C(h) / 2 = n h / 2 along z
    assert rel_l2(host(back), 0.5 * n * href) <= 1e-13


def test_pencil_plan_rejects_slab_entry_points():
    p = PencilPlan(32, torch.float64, (2, 4), 0)
    a = torch.zeros(p.real_shape, dtype=torch.float64, device="cuda")
    b = torch.zeros(p.send_shape, dtype=torch.complex128, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert _lib.gfft_exec_r2c(p._h, a.data_ptr(), b.data_ptr(), s) == _lib.GFFT_E_UNSUPPORTED
    assert _lib.gfft_exec_c2r(p._h, b.data_ptr(), a.data_ptr(), 1.0, s) == _lib.GFFT_E_UNSUPPORTED
    assert (_lib.gfft_pack_slab_for_alltoall(p._h, b.data_ptr(), a.data_ptr(), s)
            == _lib.GFFT_E_UNSUPPORTED)
    sz = p.sizes
    assert sz["grid_r"] == 2 and sz["grid_c"] == 4 and sz["col"] == 0
    assert sz["kz_width"] == 4 and sz["y_local"] == 8 and sz["slab_x"] == 16
    assert sz["pencil_bytes"] == 4 * 16 * 8 * 4 * 16
    with pytest.raises(GfftError):
        PencilPlan(32, torch.float64, (4, 32), 0)         # pc > N/2
    yp = torch.zeros(p.ypencil_shape, dtype=torch.complex128, device="cuda")
    assert (_lib.gfft_pack_slab_for_alltoall(p._h, yp.data_ptr(), b.data_ptr(), s)
            == _lib.GFFT_E_UNSUPPORTED)                   # pr <= pc: nothing to pack


def test_pencil_pack2_bit_exact():
    """pr > pc: the second-exchange pack is the oracle's permutation, and
    unpack inverts it, bit for bit."""
    n, pr, pc = 64, 8, 2
    for dtype in (torch.float64, torch.float32):
        p = PencilPlan(n, dtype, (pr, pc), 1, batch=2)
        yp, ypref = cplx_input(p.ypencil_shape, 1330, dtype)
        send = p.pack2(yp)
        back = p.unpack2(send)
        torch.cuda.synchronize()
        assert np.array_equal(host(send), oracle.pencil_pack2(host(yp), p.h))
        assert torch.equal(back, yp)


@pytest.mark.parametrize("col", [0, 31])
def test_pencil_4096_share_sampled(col):
    """Rank (0, col) of 16 x 32 on 4096^3 FP64, the size the benchmark
    times: each pass on seeded input, checked on sampled rows and lines
    that the oracle transforms one by one."""
    import synth
    n, pr, pc = 4096, 16, 32
    p = PencilPlan(n, torch.float64, (pr, pc), col)
    x, y, w, g = p.x, p.y, p.w, p.g
    rng = np.random.default_rng(77 + col)
    # z pass: rows -> first-exchange order
    xr = synth.uniform(p.real_shape, 21, torch.float64, "cuda")
    send = p.z_r2c(xr)
    torch.cuda.synchronize()
    for _ in range(6):
        xl, yl = int(rng.integers(x)), int(rng.integers(y))
        row = xr[0, xl, yl].cpu().numpy()
        ref = oracle.r2c_last(row)
        got = np.empty_like(ref)
        for c in range(pc):
            k0, k1 = oracle.pencil_kz_range(n, pc, c)
            got[k0:k1] = p.chunk(send, c)[0, xl, yl].cpu().numpy()
        assert rel_l2(got, ref) <= 1e-13
    del xr, send
    # y pass on a seeded y-pencil: line (x_l, kz_l) runs over (c', y_l)
    yp = torch.view_as_complex(synth.uniform(p.ypencil_shape + (2,), 22, torch.float64, "cuda"))
    y0 = yp.clone()
    p.y_c2c(yp, -1)
    torch.cuda.synchronize()
    for _ in range(6):
        xl, kl = int(rng.integers(x)), int(rng.integers(w))
        line = y0[0, :, xl, :, kl].reshape(-1).cpu().numpy()
        ref = oracle.c2c_axis(line, 0, -1)
        assert rel_l2(yp[0, :, xl, :, kl].reshape(-1).cpu().numpy(), ref) <= 1e-13
    del yp, y0
    # x pass on a seeded x-pencil: line (g_l, y_l, kz_l) runs over (r, x_l)
    xp = torch.view_as_complex(synth.uniform(p.xpencil_shape + (2,), 23, torch.float64, "cuda"))
    x0 = xp.clone()
    p.x_c2c(xp, -1)
    torch.cuda.synchronize()
    for _ in range(6):
        gl, yl, kl = int(rng.integers(g)), int(rng.integers(y)), int(rng.integers(w))
        line = x0[0, :, gl, :, yl, kl].reshape(-1).cpu().numpy()
        ref = oracle.c2c_axis(line, 0, -1)
        assert rel_l2(xp[0, :, gl, :, yl, kl].reshape(-1).cpu().numpy(), ref) <= 1e-13
    del xp, x0
    torch.cuda.empty_cache()


@pytest.mark.parametrize("grid", [(2, 4), (8, 2)])
def test_pencil_batched_y_and_x_passes(grid):
    """batch = 3 grids back to back through the y and x passes (and the
    second-exchange pack for pr > pc), each grid against the oracle."""
    n, (pr, pc) = 32, grid
    for dtype in (torch.float64, torch.float32):
        p = PencilPlan(n, dtype, (pr, pc), pc - 1, batch=3)
        yp, ypref = cplx_input(p.ypencil_shape, 1500 + pr, dtype)
        p.y_c2c(yp, +1)
        xp, xpref = cplx_input(p.xpencil_shape, 1510 + pr, dtype)
        p.x_c2c(xp, -1)
        torch.cuda.synchronize()
        for b in range(3):
            assert rel_l2(host(yp)[b], oracle.pencil_y_c2c(ypref[b], +1)) <= TOL[dtype]
            if p.h > 1:
                want = oracle.x_c2c(xpref[b].reshape(n, n // pr, -1), -1).reshape(xpref[b].shape)
            else:
                want = oracle.pencil_x_c2c(xpref[b], -1)
            assert rel_l2(host(xp)[b], want) <= TOL[dtype]
        if p.h > 1:
            send = p.pack2(yp)
            torch.cuda.synchronize()
            assert np.array_equal(host(send), oracle.pencil_pack2(host(yp), p.h))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("col", [0, 3])
def test_pencil_512_y_pass(dtype, col):
    """N = 512 y pencils (the FP32 tile of 16 columns, the FP64 tile with the
    split exchange), kz widths 64 and 65 (ragged last tile)."""
    n, pr, pc = 512, 2, 4
    p = PencilPlan(n, dtype, (pr, pc), col)
    yp, ypref = cplx_input(p.ypencil_shape, 1700 + col, dtype)
    p.y_c2c(yp, -1)
    torch.cuda.synchronize()
    assert rel_l2(host(yp)[0], oracle.pencil_y_c2c(ypref[0], -1)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_pencil_x_pass_streaming_kernel(dtype):
    """N = 512: the pencil x-pencil's strides are whole 128-byte lines, so
    the x pass takes its non-temporal kernel; checked against the oracle."""
    n, pr, pc = 512, 2, 4
    p = PencilPlan(n, dtype, (pr, pc), pc - 1)
    assert (p.y * p.w * (16 if dtype == torch.float64 else 8)) % 128 == 0
    xp, xpref = cplx_input(p.xpencil_shape, 1600, dtype)
    p.x_c2c(xp, +1)
    torch.cuda.synchronize()
    assert rel_l2(host(xp)[0], oracle.pencil_x_c2c(xpref[0], +1)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("grid", [(2, 4), (8, 2)])
def test_pencil_pass_copy_conjugates(dtype, grid):
    """gfft_exec_pass_copy on a pencil plan reads and writes exactly the
    y-pencil (axis 0) and x-pencil (axis 1) that the y and x passes take."""
    n, (pr, pc) = 64, grid
    p = PencilPlan(n, dtype, grid, pc - 1)
    stream = torch.cuda.current_stream().cuda_stream
    for axis, shape in ((0, p.ypencil_shape), (1, p.xpencil_shape)):
        d, _ = cplx_input(shape, 1800 + axis, dtype)
        ref = d.conj().resolve_conj()
        assert _lib.gfft_exec_pass_copy(p._h, axis, d.data_ptr(), stream) == _lib.GFFT_OK
        torch.cuda.synchronize()
        assert torch.equal(d, ref)
