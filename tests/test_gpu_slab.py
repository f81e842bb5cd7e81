"""GPU parity of the slab pipeline (section 3, steps 1-5) and its reverse.

Pack and unpack are integer permutations: compared bit for bit.  The
multi-rank pipeline is emulated on one GPU: every rank's slab runs in turn,
a host-free exchange copies chunk r of every send buffer to rank r, and the
assembled x-pencils are compared with the full-grid oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, cplx_input, host, real_input, rel_l2
from paper_2202_12756_amd import Plan

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n,p", [(16, 2), (64, 4), (64, 64), (128, 8), (256, 16)])
def test_pack_unpack_bit_exact(n, p, dtype):
    plan = Plan(n, dtype, slab_x=n // p, batch=2)
    s, sref = cplx_input((2, n // p, n, n // 2 + 1), 100 + n + p, dtype)
    send = plan.pack(s)
    back = plan.unpack(send)
    torch.cuda.synchronize()
    ref = oracle.pack_slab(host(s), p)
    assert np.array_equal(host(send), ref)
    assert torch.equal(back, s)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n,p", [(32, 2), (64, 8), (128, 4)])
def test_fused_pack_forward_and_inverse(n, p, dtype):
    x = n // p
    fused = Plan(n, dtype, slab_x=x, fuse_pack=True)
    plain = Plan(n, dtype, slab_x=x)
    xin, xref = real_input(fused.real_shape, 200 + n, dtype, )
    send = fused.r2c(xin)
    nat = plain.r2c(xin)
    torch.cuda.synchronize()
    ref = oracle.pack_slab(oracle.r2c2d_planes(xref), p)
    assert rel_l2(host(send), ref) <= TOL[dtype]
    # the fused store is the same permutation as the standalone pack
    assert torch.equal(plain.pack(nat), send)
    back = fused.c2r(send, scale=1.0 / (n * n))
    torch.cuda.synchronize()
    assert rel_l2(host(back), xref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n,p", [(32, 2), (64, 4), (64, 8), (256, 32)])
def test_virtual_ranks_match_full_grid(n, p, dtype):
    """(256, 32): chunks of N/p = 8 rows, fewer than the 16 threads that
    share a line, so each line element's offset splits between both levels
    of the send-order layout."""
    x = n // p
    k = n // 2 + 1
    f, fref = real_input((n, n, n), 300 + n + p, dtype)
    plans = Plan(n, dtype, slab_x=x, fuse_pack=True)
    sends = [plans.r2c(f[r * x:(r + 1) * x].contiguous()) for r in range(p)]
    recvs = []
    for r in range(p):
        recv = torch.empty((p, x, x, k), dtype=plans.cdtype, device="cuda")
        for i in range(p):
            recv[i].copy_(sends[i][0, r])           # chunk r of rank i
        recvs.append(recv)
    for recv in recvs:
        plans.x_c2c(recv, -1)                      # pencil [N][N/p][K]
    torch.cuda.synchronize()
    got = np.concatenate([host(rv).reshape(n, x, k) for rv in recvs], axis=1)
    assert rel_l2(got, oracle.r2c3d(fref)) <= TOL[dtype]
    # reverse: x^-1, exchange back, inverse 2D on each slab
    for recv in recvs:
        plans.x_c2c(recv, +1)
    out = []
    for r in range(p):
        back = torch.empty((1, p, x, x, k), dtype=plans.cdtype, device="cuda")
        for i in range(p):
            back[0, i].copy_(recvs[i][r])
        out.append(plans.c2r(back, scale=1.0 / n ** 3))
    torch.cuda.synchronize()
    assert rel_l2(np.concatenate([host(o)[0] for o in out]), fref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n,x,batch", [(16, 16, 1), (64, 64, 2), (128, 32, 1), (512, 2, 1),
                                         (1024, 2, 1)])
def test_inplace_padded_layout(n, x, batch, dtype):
    """FFTW-padded in-place R2C/C2R in one shared buffer (rows of N + 2)."""
    p = Plan(n, dtype, slab_x=x, batch=batch, inplace=True)
    buf = p.empty_inplace()
    f, fref = real_input((batch, x, n, n), 500 + n, dtype)
    p.real_view(buf).copy_(f)
    p.r2c_(buf)
    torch.cuda.synchronize()
    ref = (oracle.r2c3d(fref) if x == n else oracle.r2c2d_planes(fref))
    assert rel_l2(host(buf), ref) <= TOL[dtype]
    back = p.c2r_(buf, scale=1.0 / (n ** 3 if x == n else n * n))
    torch.cuda.synchronize()
    assert rel_l2(host(back), fref) <= TOL[dtype]
    # the adjoints in place
    G, gref = cplx_input(p.spectrum_shape, 510 + n, dtype)
    buf.copy_(G)
    out = p.r2c_adjoint_(buf, scale=2.0)
    torch.cuda.synchronize()
    adj = (oracle.r2c3d_adjoint(gref, n) if x == n
           else oracle.c2r2d_planes(gref / oracle.half_weights(n), n))
    assert rel_l2(host(out), 2.0 * adj) <= TOL[dtype]


def test_inplace_rejects_distinct_buffers():
    p = Plan(32, torch.float64, inplace=True)
    a, b = p.empty_inplace(), p.empty_inplace()
    from paper_2202_12756_amd import _lib
    s = torch.cuda.current_stream().cuda_stream
    assert _lib.gfft_exec_r2c(p._h, a.data_ptr(), b.data_ptr(), s) == _lib.GFFT_E_INVALID_ARG


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n,p", [(16, 2), (64, 8), (128, 4)])
def test_paper_order_pack_bit_exact(n, p, dtype):
    plan = Plan(n, dtype, slab_x=n // p, batch=2, paper_order=True)
    s, _ = cplx_input((2, n // p, n, n // 2 + 1), 600 + n + p, dtype)
    send = plan.pack(s)
    back = plan.unpack(send)
    torch.cuda.synchronize()
    assert np.array_equal(host(send), oracle.pack_slab(host(s), p, paper_order=True))
    assert torch.equal(back, s)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n,p", [(32, 2), (64, 4), (64, 8), (256, 32)])
def test_paper_order_virtual_ranks(n, p, dtype):
    """Steps 1-5 with the paper's wire format: the local xy transpose folded
    into the z pass, chunk transposes folded into the x pass."""
    x = n // p
    k = n // 2 + 1
    f, fref = real_input((n, n, n), 700 + n + p, dtype)
    plan = Plan(n, dtype, slab_x=x, fuse_pack=True, paper_order=True)
    sends = [plan.r2c(f[r * x:(r + 1) * x].contiguous()) for r in range(p)]   # [1,p,Y,X,K]
    torch.cuda.synchronize()
    ref2d = oracle.r2c2d_planes(fref[:x])
    assert rel_l2(host(sends[0])[0], oracle.pack_slab(ref2d, p, paper_order=True)) <= TOL[dtype]
    recvs = []
    for r in range(p):
        recv = torch.empty((1, p, x, x, k), dtype=plan.cdtype, device="cuda")
        for i in range(p):
            recv[0, i].copy_(sends[i][0, r])
        plan.x_c2c(recv, -1)
        recvs.append(recv)
    torch.cuda.synchronize()
    full = oracle.r2c3d(fref)                                   # [kx][ky][kz]
    for r, recv in enumerate(recvs):
        got = host(recv)[0]                                     # [i][ky_l][kx_l][kz]
        want = full[:, r * x:(r + 1) * x, :].reshape(p, x, x, k).transpose(0, 2, 1, 3)
        assert rel_l2(got, want) <= TOL[dtype]
    for recv in recvs:
        plan.x_c2c(recv, +1)
    outs = []
    for r in range(p):
        back = torch.empty((1, p, x, x, k), dtype=plan.cdtype, device="cuda")
        for i in range(p):
            back[0, i].copy_(recvs[i][0, r])
        outs.append(plan.c2r(back, scale=1.0 / n ** 3))
    torch.cuda.synchronize()
    assert rel_l2(np.concatenate([host(o)[0] for o in outs]), fref) <= TOL[dtype]
