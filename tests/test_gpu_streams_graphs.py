"""Stream and graph behaviour the C ABI promises: exec calls only enqueue
kernels on the given stream, so one plan serves concurrent streams with
disjoint buffers, and a captured sequence of exec calls replays exactly."""
import pytest
import torch

from helpers import real_input
from paper_2202_12756_amd import Plan, PencilPlan

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_one_plan_on_two_streams(dtype):
    n = 128
    p = Plan(n, dtype, batch=2)
    xa, _ = real_input(p.real_shape, 1400, dtype)
    xb, _ = real_input(p.real_shape, 1401, dtype)
    ref_a, ref_b = p.r2c(xa), p.r2c(xb)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for _ in range(3):
        Fa, Fb = p.empty_spectrum(), p.empty_spectrum()
        sa.wait_stream(torch.cuda.current_stream())
        sb.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(sa):
            p.r2c(xa, Fa)
        with torch.cuda.stream(sb):
            p.r2c(xb, Fb)
        torch.cuda.current_stream().wait_stream(sa)
        torch.cuda.current_stream().wait_stream(sb)
        outs.append((Fa, Fb))
    torch.cuda.synchronize()
    for Fa, Fb in outs:
        assert torch.equal(Fa, ref_a) and torch.equal(Fb, ref_b)


def _capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_graph_replays_match_eager_round_trip(dtype):
    """Forward + inverse captured once, replayed several times with eager
    work and synchronizations in between; every replay is bit-identical to
    the eager run."""
    n = 64
    p = Plan(n, dtype, batch=2)
    x, _ = real_input(p.real_shape, 1410, dtype)
    F, y = p.empty_spectrum(), p.empty_real()
    p.r2c(x, F)
    F_fwd = F.clone()
    p.c2r(F, y, 1.0 / n ** 3)
    y_ref, F_ref = y.clone(), F.clone()
    torch.cuda.synchronize()
    g = _capture(lambda: (p.r2c(x, F), p.c2r(F, y, 1.0 / n ** 3)))
    for _ in range(4):
        F.zero_()
        y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref) and torch.equal(F, F_ref)
    # the forward alone, captured, gives the eager spectrum
    g2 = _capture(lambda: p.r2c(x, F))
    for _ in range(2):
        F.zero_()
        g2.replay()
        torch.cuda.synchronize()
        assert torch.equal(F, F_fwd)


def test_graph_replays_of_a_pencil_chain():
    n = 64
    p = PencilPlan(n, torch.float64, (2, 4), 3)
    x, _ = real_input(p.real_shape, 1420, torch.float64)
    send = torch.empty(p.send_shape, dtype=torch.complex128, device="cuda")
    yp = torch.zeros(p.ypencil_shape, dtype=torch.complex128, device="cuda")

    def chain():
        p.z_r2c(x, send)
        yp[:, 3].copy_(p.chunk(send, 3))
        p.y_c2c(yp, -1)

    chain()
    ref = yp.clone()
    torch.cuda.synchronize()
    g = _capture(chain)
    for _ in range(3):
        yp.zero_()
        send.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(yp, ref)
