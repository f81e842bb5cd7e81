"""GPU parity of the one-pass plane transform (step 1 of the method, the 2D
R2C over (y, z) of each x-plane, and its inverse, in one kernel per plane).

The exec calls of FP32 plans run it instead of the separate z and y passes
for N = 64 and 128 in both directions and for the N = 256 forward (at 256
the inverse is faster as separate passes; these tests cover it all the same).  Checked against the FP64 oracle (section 2
forward and inverse equations, the C2R on non-Hermitian input as its
w-weighted real part) in every row layout the z passes support (natural,
all-to-all send order, the paper's chunk order, the padded in-place rows),
with batches, with the adjoints' bin weights, and against the separate z and
y passes on the same input.  Tolerance: the FP32 rel-L2 bound of 5e-6.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, cplx_input, host, real_input, rel_l2
from paper_2202_12756_amd import Plan

pytestmark = pytest.mark.gpu

F32 = torch.float32
SIZES = [64, 128, 256]


def _planes(n):
    """x-planes of a slab (fewer than N, so exec_r2c stops after step 1):
    several workgroups, small for the oracle."""
    return {64: 16, 128: 8, 256: 4}[n]


@pytest.mark.parametrize("n", SIZES)
def test_forward_and_inverse_against_oracle(n):
    x = _planes(n)
    p = Plan(n, F32, slab_x=x, batch=2)
    xin, xref = real_input(p.real_shape, 9000 + n, F32)
    S = p.r2c(xin)
    torch.cuda.synchronize()
    assert rel_l2(host(S), oracle.r2c2d_planes(xref)) <= TOL[F32]
    # inverse on a non-Hermitian half spectrum (the kz = 0 and N/2 columns
    # included): only their Hermitian parts reach the real field
    g, gref = cplx_input(p.spectrum_shape, 9100 + n, F32)
    out = p.c2r(g, scale=0.5)
    torch.cuda.synchronize()
    assert rel_l2(host(out), 0.5 * oracle.c2r2d_planes(gref, n)) <= TOL[F32]


@pytest.mark.parametrize("n", SIZES)
def test_matches_the_separate_z_and_y_passes(n):
    x = _planes(n)
    p = Plan(n, F32, slab_x=x)
    xin, xref = real_input(p.real_shape, 9200 + n, F32)
    fused = p.r2c(xin)
    two = p.z_r2c(xin)
    p.y_c2c(two, -1)
    torch.cuda.synchronize()
    ref = oracle.r2c2d_planes(xref)
    assert rel_l2(host(fused), ref) <= TOL[F32]
    assert rel_l2(host(two), ref) <= TOL[F32]
    assert rel_l2(host(fused), host(two)) <= TOL[F32]
    g, _ = cplx_input(p.spectrum_shape, 9300 + n, F32)
    a = p.c2r(g.clone(), scale=1.0)
    g2 = g.clone()
    p.y_c2c(g2, +1)
    b = p.z_c2r(g2, scale=1.0)
    torch.cuda.synchronize()
    assert rel_l2(host(a), host(b)) <= TOL[F32]


@pytest.mark.parametrize("n", SIZES)
def test_full_grid_round_trip_and_adjoints(n):
    """Full grid (x pass included); 256^3 only through the round trip."""
    p = Plan(n, F32)
    xin, xref = real_input(p.real_shape, 9400 + n, F32)
    F = p.r2c(xin)
    back = p.c2r(F.clone(), scale=1.0 / n ** 3)
    torch.cuda.synchronize()
    assert rel_l2(host(back), xref) <= TOL[F32]
    if n > 128:
        return
    assert rel_l2(host(F), oracle.r2c3d(xref)) <= TOL[F32]
    g, gref = cplx_input(p.spectrum_shape, 9500 + n, F32)
    out = p.r2c_adjoint(g.clone(), scale=0.25)
    h, href = real_input(p.real_shape, 9600 + n, F32)
    out2 = p.c2r_adjoint(h, scale=3.0)
    torch.cuda.synchronize()
    assert rel_l2(host(out), 0.25 * oracle.r2c3d_adjoint(gref, n)) <= TOL[F32]
    assert rel_l2(host(out2), 3.0 * oracle.c2r3d_adjoint(href)) <= TOL[F32]


@pytest.mark.parametrize("paper", [False, True], ids=["send_order", "paper_order"])
@pytest.mark.parametrize("n,ranks", [(64, 4), (128, 8), (256, 64)])
def test_send_orders(n, ranks, paper):
    """The plane kernel stores and loads its rows through the same row map as
    the z passes: the fused pack and the paper's chunk order."""
    x = n // ranks
    p = Plan(n, F32, slab_x=x, fuse_pack=True, paper_order=paper)
    xin, xref = real_input(p.real_shape, 9700 + n, F32)
    send = p.r2c(xin)
    torch.cuda.synchronize()
    ref = oracle.pack_slab(oracle.r2c2d_planes(xref), ranks, paper_order=paper)
    assert rel_l2(host(send), ref) <= TOL[F32]
    back = p.c2r(send, scale=1.0 / (n * n))
    torch.cuda.synchronize()
    assert rel_l2(host(back), xref) <= TOL[F32]


@pytest.mark.parametrize("n,x,batch", [(64, 64, 2), (128, 16, 1), (256, 4, 2)])
def test_in_place_padded_rows(n, x, batch):
    p = Plan(n, F32, slab_x=x, batch=batch, inplace=True)
    buf = p.empty_inplace()
    xin, xref = real_input(p.real_shape, 9800 + n, F32)
    p.real_view(buf).copy_(xin)
    p.r2c_(buf)
    torch.cuda.synchronize()
    full = oracle.r2c3d(xref) if x == n else oracle.r2c2d_planes(xref)
    assert rel_l2(host(buf), full) <= TOL[F32]
    p.c2r_(buf, scale=1.0 / (n ** 3 if x == n else n * n))
    torch.cuda.synchronize()
    assert rel_l2(host(p.real_view(buf)), xref) <= TOL[F32]


def test_single_bins_of_the_real_columns():
    """kz = 0 and kz = N/2 travel through the kernel as one packed complex
    column: a lone bin in either, with its mirror -ky elsewhere, must come
    back alone and unmixed."""
    n = 256
    p = Plan(n, F32, slab_x=1)
    k = n // 2 + 1
    for kz in (0, n // 2):
        for ky in (0, 1, 77, n // 2):
            # forward of the inverse of a single real-field mode
            G = torch.zeros(p.spectrum_shape, dtype=torch.complex64, device="cuda")
            G[0, 0, ky, kz] = 1.0 + 0.5j
            f = p.c2r(G.clone(), scale=1.0)
            F = p.r2c(f)
            torch.cuda.synchronize()
            Gh = host(G)[0, 0]
            want = np.zeros((n, k), dtype=np.complex128)
            # the real field holds the Hermitian part of the bin; its forward
            # transform is N^2 times that part
            m = (-ky) % n
            want[ky, kz] += 0.5 * Gh[ky, kz]
            want[m, kz] += 0.5 * np.conj(Gh[ky, kz])
            want *= n * n
            got = host(F)[0, 0]
            assert np.max(np.abs(got - want)) <= 1e-5 * n * n, (kz, ky)
