"""GPU parity of the hand-written adjoints and the autograd wrappers."""
import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, cplx_input, host, real_input, rel_l2
from paper_2202_12756_amd import Plan, irfft3, rfft3

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n", [16, 64])
def test_adjoints_match_oracle(n, dtype):
    p = Plan(n, dtype)
    g, gref = cplx_input(p.spectrum_shape, 400 + n, dtype)
    out = p.r2c_adjoint(g.clone(), scale=0.25)
    h, href = real_input(p.real_shape, 410 + n, dtype)
    out2 = p.c2r_adjoint(h, scale=3.0)
    torch.cuda.synchronize()
    assert rel_l2(host(out), 0.25 * oracle.r2c3d_adjoint(gref, n)) <= TOL[dtype]
    assert rel_l2(host(out2), 3.0 * oracle.c2r3d_adjoint(href)) <= TOL[dtype]


def test_adjoint_dot_products_fp64():
    n = 32
    p = Plan(n, torch.float64)
    f, _ = real_input(p.real_shape, 420, torch.float64)
    G, _ = cplx_input(p.spectrum_shape, 421, torch.float64)
    lhs = torch.sum(torch.real(torch.conj(p.r2c(f)) * G))
    rhs = torch.sum(f * p.r2c_adjoint(G.clone()))
    assert abs(float(lhs - rhs)) <= 1e-12 * abs(float(lhs))
    h, _ = real_input(p.real_shape, 422, torch.float64)
    lhs = torch.sum(p.c2r(G.clone()) * h)
    rhs = torch.sum(torch.real(torch.conj(G) * p.c2r_adjoint(h)))
    assert abs(float(lhs - rhs)) <= 1e-12 * abs(float(lhs))


def test_gradcheck_fp64():
    for n in (16,):
        p = Plan(n, torch.float64)
        u = torch.randn(p.real_shape, dtype=torch.float64, device="cuda",
                        generator=torch.Generator("cuda").manual_seed(5),
                        requires_grad=True)
        assert torch.autograd.gradcheck(lambda t: rfft3(t, p), (u,),
                                        eps=1e-6, atol=1e-8, rtol=1e-6,
                                        fast_mode=True)
        G = torch.randn(p.spectrum_shape, dtype=torch.complex128, device="cuda",
                        generator=torch.Generator("cuda").manual_seed(6),
                        requires_grad=True)
        assert torch.autograd.gradcheck(lambda t: irfft3(t, p, 0.5), (G,),
                                        eps=1e-6, atol=1e-8, rtol=1e-6,
                                        fast_mode=True)


def test_autograd_energy_loss_gradient():
    """dL1/du = 2 C2R(|k|^2 u_hat) against the oracle (FP64 and FP32)."""
    n = 32
    k2 = torch.from_numpy(oracle.k_squared(n))
    w = torch.from_numpy(oracle.half_weights(n))
    for dtype in (torch.float64, torch.float32):
        p = Plan(n, dtype)
        u0, uref = real_input(p.real_shape, 430, dtype)
        u = u0.clone().requires_grad_(True)
        F = rfft3(u, p)
        L = torch.sum((w * k2).to(dtype).cuda() * (F.real ** 2 + F.imag ** 2))
        L.backward()
        ref = oracle.energy_loss_grad(uref[0])
        assert rel_l2(host(u.grad)[0], ref) <= TOL[dtype]


def test_fp64_central_differences_energy_and_poisson():
    """Both spectral losses (energy and Poisson) through the FP64 autograd path: central differences
    (eps = 1e-3, exact for a quadratic loss up to rounding) along seeded
    uniform directions agree with the hand-written adjoint to 1e-8."""
    import synth
    n = 32
    p = Plan(n, torch.float64)
    k2 = torch.from_numpy(oracle.k_squared(n)).cuda()
    w = torch.from_numpy(oracle.half_weights(n)).cuda()
    m = torch.where(k2 > 0, -1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)),
                    torch.zeros_like(k2))

    def energy(u):
        F = rfft3(u, p)
        return torch.sum(w * k2 * (F.real ** 2 + F.imag ** 2))

    def poisson_loss(f):
        u = irfft3(m * rfft3(f, p), p, 1.0 / n ** 3)
        return torch.sum(u ** 2)

    for L, seed in ((energy, 230), (poisson_loss, 240)):
        u0, _ = real_input(p.real_shape, seed, torch.float64)
        u = u0.clone().requires_grad_(True)
        L(u).backward()
        eps = 1e-3
        with torch.no_grad():
            for s in range(3):
                d = synth.uniform(p.real_shape, seed + 1 + s, torch.float64, "cuda")
                fd = (L(u + eps * d).item() - L(u - eps * d).item()) / (2 * eps)
                an = torch.sum(u.grad * d).item()
                assert abs(fd - an) <= 1e-8 * max(1.0, abs(an)), (L.__name__, fd, an)


def test_adjoint_dot_products_at_1024():
    """Both adjoints at the benchmark size (1024^3 FP64, the launches the
    bench times), through the dot-product identities over all 2^30 points."""
    import synth
    n = 1024
    p = Plan(n, torch.float64)
    f = synth.uniform(p.real_shape, 31, torch.float64, "cuda")
    G = torch.view_as_complex(synth.uniform(p.spectrum_shape + (2,), 32, torch.float64, "cuda"))
    Ff = p.r2c(f)
    lhs = sum(torch.sum(torch.real(torch.conj(Ff[0, s:s + 64]) * G[0, s:s + 64])).item()
              for s in range(0, n, 64))
    del Ff
    At = p.r2c_adjoint(G.clone())
    rhs = sum(torch.sum(f[0, s:s + 64] * At[0, s:s + 64]).item() for s in range(0, n, 64))
    del At
    print(f"R2C adjoint identity at 1024^3: {lhs:.12e} vs {rhs:.12e}")
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    h = f                                   # reuse: any real field
    Cg = p.c2r(G.clone())
    lhs = sum(torch.sum(Cg[0, s:s + 64] * h[0, s:s + 64]).item() for s in range(0, n, 64))
    del Cg
    Bt = p.c2r_adjoint(h)
    rhs = sum(torch.sum(torch.real(torch.conj(G[0, s:s + 64]) * Bt[0, s:s + 64])).item()
              for s in range(0, n, 64))
    print(f"C2R adjoint identity at 1024^3: {lhs:.12e} vs {rhs:.12e}")
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    del Bt, G, f, p
    torch.cuda.empty_cache()
