"""Pins of the oracle's adjoints, losses and slab-algorithm permutations."""
import numpy as np
import pytest

import oracle
import synth


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
                 / np.linalg.norm(np.asarray(b).ravel()))


def rand_real(shape, seed):
    return synth.uniform(shape, seed).numpy()


def rand_cplx(shape, seed):
    return rand_real(shape, seed) + 1j * rand_real(shape, seed + 1000)


def inner_half(F, G):
    """Real inner product over the stored half: sum Re(conj(F) G)."""
    return float(np.sum(np.real(np.conj(F) * G)))


# ---------------------------------------------------------------- P10 adjoints

@pytest.mark.parametrize("n", [4, 8, 16])
def test_p10_adjoint_dot_r2c(n):
    f = rand_real((n, n, n), 101)
    G = rand_cplx((n, n, n // 2 + 1), 102)
    lhs = inner_half(oracle.r2c3d(f), G)
    rhs = float(np.sum(f * oracle.r2c3d_adjoint(G, n)))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) + 1e-12


@pytest.mark.parametrize("n", [4, 8, 16])
def test_p10_adjoint_dot_c2r(n):
    G = rand_cplx((n, n, n // 2 + 1), 103)
    h = rand_real((n, n, n), 104)
    lhs = float(np.sum(oracle.c2r3d(G, n) * h))
    rhs = inner_half(G, oracle.c2r3d_adjoint(h))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) + 1e-12


def test_p10_c2r_is_not_the_adjoint_of_r2c():
    """The unweighted C2R fails the dot test: the weights matter."""
    n = 8
    f = rand_real((n, n, n), 105)
    G = rand_cplx((n, n, n // 2 + 1), 106)
    lhs = inner_half(oracle.r2c3d(f), G)
    wrong = float(np.sum(f * oracle.c2r3d(G, n)))
    assert abs(lhs - wrong) > 1e-3 * abs(lhs)


def test_p10_adjoint_matrix_transpose():
    """Adjoint equals the transpose of the explicit real matrix (N = 4)."""
    n = 4
    nr, nc = n ** 3, n * n * (n // 2 + 1)
    A = np.zeros((2 * nc, nr))
    for i in range(nr):
        e = np.zeros(nr)
        e[i] = 1.0
        F = oracle.r2c3d(e.reshape(n, n, n)).ravel()
        A[:nc, i], A[nc:, i] = F.real, F.imag
    for q in range(2 * nc):
        v = np.zeros(nc, dtype=complex)
        if q < nc:
            v[q] = 1.0
        else:
            v[q - nc] = 1.0j
        col = oracle.r2c3d_adjoint(v.reshape(n, n, n // 2 + 1), n).ravel()
        assert np.max(np.abs(col - A[q])) <= 1e-13


# ---------------------------------------------------------------- P11, P12

def _cos_field(n, k0):
    j = np.indices((n, n, n))
    return np.cos(2 * np.pi * (k0[0] * j[0] + k0[1] * j[1] + k0[2] * j[2]) / n)


def test_p11_energy_loss_closed_form():
    n, k0 = 16, (1, -2, 3)
    u = _cos_field(n, k0)
    k2 = sum(c * c for c in k0)
    # |u_hat|^2 = (N^3/2)^2 at +k0 and -k0, each with weight |k0|^2
    assert abs(oracle.energy_loss(u) - 2 * k2 * (n ** 3 / 2) ** 2) <= 1e-6
    g = oracle.energy_loss_grad(u)
    assert rel_l2(g, 2 * k2 * n ** 3 * u) <= 1e-13


@pytest.mark.parametrize("which", ["energy", "poisson"])
def test_p11_finite_differences_and_euler(which):
    n = 8
    u = rand_real((n, n, n), 111)
    if which == "energy":
        L, dL = oracle.energy_loss, oracle.energy_loss_grad
    else:
        L, dL = oracle.poisson_loss, oracle.poisson_loss_grad
    g = dL(u)
    # Euler's theorem for a quadratic form: <grad L, u> = 2 L
    assert abs(np.sum(g * u) - 2 * L(u)) <= 1e-12 * abs(L(u))
    eps = 1e-3
    for s in range(4):
        d = rand_real((n, n, n), 120 + s)
        fd = (L(u + eps * d) - L(u - eps * d)) / (2 * eps)
        assert abs(fd - np.sum(g * d)) <= 1e-8 * max(1.0, abs(fd))


def test_p12_poisson_closed_form_and_self_adjoint():
    n, a = 16, (2, 1, -3)
    j = np.indices((n, n, n))
    f = np.sin(2 * np.pi * (a[0] * j[0] + a[1] * j[1] + a[2] * j[2]) / n)
    u = oracle.poisson(f)
    assert rel_l2(u, -f / sum(c * c for c in a)) <= 1e-13
    f1 = rand_real((n, n, n), 131)
    f2 = rand_real((n, n, n), 132)
    l = np.sum(oracle.poisson(f1) * f2)
    r = np.sum(f1 * oracle.poisson(f2))
    assert abs(l - r) <= 1e-13 * abs(l)


# ---------------------------------------------------------------- P13 slab

@pytest.mark.parametrize("p", [1, 2, 4, 8])
@pytest.mark.parametrize("paper_order", [False, True])
def test_p13_pack_is_a_permutation(p, paper_order):
    n, x = 16, 4
    s = rand_cplx((x, n, n // 2 + 1), 141)
    send = oracle.pack_slab(s, p, paper_order)
    y = n // p
    for j in range(p):
        for xl in range(x):
            for yl in range(y):
                row = send[j, yl, xl] if paper_order else send[j, xl, yl]
                assert np.array_equal(row, s[xl, j * y + yl])
    assert np.array_equal(oracle.unpack_slab(send, paper_order), s)


@pytest.mark.parametrize("p", [2, 4, 8])
def test_p13_virtual_ranks_match_full_grid(p):
    """Steps 1-5 run rank by rank on one host reproduce the full transform,
    and the reversed steps give back the field."""
    n = 16
    f = rand_real((n, n, n), 151)
    full = oracle.r2c3d(f)
    xs = n // p
    sends = [oracle.pack_slab(oracle.r2c2d_planes(f[r * xs:(r + 1) * xs]), p)
             for r in range(p)]
    recv = oracle.exchange(sends)
    outs = [oracle.x_c2c(rv.reshape(n, xs, n // 2 + 1), -1) for rv in recv]
    got = np.concatenate(outs, axis=1)          # [kx][ky = r*Y + ky_l][kz]
    assert rel_l2(got, full) <= 1e-13
    # inverse in reverse order
    back_recv = [oracle.x_c2c(o, +1).reshape(p, xs, xs, n // 2 + 1)
                 for o in outs]
    back_send = oracle.exchange(back_recv)
    planes = [oracle.c2r2d_planes(oracle.unpack_slab(bs), n, 1.0 / n ** 3)
              for bs in back_send]
    assert rel_l2(np.concatenate(planes, axis=0), f) <= 1e-13


def test_kz_planes_sample():
    n = 16
    f = rand_real((n, n, n), 161)
    full = oracle.r2c3d(f)
    kz = [0, 1, 5, n // 2]
    got = oracle.r2c3d_kz_planes(f, kz)
    assert rel_l2(got, full[:, :, kz]) <= 1e-13
