"""Error paths that need a live plan, degenerate inputs, and the largest full
grids one GPU holds (2048^3 FP64, 137 GB; 2048^3 FP32), checked by closed forms."""
import math

import numpy as np
import pytest
import torch

import oracle
from helpers import cplx_input, host, real_input, rel_l2
from paper_2202_12756_amd import GfftError, Plan, _lib

pytestmark = pytest.mark.gpu


def _stream():
    return torch.cuda.current_stream().cuda_stream


def test_exec_rejects_bad_pointers_and_arguments():
    n = 32
    p = Plan(n, torch.float64)
    x = torch.zeros(p._nreal() + 2, dtype=torch.float64, device="cuda")
    F = torch.zeros(p._ncplx() + 1, dtype=torch.complex128, device="cuda")
    s = _stream()
    base_x, base_f = x.data_ptr(), F.data_ptr()
    assert _lib.gfft_exec_r2c(p._h, base_x + 8, base_f, s) == _lib.GFFT_E_ALIGN
    assert _lib.gfft_exec_r2c(p._h, base_x, base_f + 8, s) == _lib.GFFT_E_ALIGN
    assert _lib.gfft_exec_r2c(p._h, None, base_f, s) == _lib.GFFT_E_INVALID_ARG
    # overlapping input and output
    assert _lib.gfft_exec_r2c(p._h, base_f, base_f + 16, s) == _lib.GFFT_E_INVALID_ARG
    assert _lib.gfft_exec_c2r(p._h, base_f, base_f + 16, 1.0, s) == _lib.GFFT_E_INVALID_ARG
    assert _lib.gfft_exec_c2r(p._h, base_f, base_x, float("nan"), s) == _lib.GFFT_E_INVALID_ARG
    assert _lib.gfft_exec_c2r(p._h, base_f, base_x, float("inf"), s) == _lib.GFFT_E_INVALID_ARG
    assert _lib.gfft_exec_x_c2c(p._h, base_f, 0, s) == _lib.GFFT_E_INVALID_ARG
    assert _lib.gfft_exec_y_c2c(p._h, base_f, 2, s) == _lib.GFFT_E_INVALID_ARG
    assert _lib.gfft_pack_slab_for_alltoall(p._h, base_f, base_f, s) == _lib.GFFT_E_INVALID_ARG
    torch.cuda.synchronize()
    # the Python layer checks what the ABI cannot see
    with pytest.raises(ValueError):
        p.r2c(torch.zeros(5, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        p.r2c(torch.zeros(p.real_shape, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        p.r2c(torch.zeros((n, n, n, 1), dtype=torch.float64, device="cuda")[..., 0].transpose(0, 2))
    with pytest.raises(GfftError):
        Plan(48, torch.float64)


def test_plan_device_fixed_at_creation():
    # a plan made without a device belongs to the device current at creation;
    # its calls run with that device current, on its current stream
    p = Plan(16, torch.float64)
    assert p.device == torch.device("cuda", torch.cuda.current_device())
    x = torch.zeros(p.real_shape, dtype=torch.float64, device="cuda")
    x[0, 0, 0, 0] = 1.0
    F = p.r2c(x)
    torch.cuda.synchronize()
    assert torch.equal(F, torch.ones_like(F))      # transform of a delta at the origin
    with pytest.raises(ValueError):
        p.r2c(x.cpu())


def test_plan_query_sizes():
    p = Plan(64, torch.float32, slab_x=16, batch=3)
    sz = p.sizes
    assert sz["ranks"] == 4 and sz["k"] == 33 and sz["batch"] == 3
    assert sz["real_bytes"] == 3 * 16 * 64 * 64 * 4
    assert sz["complex_bytes"] == 3 * 16 * 64 * 33 * 8
    assert sz["pencil_bytes"] == 3 * 64 * 16 * 33 * 8
    assert sz["chunk_bytes"] == 16 * 16 * 33 * 8


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_degenerate_inputs(dtype):
    n = 64
    p = Plan(n, dtype)
    z = p.r2c(torch.zeros(p.real_shape, dtype=dtype, device="cuda"))
    assert torch.count_nonzero(z).item() == 0
    c = p.r2c(torch.full(p.real_shape, 0.5, dtype=dtype, device="cuda"))
    ch = host(c)[0]
    assert abs(ch[0, 0, 0] - 0.5 * n ** 3) <= 1e-12 * n ** 3
    ch[0, 0, 0] = 0
    assert np.max(np.abs(ch)) <= (1e-9 if dtype == torch.float64 else 5e-2)
    # delta at the origin: a flat spectrum
    d = torch.zeros(p.real_shape, dtype=dtype, device="cuda")
    d[0, 0, 0, 0] = 1.0
    dh = host(p.r2c(d))
    assert np.max(np.abs(dh - 1.0)) <= (1e-14 if dtype == torch.float64 else 1e-6)
    # Nyquist-only field (-1)^(x+y+z): all energy in the (N/2, N/2, N/2) bin
    j = torch.arange(n, device="cuda")
    alt = ((j[:, None, None] + j[None, :, None] + j[None, None, :]) % 2) * -2.0 + 1.0
    ah = host(p.r2c(alt.to(dtype).reshape(p.real_shape)))[0]
    assert abs(ah[n // 2, n // 2, n // 2] - n ** 3) <= 1e-9 * n ** 3
    ah[n // 2, n // 2, n // 2] = 0
    assert np.max(np.abs(ah)) <= (1e-9 if dtype == torch.float64 else 1e-1)


def test_inverse_of_a_single_nonhermitian_bin():
    """C2R keeps only the real part of kz = 0 and kz = N/2 bins (reading R3)."""
    n = 32
    p = Plan(n, torch.float64)
    G = torch.zeros(p.spectrum_shape, dtype=torch.complex128, device="cuda")
    G[0, 3, 5, 0] = 2.0 + 7.0j          # kz = 0: Im is dropped by C2R
    G[0, 1, 2, n // 2] = -1.0 + 4.0j    # kz = N/2: Im dropped too
    G[0, 2, 0, 3] = 0.25 - 0.5j         # interior bin: weight 2
    out = host(p.c2r(G.clone()))[0]
    ref = oracle.c2r3d(host(G)[0], n)
    assert rel_l2(out, ref) <= 1e-13


def _plane_wave(n, k0, out):
    """cos(2 pi k0.j / N) into `out` [1, N, N, N] (FP64 phases, exact mod N)."""
    j = torch.arange(n, dtype=torch.float64, device="cuda")
    for x0 in range(0, n, 64):
        xs = j[x0:x0 + 64]
        ph = (k0[0] * xs[:, None, None] + k0[1] * j[None, :, None]
              + k0[2] * j[None, None, :]) % n
        out[0, x0:x0 + 64] = torch.cos(ph * (2 * math.pi / n)).to(out.dtype)


# tolerances: peak error and off-peak residual relative to the peak N^3/2,
# Parseval's relative mismatch, round-trip relative L2
_CLOSED_TOL = {torch.float64: (1e-12, 1e-13, 1e-12, 1e-13),
               torch.float32: (5e-6, 5e-6, 1e-5, 5e-6)}


@pytest.mark.parametrize("n,dtype", [(1024, torch.float64), (2048, torch.float64),
                                     (2048, torch.float32)], ids=["1024-f64", "2048-f64", "2048-f32"])
def test_largest_full_grid_closed_forms(n, dtype):
    """The largest full grids one GPU holds (2048^3 FP64: 137 GB of buffers),
    checked without a host oracle: a plane wave's exact spectrum (N^3/2 at k0,
    nothing elsewhere in the stored half), then Parseval and the round trip
    on a seeded field.  Reductions run in slabs, in FP64, to keep temporaries
    small and the sums exact enough for the FP64 bounds."""
    import synth

    t_peak, t_res, t_pars, t_rt = _CLOSED_TOL[dtype]
    k0 = (3, n - 5, 7)
    p = Plan(n, dtype)
    f = torch.empty(p.real_shape, dtype=dtype, device="cuda")
    _plane_wave(n, k0, f)
    F = p.r2c(f)
    peak = complex(F[0, k0[0], k0[1], k0[2]].item())
    assert abs(peak - n ** 3 / 2) <= t_peak * n ** 3 / 2
    F[0, k0[0], k0[1], k0[2]] = 0
    resid = math.sqrt(sum(torch.sum(F[0, s:s + 64].abs().double() ** 2).item()
                          for s in range(0, n, 64)))
    print(f"{n}^3 {dtype} plane wave: peak error {abs(peak - n ** 3 / 2):.3e}, "
          f"residual / peak {resid / (n ** 3 / 2):.3e}")
    assert resid <= t_res * n ** 3 / 2
    # Parseval and the round trip on seeded uniform data
    for s in range(0, n, 128):
        f[0, s:s + 128] = synth.uniform((128, n, n), 9, dtype, "cuda", offset=s * n * n)
    p.r2c(f, F)
    w = torch.full((n // 2 + 1,), 2.0, dtype=torch.float64, device="cuda")
    w[0] = 1
    w[-1] = 1
    e_phys = sum(torch.sum(f[0, s:s + 64].double() ** 2).item() for s in range(0, n, 64))
    e_spec = sum(torch.sum(w * F[0, s:s + 64].abs().double() ** 2).item()
                 for s in range(0, n, 64)) / n ** 3
    assert abs(e_phys - e_spec) <= t_pars * e_phys
    y = torch.empty_like(f)          # 2048^3 FP64: f, F and y hold 206 GB
    p.c2r(F, y, scale=1.0 / n ** 3)
    num = sum(torch.sum((y[0, s:s + 64].double() - f[0, s:s + 64].double()) ** 2).item()
              for s in range(0, n, 64))
    rt = math.sqrt(num / e_phys)
    print(f"{n}^3 {dtype}: Parseval rel {abs(e_phys - e_spec) / e_phys:.3e}, round trip {rt:.3e}")
    assert rt <= t_rt
    del f, F, y, p
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_line_alignment_paths_agree(dtype):
    """x lines take non-temporal loads and stores only when every tile owns
    whole 128-byte lines; a spectrum 16 bytes off a line boundary takes the
    plain kernel.  The arithmetic is the same, so the results are identical."""
    n = 512
    p = Plan(n, dtype)
    f, _ = real_input(p.real_shape, 77, dtype)
    F1 = p.r2c(f)
    shift = 16 // (16 if dtype == torch.float64 else 8)          # 16 bytes in complex values
    buf = torch.empty(p._ncplx() + 16, dtype=p.cdtype, device="cuda")
    assert buf.data_ptr() % 128 == 0
    F2 = buf[shift:shift + p._ncplx()].view(p.spectrum_shape)
    assert F2.data_ptr() % 128 == 16
    p.r2c(f, F2)
    torch.cuda.synchronize()
    assert torch.equal(F1, F2)
    y1 = p.c2r(F1, scale=1.0 / n ** 3)
    y2 = p.c2r(F2, scale=1.0 / n ** 3)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


@pytest.mark.parametrize("nbytes", [16, 4096, 16 * 1000003, (1 << 28) + 48])
def test_device_copy_is_bit_exact(nbytes):
    """The bandwidth yardstick copies every byte (ragged lengths included) and
    nothing past the end."""
    from paper_2202_12756_amd import device_copy

    src = torch.randint(-2 ** 62, 2 ** 62, (nbytes // 8,), dtype=torch.int64, device="cuda")
    dst = torch.full((nbytes // 8 + 2,), -1, dtype=torch.int64, device="cuda")
    device_copy(dst[: nbytes // 8], src)
    torch.cuda.synchronize()
    assert torch.equal(dst[: nbytes // 8], src)
    assert torch.equal(dst[nbytes // 8:], torch.full((2,), -1, dtype=torch.int64, device="cuda"))
    with pytest.raises(ValueError):
        device_copy(dst[:3], src)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n,x", [(64, 64), (256, 256), (1024, 2)])
def test_pass_copy_conjugates_in_place(n, x, dtype):
    """gfft_exec_pass_copy reads and writes exactly the elements of the y
    (axis 0) and x (axis 1) passes, storing each one's conjugate: bit-exact,
    on full grids (the x pass's streaming kernel at N = 256 in FP32) and a
    1024-point slab (ragged 16-column tiles)."""
    p = Plan(n, dtype, slab_x=x) if x < n else Plan(n, dtype)
    g, _ = cplx_input(p.spectrum_shape, 4300 + n, dtype)
    ref = g.conj().resolve_conj()
    p.pass_copy(g, 0)
    torch.cuda.synchronize()
    assert torch.equal(g, ref)
    pen, _ = cplx_input(p.pencil_shape, 4400 + n, dtype)
    ref = pen.conj().resolve_conj()
    p.pass_copy(pen, 1)
    torch.cuda.synchronize()
    assert torch.equal(pen, ref)
    with pytest.raises(ValueError):
        p.pass_copy(g, 2)
    assert _lib.gfft_exec_pass_copy(p._h, 2, g.data_ptr(), 0) == _lib.GFFT_E_INVALID_ARG
