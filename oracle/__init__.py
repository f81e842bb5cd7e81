"""CPU oracle for the slab-decomposed 3D real FFT.

TEST INFRASTRUCTURE ONLY: the plain FP64 reference the GPU library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it.  It shares no code with the GPU library and
never imports it.

The arithmetic lives in ``oracle.c`` (FP64, one line at a time, OpenMP over
lines); this module only composes the 1D transforms along the three axes and
writes out the index permutations of the slab algorithm with numpy reshapes.

Paper passages followed (Verma et al., "Scalable Multi-node Fast Fourier
Transform on GPUs"):
  * section 2, forward/inverse DFT equations: unnormalized sums with
    exp(-/+ 2 pi i k.j / N);
  * section 2, Hermitian symmetry of the transform of a real field: only
    kz = 0..N/2 is stored (FFTW convention, K = N/2 + 1);
  * section 2, slab decomposition: rank r owns x in [r N/p, (r+1) N/p);
  * section 3, steps 1-5 of the forward algorithm: 2D R2C on every yz plane,
    local xy transpose, all-to-all in chunks of (N/p) x (N/p) x K, chunk
    transpose, strided 1D C2C along x; the inverse runs them in reverse order;
  * section 2, pencil decomposition: a pr x pc grid of ranks holding
    (N/pr) x (N/pc) x N real values each (the spectral layouts of the two
    exchanges are the library's reading, written out below).

Every function here is unnormalized; ``scale`` arguments multiply results.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# ORACLE_LIB names another build of oracle.c (the sanitized build of the CPU
# tests); by default the in-tree liboracle.so
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB")
_lib = None

DIRECT = 0
RADIX2 = 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc and OpenMP."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
             "-shared", _SRC, "-o", tmp, "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        path = _LIB_OVERRIDE or _LIB
        if not _LIB_OVERRIDE and not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(path)
        i64, dp, ip = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        lib.oracle_c2c_axis.argtypes = [i64, i64, i64, dp, dp, ip, ip]
        lib.oracle_r2c_rows.argtypes = [i64, i64, dp, dp, ip]
        lib.oracle_c2r_rows.argtypes = [i64, i64, dp, dp, ip]
        lib.oracle_zsum_rows.argtypes = [i64, i64, dp, i64, dp, dp]
        for f in (lib.oracle_c2c_axis, lib.oracle_r2c_rows,
                  lib.oracle_c2r_rows, lib.oracle_zsum_rows):
            f.restype = ip
        lib.oracle_num_threads.restype = ip
        lib.oracle_set_num_threads.argtypes = [ip]
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _pick(method, n):
    if method is None:
        return RADIX2 if n & (n - 1) == 0 else DIRECT
    return method


def c2c_axis(a: np.ndarray, axis: int, sign: int, method=None) -> np.ndarray:
    """1D complex DFT along ``axis`` (sign -1 forward, +1 inverse), FP64."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    axis = axis % a.ndim
    n = a.shape[axis]
    b = int(np.prod(a.shape[:axis], dtype=np.int64))
    m = int(np.prod(a.shape[axis + 1:], dtype=np.int64))
    out = np.empty_like(a)
    rc = _load().oracle_c2c_axis(b, n, m, _ptr(a), _ptr(out), int(sign),
                                 _pick(method, n))
    if rc:
        raise ValueError("oracle_c2c_axis rejected its arguments")
    return out


def r2c_last(f: np.ndarray, method=None) -> np.ndarray:
    """Real rows of length N along the last axis -> K = N//2 + 1 complex bins."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    n = f.shape[-1]
    rows = int(np.prod(f.shape[:-1], dtype=np.int64))
    out = np.empty(f.shape[:-1] + (n // 2 + 1,), dtype=np.complex128)
    if _load().oracle_r2c_rows(rows, n, _ptr(f), _ptr(out), _pick(method, n)):
        raise ValueError("oracle_r2c_rows rejected its arguments")
    return out


def c2r_last(g: np.ndarray, n: int, method=None) -> np.ndarray:
    """Half-spectrum rows (K = n//2 + 1 bins) -> n reals, w-weighted real part."""
    g = np.ascontiguousarray(g, dtype=np.complex128)
    if g.shape[-1] != n // 2 + 1:
        raise ValueError("last axis must hold n//2 + 1 bins")
    rows = int(np.prod(g.shape[:-1], dtype=np.int64))
    out = np.empty(g.shape[:-1] + (n,), dtype=np.float64)
    if _load().oracle_c2r_rows(rows, n, _ptr(g), _ptr(out), _pick(method, n)):
        raise ValueError("oracle_c2r_rows rejected its arguments")
    return out


# --------------------------------------------------------------------------
# 3D transforms of a full grid (section 2 equations, real field, half along z)
# --------------------------------------------------------------------------

def r2c3d(f: np.ndarray, method=None) -> np.ndarray:
    """Forward DFT of a real [..., Nx, Ny, Nz] grid, kz = 0..Nz/2 kept.

    Separable evaluation: real-to-half along z, then complex DFT along y,
    then along x (leading axes, if any, are a batch).
    """
    g = r2c_last(f, method)
    g = c2c_axis(g, -2, -1, method)
    return c2c_axis(g, -3, -1, method)


def c2r3d(g: np.ndarray, n: int, scale: float = 1.0, method=None) -> np.ndarray:
    """Inverse DFT of a half spectrum [..., Nx, Ny, K] to a real grid.

    Inverse complex DFT along x, then y, then the w-weighted real part along
    z (the same order reversed, section 3).  Result times ``scale``.
    """
    h = c2c_axis(g, -3, +1, method)
    h = c2c_axis(h, -2, +1, method)
    f = c2r_last(h, n, method)
    if scale != 1.0:
        f *= scale
    return f


# --------------------------------------------------------------------------
# One rank's share of the slab algorithm (section 3, steps 1-5)
# --------------------------------------------------------------------------

def r2c2d_planes(slab: np.ndarray, method=None) -> np.ndarray:
    """Step 1: 2D R2C over (y, z) of every x-plane of a [..., X, N, N] slab."""
    g = r2c_last(slab, method)
    return c2c_axis(g, -2, -1, method)


def c2r2d_planes(g: np.ndarray, n: int, scale: float = 1.0,
                 method=None) -> np.ndarray:
    """Inverse of step 1: inverse DFT along y, then C2R along z, times scale."""
    h = c2c_axis(g, -2, +1, method)
    f = c2r_last(h, n, method)
    if scale != 1.0:
        f *= scale
    return f


def pack_slab(s: np.ndarray, p: int, paper_order: bool = False) -> np.ndarray:
    """Steps 2 and the chunking of step 3 as one permutation.

    ``s`` is a rank's [..., X, N, K] half spectrum.  Chunk j holds the
    wavenumbers ky in [j N/p, (j+1) N/p) of every local plane and is destined
    for rank j.  Default order inside a chunk: [x_l][ky_l][kz]; with
    ``paper_order`` the chunk holds [ky_l][x_l][kz], the order the paper's
    local xy transpose produces.  Output shape [..., p, X, N/p, K] (or
    [..., p, N/p, X, K]).
    """
    *lead, x, n, k = s.shape
    if n % p:
        raise ValueError("p must divide N")
    y = n // p
    t = s.reshape(*lead, x, p, y, k)
    nl = len(lead)
    # [.., x, j, y_l, k] -> [.., j, x, y_l, k]
    perm = list(range(nl)) + [nl + 1, nl, nl + 2, nl + 3]
    if paper_order:
        perm = list(range(nl)) + [nl + 1, nl + 2, nl, nl + 3]
    return np.ascontiguousarray(t.transpose(perm))


def unpack_slab(send: np.ndarray, paper_order: bool = False) -> np.ndarray:
    """Inverse permutation of :func:`pack_slab`."""
    *lead, p, a, b, k = send.shape
    nl = len(lead)
    if paper_order:   # [j, y_l, x, k] -> [x, j, y_l, k]
        perm = list(range(nl)) + [nl + 2, nl, nl + 1, nl + 3]
        x, y = b, a
    else:             # [j, x, y_l, k] -> [x, j, y_l, k]
        perm = list(range(nl)) + [nl + 1, nl, nl + 2, nl + 3]
        x, y = a, b
    t = np.ascontiguousarray(send.transpose(perm))
    return t.reshape(*lead, x, p * y, k)


def exchange(sends: list[np.ndarray]) -> list[np.ndarray]:
    """Step 3 on one host: rank r receives chunk r of every rank's send buffer.

    ``sends[i]`` is rank i's [p, X, Y, K] buffer (default order).  The chunk
    keeps its internal order; chunk order equals rank order.  Returns, per
    rank r, the received [p, X, Y, K] buffer, which read as [N, Y, K] (x
    slowest) is the x-pencil of step 5 with no chunk transpose needed.
    """
    p = len(sends)
    return [np.stack([sends[i][r] for i in range(p)]) for r in range(p)]


def x_c2c(pencil: np.ndarray, sign: int, method=None) -> np.ndarray:
    """Step 5: strided batched 1D DFT along x of an [..., N, Y, K] pencil."""
    return c2c_axis(pencil, -3, sign, method)


# --------------------------------------------------------------------------
# Pencil decomposition (section 2): p = pr x pc ranks, rank (r, c) holding
# the (N/pr) x (N/pc) x N real values x in [r X, (r+1) X), y in [c Y,
# (c+1) Y).  The paper names this decomposition but fixes none of its
# spectral layouts; the ones written out here are the library's reading
# (pr <= pc <= N/2): two exchanges, kz cut across the grid columns.
# --------------------------------------------------------------------------

def pencil_kz_range(n: int, pc: int, c: int) -> tuple[int, int]:
    """Bins [k0, k1) of kz that grid column c holds after exchange 1: N/(2 pc)
    bins each, and the Nyquist bin kz = N/2 with the last column."""
    w0 = n // (2 * pc)
    return c * w0, (c + 1) * w0 + (1 if c == pc - 1 else 0)


def pencil_send(rows: np.ndarray, pc: int) -> np.ndarray:
    """First-exchange order of a rank's half-spectrum rows [..., X, Y, K]:
    chunk c' (for rank (r, c')) is its kz bins as an [X][Y][w_c'] block;
    the chunks lie back to back -> [..., X*Y*K]."""
    *lead, x, y, k = rows.shape
    n = 2 * (k - 1)
    parts = []
    for c in range(pc):
        k0, k1 = pencil_kz_range(n, pc, c)
        parts.append(rows[..., k0:k1].reshape(*lead, x * y * (k1 - k0)))
    return np.concatenate(parts, axis=-1)


def pencil_unsend(flat: np.ndarray, x: int, y: int, pc: int) -> np.ndarray:
    """Inverse of :func:`pencil_send`: [..., X*Y*K] -> [..., X, Y, K]."""
    *lead, total = flat.shape
    k = total // (x * y)
    n = 2 * (k - 1)
    out = np.empty((*lead, x, y, k), dtype=flat.dtype)
    for c in range(pc):
        k0, k1 = pencil_kz_range(n, pc, c)
        out[..., k0:k1] = flat[..., x * y * k0:x * y * k1].reshape(*lead, x, y, k1 - k0)
    return out


def pencil_exchange1(sends: list[np.ndarray], x: int, y: int) -> list[np.ndarray]:
    """Exchange 1 inside one grid row: ``sends[c']`` is rank (r, c')'s
    first-exchange buffer [..., X*Y*K]; rank (r, c) receives chunk c of every
    rank into block c' of its y-pencil [..., pc, X, Y, w_c]."""
    pc = len(sends)
    k = sends[0].shape[-1] // (x * y)
    n = 2 * (k - 1)
    out = []
    for c in range(pc):
        k0, k1 = pencil_kz_range(n, pc, c)
        blocks = [s[..., x * y * k0:x * y * k1].reshape(*s.shape[:-1], x, y, k1 - k0)
                  for s in sends]
        out.append(np.stack(blocks, axis=-4))
    return out


def pencil_exchange1_back(ypencils: list[np.ndarray]) -> list[np.ndarray]:
    """Inverse of :func:`pencil_exchange1`: every block back to its sender,
    giving each rank (r, c') its first-exchange buffer [..., X*Y*K]."""
    pc = len(ypencils)
    lead = ypencils[0].shape[:-4]
    out = []
    for cp in range(pc):
        out.append(np.concatenate([ypencils[c][..., cp, :, :, :].reshape(*lead, -1)
                                   for c in range(pc)], axis=-1))
    return out


def pencil_y_c2c(ypencil: np.ndarray, sign: int, method=None) -> np.ndarray:
    """1D DFT along y of a y-pencil [..., pc, X, Y, w] (y = c' Y + y_l)."""
    *lead, pc, x, y, w = ypencil.shape
    nl = len(lead)
    perm = list(range(nl)) + [nl + 1, nl, nl + 2, nl + 3]        # -> [X, pc, Y, w]
    lines = np.ascontiguousarray(ypencil.transpose(perm)).reshape(*lead, x, pc * y, w)
    lines = c2c_axis(lines, -2, sign, method)
    return np.ascontiguousarray(lines.reshape(*lead, x, pc, y, w).transpose(perm))


def pencil_exchange2(ypencils: list[np.ndarray], pr: int) -> list[np.ndarray]:
    """Exchange 2 inside one grid column: ``ypencils[r]`` is rank (r, c)'s
    y-pencil [..., pc, X, Y, w].  pr <= pc: rank (r', c) receives blocks
    [r' g, (r'+1) g) (g = pc/pr) of every rank r as block r of its x-pencil
    [..., pr, g, X, Y, w].  pr > pc (h = pr/pc): rank r' = c' h + s receives
    rows [s N/pr, (s+1) N/pr) of block c' of every rank r as block r of its
    x-pencil [..., pr, X, N/pr, w]."""
    pc = ypencils[0].shape[-4]
    if pr <= pc:
        g = pc // pr
        return [np.stack([yp[..., rp * g:(rp + 1) * g, :, :, :] for yp in ypencils], axis=-5)
                for rp in range(pr)]
    h = pr // pc
    yr = ypencils[0].shape[-2] // h
    return [np.stack([yp[..., rp // h, :, (rp % h) * yr:(rp % h + 1) * yr, :] for yp in ypencils],
                     axis=-4)
            for rp in range(pr)]


def pencil_exchange2_back(xpencils: list[np.ndarray], pc: int) -> list[np.ndarray]:
    """Inverse of :func:`pencil_exchange2` (``pc`` columns in the grid)."""
    pr = len(xpencils)
    if pr <= pc:
        return [np.concatenate([xpencils[rp][..., r, :, :, :, :] for rp in range(pr)], axis=-4)
                for r in range(pr)]
    h = pr // pc
    out = []
    for r in range(pr):
        blocks = [np.concatenate([xpencils[cp * h + s][..., r, :, :, :] for s in range(h)],
                                 axis=-2)
                  for cp in range(pc)]
        out.append(np.stack(blocks, axis=-4))
    return out


def pencil_pack2(ypencil: np.ndarray, h: int) -> np.ndarray:
    """Second-exchange send order of a pr > pc rank (h = pr/pc): run (c', s)
    = rows [s Y/h, (s+1) Y/h) of y-pencil block c', for peer c' h + s:
    [..., pc, X, Y, w] -> [..., pc, h, X, Y/h, w]."""
    *lead, pc, x, y, w = ypencil.shape
    nl = len(lead)
    t = ypencil.reshape(*lead, pc, x, h, y // h, w)
    perm = list(range(nl)) + [nl, nl + 2, nl + 1, nl + 3, nl + 4]
    return np.ascontiguousarray(t.transpose(perm))


def pencil_x_c2c(xpencil: np.ndarray, sign: int, method=None) -> np.ndarray:
    """1D DFT along x of an x-pencil [..., pr, g, X, Y, w] (x = r X + x_l)."""
    *lead, pr, g, x, y, w = xpencil.shape
    nl = len(lead)
    perm = list(range(nl)) + [nl + 1, nl, nl + 2, nl + 3, nl + 4]  # -> [g, pr, X, Y, w]
    lines = np.ascontiguousarray(xpencil.transpose(perm)).reshape(*lead, g, pr * x, y, w)
    lines = c2c_axis(lines, -3, sign, method)
    return np.ascontiguousarray(lines.reshape(*lead, g, pr, x, y, w).transpose(perm))


# --------------------------------------------------------------------------
# Weights, adjoints and the differentiable workloads
# --------------------------------------------------------------------------

def half_weights(n: int) -> np.ndarray:
    """w(kz) of the stored half spectrum: 1 at kz = 0 and kz = N/2, else 2."""
    k = np.arange(n // 2 + 1)
    w = np.full(k.shape, 2.0)
    w[0] = 1.0
    if n % 2 == 0:
        w[-1] = 1.0
    return w


def r2c3d_adjoint(g: np.ndarray, n: int, method=None) -> np.ndarray:
    """Adjoint of the forward R2C for <F,G> = sum over the half of Re(F* G).

    R2C^T(G)(j) = sum_{k in half} Re(G(k) exp(+2 pi i k.j/N)) = C2R(G / w).
    """
    return c2r3d(np.asarray(g) / half_weights(n), n, 1.0, method)


def c2r3d_adjoint(h: np.ndarray, method=None) -> np.ndarray:
    """Adjoint of C2R: C2R^T(h) = w * R2C(h)."""
    n = h.shape[-1]
    return r2c3d(h, method) * half_weights(n)


def wavenumbers(n: int):
    """Signed integer wavenumbers along x/y (length n) and z (n//2 + 1)."""
    k = np.arange(n)
    kxy = np.where(k <= n // 2, k, k - n).astype(np.float64)
    kz = np.arange(n // 2 + 1, dtype=np.float64)
    return kxy, kz


def k_squared(n: int) -> np.ndarray:
    kxy, kz = wavenumbers(n)
    return (kxy[:, None, None] ** 2 + kxy[None, :, None] ** 2
            + kz[None, None, :] ** 2)


def energy_loss(u: np.ndarray) -> float:
    """L1(u) = sum over the full spectrum of |k|^2 |u_hat(k)|^2.

    Over the stored half this is sum w(kz) |k|^2 |u_hat|^2 (the bins kz and
    -kz carry equal energy for a real field).
    """
    n = u.shape[-1]
    uh = r2c3d(u)
    return float(np.sum(half_weights(n) * k_squared(n) * np.abs(uh) ** 2))


def energy_loss_grad(u: np.ndarray) -> np.ndarray:
    """dL1/du = 2 C2R(|k|^2 u_hat) (unnormalized C2R)."""
    n = u.shape[-1]
    return 2.0 * c2r3d(k_squared(n) * r2c3d(u), n)


def poisson(f: np.ndarray) -> np.ndarray:
    """Spectral Poisson solve: u = N^-3 C2R(m R2C(f)), m = -1/|k|^2, m(0) = 0."""
    n = f.shape[-1]
    k2 = k_squared(n)
    m = np.zeros_like(k2)
    nz = k2 > 0
    m[nz] = -1.0 / k2[nz]
    return c2r3d(m * r2c3d(f), n, 1.0 / n ** 3)


def poisson_loss(f: np.ndarray) -> float:
    """L2(f) = sum_j u(j)^2 with u = poisson(f)."""
    return float(np.sum(poisson(f) ** 2))


def poisson_loss_grad(f: np.ndarray) -> np.ndarray:
    """dL2/df = 2 poisson(poisson(f)): the solve is self-adjoint."""
    return 2.0 * poisson(poisson(f))


# --------------------------------------------------------------------------
# Sampled checks of large transforms
# --------------------------------------------------------------------------

def r2c3d_kz_planes(f: np.ndarray, kz) -> np.ndarray:
    """Whole kz-planes F(:, :, kz_q) of the forward R2C of a real [N,N,N] grid.

    The z sum of the forward equation is evaluated directly for the requested
    kz only, then the complex DFT along y and along x.  Returns [N, N, nq].
    """
    f = np.ascontiguousarray(f, dtype=np.float64)
    nx, ny, n = f.shape
    kz = np.ascontiguousarray(np.asarray(kz, dtype=np.int64))
    a = np.empty((nx, ny, kz.size), dtype=np.complex128)
    if _load().oracle_zsum_rows(nx * ny, n, _ptr(f), kz.size, _ptr(kz),
                                _ptr(a)):
        raise ValueError("oracle_zsum_rows rejected its arguments")
    a = c2c_axis(a, 1, -1)
    return c2c_axis(a, 0, -1)
