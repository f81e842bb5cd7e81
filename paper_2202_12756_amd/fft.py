"""Torch-facing plan object over the C ABI.

Torch supplies device memory and the stream; the wrapper checks shapes,
dtypes, devices and contiguity (the C ABI cannot see buffer lengths), then
passes raw device addresses and the current HIP stream to libgfft.so.
"""
from __future__ import annotations

import torch

from . import _lib

_REAL = {torch.float64: _lib.GFFT_F64, torch.float32: _lib.GFFT_F32}
_CPLX = {torch.float64: torch.complex128, torch.float32: torch.complex64}


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _resolve(device) -> torch.device:
    """The plan's device with its index fixed (the current one if none is given)."""
    dev = torch.device(device if device is not None else "cuda")
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    return dev


def device_copy(dst: torch.Tensor, src: torch.Tensor) -> torch.Tensor:
    """Copy ``src`` into ``dst`` (same byte size, both contiguous on one GPU)
    with the library's streaming copy kernel, on the current torch stream."""
    if not (isinstance(dst, torch.Tensor) and isinstance(src, torch.Tensor)):
        raise TypeError("dst and src must be torch.Tensors")
    if dst.device != src.device or dst.device.type != "cuda":
        raise ValueError("dst and src must live on the same GPU")
    if not (dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("dst and src must be contiguous")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src must have the same byte size")
    with torch.cuda.device(dst.device):
        _lib.check(_lib.gfft_device_copy(dst.data_ptr(), src.data_ptr(), nbytes,
                                         _stream(dst.device)), "gfft_device_copy")
    return dst


class _Exec:
    def _exec(self, fn, *args):
        """Call a library entry point with the plan's device current, on that
        device's current torch stream (the library refuses any other device)."""
        with torch.cuda.device(self.device):
            _lib.check(fn(self._h, *args, _stream(self.device)), fn.__name__)


class Plan(_Exec):
    """One GPU's share of an N^3 real FFT (full grid when slab_x == n).

    Layouts (C order, z fastest): real [batch, X, N, N]; half spectrum
    [batch, X, N, K] complex, or the send order [batch, p, X, N/p, K] when
    ``fuse_pack``; x-pencil [batch, N, N/p, K].  For batch == 1 the leading
    batch dimension may be omitted.  ``mfma_terms`` (FP32 only) runs the first
    radix-16 stage of the y and x passes on the matrix cores with 2 or 3
    BF16 terms per operand.  ``inplace`` plans transform one shared buffer
    (a complex [batch, X, N, K] tensor whose real view holds rows of N reals
    padded to N + 2): use ``empty_inplace``, ``real_view``, ``r2c_`` and
    ``c2r_``.  ``paper_order`` uses the paper's chunk order [ky_l][x_l][kz]
    as the exchange format (send buffer and received pencil
    [batch, p, N/p, X, K]).
    """

    def __init__(self, n: int, dtype=torch.float64, slab_x: int | None = None,
                 batch: int = 1, fuse_pack: bool = False, device=None,
                 mfma_terms: int = 0, inplace: bool = False,
                 paper_order: bool = False):
        if dtype not in _REAL:
            raise TypeError("dtype must be torch.float64 or torch.float32")
        self.n = int(n)
        self.dtype = dtype
        self.cdtype = _CPLX[dtype]
        self.slab_x = int(slab_x if slab_x is not None else n)
        self.batch = int(batch)
        self.fuse_pack = bool(fuse_pack)
        self.device = _resolve(device)
        self.mfma_terms = int(mfma_terms)
        self.inplace = bool(inplace)
        self.paper_order = bool(paper_order)
        flags = _lib.GFFT_FUSE_PACK if fuse_pack else 0
        if self.inplace:
            flags |= _lib.GFFT_INPLACE
        if self.paper_order:
            flags |= _lib.GFFT_PACK_PAPER_ORDER
        if self.mfma_terms not in (0, 2, 3):
            raise ValueError("mfma_terms must be 0, 2 or 3")
        if self.mfma_terms == 2:
            flags |= _lib.GFFT_MFMA_BF16X2
        elif self.mfma_terms == 3:
            flags |= _lib.GFFT_MFMA_BF16X3
        with torch.cuda.device(self.device):
            st, h = _lib.gfft_plan_create(self.n, _REAL[dtype], self.slab_x,
                                          self.batch, flags)
        _lib.check(st, "gfft_plan_create")
        self._h = h
        st, s = _lib.gfft_plan_query(h)
        _lib.check(st, "gfft_plan_query")
        self.k = s.k
        self.ranks = s.ranks
        self.sizes = {f: getattr(s, f) for f, _ in _lib.gfft_plan_sizes._fields_}

    # ------------------------------------------------------------ shapes
    @property
    def real_shape(self):
        return (self.batch, self.slab_x, self.n, self.n)

    @property
    def spectrum_shape(self):
        if self.fuse_pack:
            return self.send_shape
        return (self.batch, self.slab_x, self.n, self.k)

    @property
    def send_shape(self):
        y = self.n // self.ranks
        if self.paper_order:      # chunk j = [ky_l][x_l][kz]
            return (self.batch, self.ranks, y, self.slab_x, self.k)
        return (self.batch, self.ranks, self.slab_x, y, self.k)

    @property
    def pencil_shape(self):
        y = self.n // self.ranks
        if self.paper_order:      # received chunks [i][ky_l][x_l][kz]
            return (self.batch, self.ranks, y, self.slab_x, self.k)
        return (self.batch, self.n, y, self.k)

    def _check(self, t: torch.Tensor, dtype, numel: int, what: str):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{what} must be a torch.Tensor")
        if t.dtype != dtype:
            raise TypeError(f"{what} must have dtype {dtype}, got {t.dtype}")
        if t.device != self.device:
            raise ValueError(f"{what} must live on {self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if t.numel() != numel:
            raise ValueError(f"{what} has {t.numel()} elements, plan needs {numel}")
        return t.data_ptr()

    def _nreal(self):
        rs = self.n + 2 if self.inplace else self.n
        return self.batch * self.slab_x * self.n * rs

    def _ncplx(self):
        return self.batch * self.slab_x * self.n * self.k

    def _npencil(self):
        return self.batch * self.n * (self.n // self.ranks) * self.k

    def empty_real(self):
        return torch.empty(self.real_shape, dtype=self.dtype, device=self.device)

    def empty_spectrum(self):
        return torch.empty(self.spectrum_shape, dtype=self.cdtype,
                           device=self.device)

    # ------------------------------------------------------------ transforms
    def r2c(self, x: torch.Tensor, out: torch.Tensor | None = None):
        out = self.empty_spectrum() if out is None else out
        a = self._check(x, self.dtype, self._nreal(), "input")
        b = self._check(out, self.cdtype, self._ncplx(), "output")
        self._exec(_lib.gfft_exec_r2c, a, b)
        return out

    def c2r(self, g: torch.Tensor, out: torch.Tensor | None = None,
            scale: float = 1.0):
        """Inverse (clobbers ``g``)."""
        out = self.empty_real() if out is None else out
        a = self._check(g, self.cdtype, self._ncplx(), "input")
        b = self._check(out, self.dtype, self._nreal(), "output")
        self._exec(_lib.gfft_exec_c2r, a, b, float(scale))
        return out

    def r2c_adjoint(self, g: torch.Tensor, out=None, scale: float = 1.0):
        """scale * R2C^T(g) = scale * C2R(g / w) (clobbers ``g``)."""
        out = self.empty_real() if out is None else out
        a = self._check(g, self.cdtype, self._ncplx(), "input")
        b = self._check(out, self.dtype, self._nreal(), "output")
        self._exec(_lib.gfft_exec_r2c_adjoint, a, b, float(scale))
        return out

    def c2r_adjoint(self, h: torch.Tensor, out=None, scale: float = 1.0):
        """scale * C2R^T(h) = scale * w * R2C(h)."""
        out = self.empty_spectrum() if out is None else out
        a = self._check(h, self.dtype, self._nreal(), "input")
        b = self._check(out, self.cdtype, self._ncplx(), "output")
        self._exec(_lib.gfft_exec_c2r_adjoint, a, b, float(scale))
        return out

    def pack(self, slab: torch.Tensor, out: torch.Tensor | None = None):
        out = (torch.empty(self.send_shape, dtype=self.cdtype,
                           device=self.device) if out is None else out)
        a = self._check(slab, self.cdtype, self._ncplx(), "slab")
        b = self._check(out, self.cdtype, self._ncplx(), "send")
        self._exec(_lib.gfft_pack_slab_for_alltoall, a, b)
        return out

    def unpack(self, recv: torch.Tensor, out: torch.Tensor | None = None):
        out = (torch.empty((self.batch, self.slab_x, self.n, self.k),
                           dtype=self.cdtype, device=self.device)
               if out is None else out)
        a = self._check(recv, self.cdtype, self._ncplx(), "recv")
        b = self._check(out, self.cdtype, self._ncplx(), "slab")
        self._exec(_lib.gfft_unpack_slab_from_alltoall, a, b)
        return out

    def x_c2c(self, pencil: torch.Tensor, sign: int):
        a = self._check(pencil, self.cdtype, self._npencil(), "pencil")
        self._exec(_lib.gfft_exec_x_c2c, a, int(sign))
        return pencil

    def pass_copy(self, data: torch.Tensor, axis: int):
        """Yardstick: the y (axis 0) or x (axis 1) pass's loads and stores on
        ``data`` (its buffer for that pass), no transform: ``data`` becomes
        its conjugate."""
        if axis not in (0, 1):
            raise ValueError("axis must be 0 (y pass) or 1 (x pass)")
        n = self._ncplx() if axis == 0 else self._npencil()
        a = self._check(data, self.cdtype, n, "data")
        self._exec(_lib.gfft_exec_pass_copy, int(axis), a)
        return data

    # ------------------------------------------------------------ in place
    def empty_inplace(self):
        """The shared buffer of an in-place plan (complex, spectrum shape)."""
        return torch.empty((self.batch, self.slab_x, self.n, self.k),
                           dtype=self.cdtype, device=self.device)

    def real_view(self, buf: torch.Tensor) -> torch.Tensor:
        """The [batch, X, N, N] real field inside a padded shared buffer."""
        r = torch.view_as_real(buf).reshape(self.batch, self.slab_x, self.n, 2 * self.k)
        return r[..., : self.n]

    def _inplace_ptr(self, buf):
        if not self.inplace:
            raise ValueError("plan was not created with inplace=True")
        return self._check(buf, self.cdtype, self._ncplx(), "buffer")

    def r2c_(self, buf: torch.Tensor):
        """In-place forward transform of the padded field in ``buf``."""
        a = self._inplace_ptr(buf)
        self._exec(_lib.gfft_exec_r2c, a, a)
        return buf

    def c2r_(self, buf: torch.Tensor, scale: float = 1.0):
        """In-place inverse; returns the real view of ``buf``."""
        a = self._inplace_ptr(buf)
        self._exec(_lib.gfft_exec_c2r, a, a, float(scale))
        return self.real_view(buf)

    def r2c_adjoint_(self, buf: torch.Tensor, scale: float = 1.0):
        a = self._inplace_ptr(buf)
        self._exec(_lib.gfft_exec_r2c_adjoint, a, a, float(scale))
        return self.real_view(buf)

    def c2r_adjoint_(self, buf: torch.Tensor, scale: float = 1.0):
        a = self._inplace_ptr(buf)
        self._exec(_lib.gfft_exec_c2r_adjoint, a, a, float(scale))
        return buf

    # ------------------------------------------------------------ passes
    def z_r2c(self, x, out=None, scale: float = 1.0, weighted: bool = False):
        out = self.empty_spectrum() if out is None else out
        a = self._check(x, self.dtype, self._nreal(), "input")
        b = self._check(out, self.cdtype, self._ncplx(), "output")
        self._exec(_lib.gfft_exec_z_r2c, a, b, float(scale), int(weighted))
        return out

    def y_c2c(self, data, sign: int):
        a = self._check(data, self.cdtype, self._ncplx(), "data")
        self._exec(_lib.gfft_exec_y_c2c, a, int(sign))
        return data

    def z_c2r(self, g, out=None, scale: float = 1.0, weighted: bool = False):
        out = self.empty_real() if out is None else out
        a = self._check(g, self.cdtype, self._ncplx(), "input")
        b = self._check(out, self.dtype, self._nreal(), "output")
        self._exec(_lib.gfft_exec_z_c2r, a, b, float(scale), int(weighted))
        return out

    # ------------------------------------------------------------ lifetime
    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            _lib.check(_lib.gfft_plan_destroy(h), "gfft_plan_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PencilPlan(_Exec):
    """Rank (r, c)'s share of an N^3 real FFT on a pr x pc pencil grid.

    Real pencil [batch, X, Y, N] (X = N/pr, Y = N/pc, z fastest).  The z pass
    writes the half spectrum in first-exchange order, ``send_shape`` =
    [batch, X*Y*K]: chunk c' = kz in ``kz_range(c')``, a [X, Y, w_c'] block
    (``chunk`` gives views).  After exchange 1 the y pass runs on the
    y-pencil [batch, pc, X, Y, w] (block c' from rank (r, c')); after
    exchange 2 the x pass runs on the x-pencil: for pr <= pc
    [batch, pr, g, X, Y, w] (g = pc/pr; block r from rank (r, c) = its
    y-pencil blocks [r' g, (r'+1) g) for destination r'); for pr > pc
    [batch, pr, X, N/pr, w] (block r = run (c', s), r' = c' h + s, of rank
    (r, c)'s packed y-pencil ``pack2`` [batch, pc, h, X, N/pr, w]).
    Requires pc <= N/2.
    """

    _check = Plan._check

    def __init__(self, n: int, dtype=torch.float64, grid=(1, 1), col: int = 0,
                 batch: int = 1, device=None, mfma_terms: int = 0):
        if dtype not in _REAL:
            raise TypeError("dtype must be torch.float64 or torch.float32")
        self.n = int(n)
        self.dtype = dtype
        self.cdtype = _CPLX[dtype]
        self.pr, self.pc = (int(v) for v in grid)
        self.col = int(col)
        self.batch = int(batch)
        self.device = _resolve(device)
        if int(mfma_terms) not in (0, 2, 3):
            raise ValueError("mfma_terms must be 0, 2 or 3")
        flags = {0: 0, 2: _lib.GFFT_MFMA_BF16X2, 3: _lib.GFFT_MFMA_BF16X3}[int(mfma_terms)]
        with torch.cuda.device(self.device):
            st, h = _lib.gfft_pencil_plan_create(self.n, _REAL[dtype], self.pr, self.pc,
                                                 self.col, self.batch, flags)
        _lib.check(st, "gfft_pencil_plan_create")
        self._h = h
        st, s = _lib.gfft_plan_query(h)
        _lib.check(st, "gfft_plan_query")
        self.sizes = {f: getattr(s, f) for f, _ in _lib.gfft_plan_sizes._fields_}
        self.k = s.k
        self.x = s.slab_x
        self.y = s.y_local
        self.w = s.kz_width
        self.w0 = self.n // (2 * self.pc)
        self.g = max(self.pc // self.pr, 1)
        self.h = max(self.pr // self.pc, 1)

    def kz_range(self, c: int):
        """The kz bins [k0, k1) that column c holds after exchange 1."""
        k0 = c * self.w0
        return k0, k0 + self.w0 + (1 if c == self.pc - 1 else 0)

    @property
    def real_shape(self):
        return (self.batch, self.x, self.y, self.n)

    @property
    def send_shape(self):
        return (self.batch, self.x * self.y * self.k)

    @property
    def ypencil_shape(self):
        return (self.batch, self.pc, self.x, self.y, self.w)

    @property
    def xpencil_shape(self):
        if self.h > 1:
            return (self.batch, self.pr, self.x, self.n // self.pr, self.w)
        return (self.batch, self.pr, self.g, self.x, self.y, self.w)

    @property
    def send2_shape(self):
        """Second-exchange send order of a pr > pc plan (run (c', s) for
        peer c' h + s)."""
        return (self.batch, self.pc, self.h, self.x, self.n // self.pr, self.w)

    def pack2(self, ypencil, out=None):
        """Split each y-pencil block into h runs for exchange 2 (pr > pc)."""
        out = (torch.empty(self.send2_shape, dtype=self.cdtype, device=self.device)
               if out is None else out)
        a = self._check(ypencil, self.cdtype, self._n(self.ypencil_shape), "y-pencil")
        b = self._check(out, self.cdtype, self._n(self.send2_shape), "send")
        self._exec(_lib.gfft_pack_slab_for_alltoall, a, b)
        return out

    def unpack2(self, send, out=None):
        """Inverse of ``pack2``."""
        out = (torch.empty(self.ypencil_shape, dtype=self.cdtype, device=self.device)
               if out is None else out)
        a = self._check(send, self.cdtype, self._n(self.send2_shape), "send")
        b = self._check(out, self.cdtype, self._n(self.ypencil_shape), "y-pencil")
        self._exec(_lib.gfft_unpack_slab_from_alltoall, a, b)
        return out

    def chunk(self, send: torch.Tensor, c: int) -> torch.Tensor:
        """View [batch, X, Y, w_c] of chunk c of a first-exchange buffer."""
        k0, k1 = self.kz_range(c)
        rows = self.x * self.y
        return send[:, rows * k0: rows * k1].view(self.batch, self.x, self.y, k1 - k0)

    def _n(self, shape):
        out = 1
        for v in shape:
            out *= v
        return out

    def z_r2c(self, x, out=None, scale: float = 1.0, weighted: bool = False):
        out = (torch.empty(self.send_shape, dtype=self.cdtype, device=self.device)
               if out is None else out)
        a = self._check(x, self.dtype, self._n(self.real_shape), "input")
        b = self._check(out, self.cdtype, self._n(self.send_shape), "output")
        self._exec(_lib.gfft_exec_z_r2c, a, b, float(scale), int(weighted))
        return out

    def y_c2c(self, ypencil, sign: int):
        a = self._check(ypencil, self.cdtype, self._n(self.ypencil_shape), "y-pencil")
        self._exec(_lib.gfft_exec_y_c2c, a, int(sign))
        return ypencil

    def x_c2c(self, xpencil, sign: int):
        a = self._check(xpencil, self.cdtype, self._n(self.xpencil_shape), "x-pencil")
        self._exec(_lib.gfft_exec_x_c2c, a, int(sign))
        return xpencil

    def z_c2r(self, g, out=None, scale: float = 1.0, weighted: bool = False):
        """Inverse z pass from first-exchange order (reads ``g``)."""
        out = (torch.empty(self.real_shape, dtype=self.dtype, device=self.device)
               if out is None else out)
        a = self._check(g, self.cdtype, self._n(self.send_shape), "input")
        b = self._check(out, self.dtype, self._n(self.real_shape), "output")
        self._exec(_lib.gfft_exec_z_c2r, a, b, float(scale), int(weighted))
        return out

    close = Plan.close
    __del__ = Plan.__del__
