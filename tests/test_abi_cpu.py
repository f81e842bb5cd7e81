"""The C ABI on the host: symbols, status codes and argument checks.

No compute calls: these run without a GPU.  Every check here happens on the
host before any HIP call, as include/gfft.h promises.
"""
import ctypes
import os
import re

import pytest

from paper_2202_12756_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gfft.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gfft_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


def test_status_strings_and_version():
    for st in range(-6, 1):
        s = _lib.status_string(st)
        assert s and s != "unknown status"
    assert _lib.status_string(-99) == "unknown status"
    assert _lib.gfft_version() >= 100


@pytest.mark.parametrize("args,expect", [
    ((64, 0, 64, 1, 0), None),                                 # valid
    ((63, 0, 63, 1, 0), _lib.GFFT_E_UNSUPPORTED),              # not 2^m
    ((8, 0, 8, 1, 0), _lib.GFFT_E_UNSUPPORTED),                # below 16
    ((8192, 0, 8192, 1, 0), _lib.GFFT_E_UNSUPPORTED),          # above 4096
    ((64, 0, 3, 1, 0), _lib.GFFT_E_INVALID_ARG),               # X does not divide N
    ((64, 0, 128, 1, 0), _lib.GFFT_E_INVALID_ARG),             # X > N
    ((64, 0, 0, 1, 0), _lib.GFFT_E_INVALID_ARG),               # X = 0
    ((64, 0, 64, 0, 0), _lib.GFFT_E_INVALID_ARG),              # batch 0
    ((64, 2, 64, 1, 0), _lib.GFFT_E_INVALID_ARG),              # bad dtype
    ((64, 0, 64, 1, 1 << 7), _lib.GFFT_E_INVALID_ARG),         # unknown flag
    ((0, 0, 1, 1, 0), _lib.GFFT_E_INVALID_ARG),                # N = 0
    ((4096, 0, 4096, 1 << 40, 0), _lib.GFFT_E_UNSUPPORTED),    # size overflow
    ((64, 1, 64, 1, 2), None),                                 # FP32 + 2-term MFMA
    ((64, 1, 64, 1, 4), None),                                 # FP32 + 3-term MFMA
    ((64, 0, 64, 1, 2), _lib.GFFT_E_UNSUPPORTED),              # MFMA needs FP32
    ((16, 1, 16, 1, 4), _lib.GFFT_E_UNSUPPORTED),              # MFMA needs N >= 32
    ((64, 1, 64, 1, 6), _lib.GFFT_E_INVALID_ARG),              # both MFMA flags
    ((64, 0, 64, 1, 8), None),                                 # in place
    ((64, 0, 16, 1, 9), _lib.GFFT_E_UNSUPPORTED),              # in place + send order
    ((64, 0, 16, 1, 17), None),                                # paper chunk order, fused
    ((64, 0, 64, 1, 16), _lib.GFFT_E_UNSUPPORTED),             # paper order needs a slab
])
def test_plan_create_validates_on_host(args, expect):
    st, h = _lib.gfft_plan_create(*args)
    if expect is None:
        # valid arguments: without a gfx950 device the next check reports it
        if not _has_gpu():
            assert st == _lib.GFFT_E_NO_DEVICE
            assert not h.value
        else:
            assert st == _lib.GFFT_OK
            assert _lib.gfft_plan_destroy(h) == _lib.GFFT_OK
    else:
        assert st == expect
        assert not h.value


@pytest.mark.parametrize("args,expect", [
    ((64, 0, 2, 4, 1, 1, 0), None),                            # valid
    ((64, 0, 8, 16, 15, 1, 0), None),                          # p = 128 > N
    ((64, 0, 1, 1, 0, 1, 0), None),                            # one rank
    ((64, 0, 4, 2, 0, 1, 0), None),                            # pr > pc (packed exchange 2)
    ((64, 0, 64, 32, 0, 1, 0), None),                          # p = N^2/2
    ((16, 0, 32, 4, 0, 1, 0), _lib.GFFT_E_UNSUPPORTED),        # pr > N
    ((64, 0, 2, 64, 0, 1, 0), _lib.GFFT_E_UNSUPPORTED),        # pc > N/2
    ((64, 0, 3, 4, 0, 1, 0), _lib.GFFT_E_INVALID_ARG),         # pr not 2^m
    ((64, 0, 2, 4, 4, 1, 0), _lib.GFFT_E_INVALID_ARG),         # col >= pc
    ((64, 0, 2, 4, -1, 1, 0), _lib.GFFT_E_INVALID_ARG),        # col < 0
    ((64, 0, 0, 4, 0, 1, 0), _lib.GFFT_E_INVALID_ARG),         # pr = 0
    ((64, 0, 2, 4, 0, 0, 0), _lib.GFFT_E_INVALID_ARG),         # batch 0
    ((48, 0, 2, 4, 0, 1, 0), _lib.GFFT_E_UNSUPPORTED),         # N not 2^m
    ((64, 0, 2, 4, 0, 1, 1), _lib.GFFT_E_UNSUPPORTED),         # slab flag
    ((64, 0, 2, 4, 0, 1, 8), _lib.GFFT_E_UNSUPPORTED),         # in place
    ((64, 1, 2, 4, 0, 1, 2), None),                            # FP32 + MFMA
    ((64, 0, 2, 4, 0, 1, 2), _lib.GFFT_E_UNSUPPORTED),         # MFMA needs FP32
    ((64, 0, 2, 4, 0, 1, 1 << 9), _lib.GFFT_E_INVALID_ARG),    # unknown flag
    ((4096, 0, 1, 1, 0, 1 << 40, 0), _lib.GFFT_E_UNSUPPORTED), # size overflow
])
def test_pencil_plan_create_validates_on_host(args, expect):
    st, h = _lib.gfft_pencil_plan_create(*args)
    if expect is None:
        if not _has_gpu():
            assert st == _lib.GFFT_E_NO_DEVICE
            assert not h.value
        else:
            assert st == _lib.GFFT_OK
            assert _lib.gfft_plan_destroy(h) == _lib.GFFT_OK
    else:
        assert st == expect
        assert not h.value


def test_null_plan_and_out_pointer():
    lib = _lib.load()
    assert lib.gfft_plan_create(None, 64, 0, 64, 1, 0) == _lib.GFFT_E_INVALID_ARG
    assert lib.gfft_pencil_plan_create(None, 64, 0, 2, 4, 0, 1, 0) == _lib.GFFT_E_INVALID_ARG
    assert _lib.gfft_plan_destroy(None) == _lib.GFFT_OK
    st, _ = _lib.gfft_plan_query(None)
    assert st == _lib.GFFT_E_INVALID_ARG
    for fn, extra in ((_lib.gfft_exec_r2c, (16, 32, None)),
                      (_lib.gfft_exec_c2r, (16, 32, 1.0, None)),
                      (_lib.gfft_exec_r2c_adjoint, (16, 32, 1.0, None)),
                      (_lib.gfft_exec_c2r_adjoint, (16, 32, 1.0, None)),
                      (_lib.gfft_pack_slab_for_alltoall, (16, 32, None)),
                      (_lib.gfft_unpack_slab_from_alltoall, (16, 32, None)),
                      (_lib.gfft_exec_x_c2c, (16, -1, None)),
                      (_lib.gfft_exec_y_c2c, (16, -1, None)),
                      (_lib.gfft_exec_z_r2c, (16, 32, 1.0, 0, None)),
                      (_lib.gfft_exec_z_c2r, (16, 32, 1.0, 0, None)),
                      (_lib.gfft_exec_pass_copy, (0, 16, None))):
        assert fn(None, *extra) == _lib.GFFT_E_INVALID_ARG


def test_device_copy_validates_on_host():
    """Every argument check of the copy runs before any HIP call."""
    assert _lib.gfft_device_copy(None, 4096, 64, None) == _lib.GFFT_E_INVALID_ARG
    assert _lib.gfft_device_copy(4096, None, 64, None) == _lib.GFFT_E_INVALID_ARG
    assert _lib.gfft_device_copy(4096, 8192, 24, None) == _lib.GFFT_E_INVALID_ARG   # not 16 x k
    assert _lib.gfft_device_copy(4096, 8192, -16, None) == _lib.GFFT_E_INVALID_ARG
    assert _lib.gfft_device_copy(4104, 8192, 64, None) == _lib.GFFT_E_ALIGN
    assert _lib.gfft_device_copy(4096, 4096 + 32, 64, None) == _lib.GFFT_E_INVALID_ARG  # overlap
    assert _lib.gfft_device_copy(4096, 8192, 0, None) == _lib.GFFT_OK                # nothing to do


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_product_path_has_no_cpu_fallback():
    """The package never imports the oracle or torch.fft."""
    pkg = os.path.join(ROOT, "paper_2202_12756_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn
            assert "torch.fft" not in src, fn
            assert "numpy.fft" not in src and "np.fft" not in src, fn


C_CLIENT = r"""
#include <stdio.h>
#include <string.h>
#include "gfft.h"
int main(void) {
    gfft_plan *p = 0;
    /* host-side validation runs before any device query */
    if (gfft_plan_create(&p, 48, GFFT_F64, 48, 1, 0) != GFFT_E_UNSUPPORTED) return 1;
    if (gfft_pencil_plan_create(&p, 64, GFFT_F32, 2, 64, 0, 1, 0) != GFFT_E_UNSUPPORTED) return 2;
    if (p != 0) return 3;
    if (gfft_plan_destroy(0) != GFFT_OK) return 4;
    if (strcmp(gfft_status_string(GFFT_E_ALIGN), "data pointer not 16-byte aligned") != 0) return 5;
    if (gfft_version() < 100) return 6;
    gfft_status st = gfft_plan_create(&p, 64, GFFT_F64, 64, 1, 0);
    printf("%d\n", (int)st);
    if (st == GFFT_OK) gfft_plan_destroy(p);
    return 0;
}
"""


def test_header_is_c_and_the_library_links_from_c(tmp_path):
    """include/gfft.h compiles as C99, and a C program linked against
    libgfft.so gets the host-side checks and status strings."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    lib = _lib.load()._name
    src = tmp_path / "client.c"
    src.write_text(C_CLIENT)
    exe = tmp_path / "client"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), lib, f"-Wl,-rpath,{os.path.dirname(lib)}", "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stderr)
    st = int(r.stdout.strip())
    assert st in (_lib.GFFT_OK, _lib.GFFT_E_NO_DEVICE)
