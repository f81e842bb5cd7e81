"""Shared test helpers (no FFT arithmetic here)."""
import numpy as np
import torch

import synth

# Tolerances on relative L2 error against the FP64 oracle.
TOL = {torch.float64: 1e-13, torch.float32: 5e-6}


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.linalg.norm((a.astype(np.complex128) - b).ravel())
    return float(d / np.linalg.norm(b.ravel()))


def real_input(shape, seed, dtype, device="cuda"):
    """Seeded uniform reals; the oracle gets the exact same values in FP64."""
    x = synth.uniform(shape, seed, dtype, "cpu")
    return x.to(device), x.double().numpy()


def cplx_input(shape, seed, dtype, device="cuda"):
    re = synth.uniform(shape, seed, dtype, "cpu")
    im = synth.uniform(shape, seed + 1000, dtype, "cpu")
    c = torch.complex(re, im)
    return c.to(device), (re.double() + 1j * im.double()).numpy()


def host(t: torch.Tensor) -> np.ndarray:
    t = t.detach().cpu()
    if t.is_complex():
        return t.to(torch.complex128).numpy()
    return t.double().numpy()
