"""Helpers for the GPU tests: skip cleanly without a device, print the case
before each GPU step, compare with tolerance."""
import sys

import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def announce(*parts):
    print("[gpu case]", *parts, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def block_errs(S, y, yref):
    """Relative 2-norm errors over all rows, the velocity rows and the
    pressure rows (velocity rows scale like h, pressure rows like h^2)."""
    o = S.offsets[3]
    return rel_err(y, yref), rel_err(y[:o], yref[:o]), rel_err(y[o:], yref[o:])
