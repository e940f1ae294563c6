"""Shared helpers of the GPU parity tests (comparison metrics, set-up)."""

from __future__ import annotations

import numpy as np


def site_rel_err(got, ref, ncomp=12):
    """Per-site relative error: ||got(x) - ref(x)||_2 / max(||ref(x)||_2, RMS_x ||ref||_2).

    The RMS floor keeps near-zero sites meaningful.  ncomp: complex numbers
    per site (12 for spinors, 3 for staggered colour vectors).  Returns the
    maximum over sites (and right-hand sides)."""
    got = np.asarray(got).reshape(-1, ncomp)
    ref = np.asarray(ref).reshape(-1, ncomp)
    d = np.linalg.norm(got - ref, axis=1)
    n = np.linalg.norm(ref, axis=1)
    rms = np.sqrt(np.mean(n ** 2))
    den = np.maximum(n, rms if rms > 0 else 1.0)
    return float(np.max(d / den))


def gpu_ok():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
