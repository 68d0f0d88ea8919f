"""Shared test helpers (no method arithmetic here)."""

import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

FP64_TOL = 1e-12  # relative L-infinity, FP64 library vs FP64 oracle
FP32_TOL = 1e-5   # relative L-infinity, FP32 library vs FP64 oracle


def rel_linf(q, ref):
    """Per-component relative L-infinity error: max|q_m - ref_m| / max|ref_m|;
    a component whose reference is identically zero is divided by the largest
    magnitude over all components instead.  Returns an array of 3 errors."""
    q = np.asarray(q, np.float64)
    ref = np.asarray(ref, np.float64)
    allmax = np.abs(ref).max()
    out = np.zeros(3)
    for m in range(3):
        d = np.abs(q[m] - ref[m]).max()
        s = np.abs(ref[m]).max()
        out[m] = d / (s if s > 0 else (allmax if allmax > 0 else 1.0))
    return out


def header_symbols():
    """Function names declared in include/wavestep.h."""
    src = open(os.path.join(ROOT, "include", "wavestep.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ws_[a-z_]+)\s*\(", src)))
