"""Shared helpers for the GPU parity tests (inputs from synth, references from oracle)."""
import numpy as np

import synth


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    nb = np.linalg.norm(b)
    # a zero reference (e.g. duals at the first iteration) compares in absolute terms
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def problem(n, M, d, scheme="equal", seed=0, blobs=5, points=10, outliers=0.0):
    rng = np.random.default_rng(seed)
    x = synth.sky(n, blobs, points, rng)
    uv = synth.uv_coverage(M, rng, outlier_frac=outliers)
    uvs, off, _ = synth.partition(uv, d, scheme, rng)
    return x, uvs, off


def to_user(y_plan, order):
    out = np.empty_like(y_plan)
    out[order] = y_plan
    return out


def to_plan(y_user, order):
    return y_user[order]
