"""Shared test helpers: the relative-error metric and array plumbing."""
import numpy as np


def chan_rel_err(got, ref, layout):
    """Max over channels of max_t |got - ref| / max_t |ref| (per-channel
    relative error; signals and per-sample coefficient grads alike)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.shape != ref.shape:
        raise AssertionError(f"shape {got.shape} != {ref.shape}")
    if got.size == 0:
        return 0.0
    # move the channel axis first
    if layout == "TB":
        got = np.moveaxis(got, 1, 0)
        ref = np.moveaxis(ref, 1, 0)
    B = got.shape[0]
    g = got.reshape(B, -1)
    r = ref.reshape(B, -1)
    num = np.abs(g - r).max(axis=1)
    den = np.abs(r).max(axis=1)
    den = np.where(den == 0, 1.0, den)
    return float((num / den).max())


def vec_rel_err(got, ref):
    """Per row (channel): ||got - ref||_inf / ||ref||_inf, max over rows."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.shape != ref.shape:
        raise AssertionError(f"shape {got.shape} != {ref.shape}")
    if got.size == 0:
        return 0.0
    g = got.reshape(got.shape[0], -1)
    r = ref.reshape(ref.shape[0], -1)
    den = np.abs(r).max(axis=1)
    den = np.where(den == 0, 1.0, den)
    return float((np.abs(g - r).max(axis=1) / den).max())
