"""Test-side helpers: oracle references and device set-up.

Only the test suite uses this module.  Oracle values come from ``oracle``
alone; device values from the library through the binding.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2204_14194_amd import synth

_CLASS_CACHE = {}


def classes_of(phi: np.ndarray) -> np.ndarray:
    key = (phi.shape, phi[:, :7].tobytes())
    if key not in _CLASS_CACHE:
        _CLASS_CACHE[key] = oracle.duplicate_classes(phi)
    return _CLASS_CACHE[key]


def oracle_blocks(images, blocks, phi, M, N, rho_hat, gamma, iters, method="fase",
                  sample=None, table_cache=None):
    """Oracle result per block: list of (SEResult, g over the loss (lh*lw,)).
    ``images`` is (n_img, H, W) uint8; the lost mask covers every block of
    ``blocks`` (of that image)."""
    n_img, H, W = images.shape
    lost = np.stack([synth.lost_mask(H, W, blocks, i) for i in range(n_img)])
    cls = classes_of(phi)
    idx = range(len(blocks)) if sample is None else sample
    cache = {} if table_cache is None else table_cache
    out = []
    for i in idx:
        b = blocks[i]
        _, per = oracle.conceal(images[b.img], lost[b.img], [b], phi, M, N, rho_hat, gamma,
                                iters, method=method, classes=cls, table_cache=cache)
        res, g = per[0]
        out.append((res, g.reshape(-1)))
    return out


def compare_selections(sel_dev: np.ndarray, sel_ref: np.ndarray, cls: np.ndarray) -> bool:
    """Selections agree modulo classes of parallel atoms."""
    return bool(np.array_equal(cls[np.asarray(sel_dev)], cls[np.asarray(sel_ref)]))


def min_margin(res) -> float:
    best, second = res.best, res.second
    with np.errstate(invalid="ignore", divide="ignore"):
        m = np.where(best > 0, (best - second) / best, np.inf)
    return float(np.min(m))
