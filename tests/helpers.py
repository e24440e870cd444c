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
    """Smallest relative gap between the winning score |R_u| D_u and the best
    score outside the winner's class, over all iterations."""
    best, second = np.sqrt(res.best), np.sqrt(res.second)
    with np.errstate(invalid="ignore", divide="ignore"):
        m = np.where(best > 0, (best - second) / best, np.inf)
    return float(np.min(m))


def _check_block(i, s, w, phi, cls, cache, gamma, iters, sel_i, g_i, loss_idx, got, tol, delta,
                 pasted=None, q14=False):
    """One block of oracle_check: returns (err, margin, agreed).  ``got``: the
    pasted values of the loss samples selected by ``pasted`` (all if None).
    ``q14``: the reference runs on the table's 16-bit fixed-point words."""
    key = w.tobytes()
    if key not in cache:
        C, D = oracle.table_generation(phi, w)
        Gq = None
        if q14:
            Gq = oracle.quantise_table(oracle.unit_table(C, D)).astype(np.float64) * 2.0 ** -14
        cache[key] = (C, D, Gq)
    C, D, Gq = cache[key]

    def run(forced=None):
        if q14:
            return oracle.fase_unit(s, w, phi, Gq, D, gamma, iters, cls, forced=forced)
        return oracle.fase(s, w, phi, C, D, gamma, iters, cls, forced=forced)
    res = run()
    margin = min_margin(res)
    agreed = compare_selections(sel_i, res.sel, cls)
    if agreed:
        ref = res
    else:
        ref = run(forced=sel_i)
        ok = np.sqrt(ref.picked) >= np.sqrt(ref.best) * (1.0 - delta)
        assert ok.all(), (f"block {i}: iteration {int(np.argmin(ok))} picked an atom "
                          f"outside the near-tie window")
    # the model's real part replaces the loss (a complex dictionary gives a
    # complex model)
    gref = np.real(ref.g)[loss_idx]
    n = len(loss_idx)
    err = float(np.abs(g_i[:n].astype(np.float64) - gref).max())
    assert err <= tol, f"block {i}: max |g - g_oracle| = {err}"
    if pasted is not None:
        gref = gref[pasted]
    q_ref = np.clip(np.rint(gref), 0, 255)
    near = np.abs(np.abs(gref - np.floor(gref)) - 0.5) < tol
    assert ((got.astype(np.float64) == q_ref) | near).all(), f"block {i}: pasted pixels differ"
    return err, margin, agreed


def oracle_check(images, blocks, phi, M, N, rho_hat, gamma, iters, sel, g, out,
                 sample=None, tol=1e-3, delta=1e-3, q14=False):
    """Compare device results with the FP64 oracle (Algorithm 3, which the CPU
    pins tie to Algorithm 1) block by block.

    Where the device's selections equal the oracle's (modulo classes of
    parallel atoms) the model over the loss must agree within ``tol``.  Where
    they differ, the difference must come from a near-tie: the oracle is
    re-run along the device's selections and every device pick must score
    within the relative window ``delta`` of that iteration's best score; the
    model must then agree with that run within ``tol``.  In both cases the
    pasted pixels are the rounded model.  ``q14``: the oracle runs Algorithm 3
    on the 16-bit fixed-point words of its own table (oracle.fase_unit).
    Returns dict(worst, margin, agree, n)."""
    n_img, H, W = images.shape
    lost = np.stack([synth.lost_mask(H, W, blocks, i) for i in range(n_img)])
    cls = classes_of(phi)
    idx = list(range(len(blocks))) if sample is None else [int(i) for i in sample]
    cache = {}
    worst, margin, agree = 0.0, np.inf, 0
    for i in idx:
        b = blocks[i]
        s, sup = oracle.area_signal(images[b.img], lost[b.img], b.y0, b.x0, M, N)
        w = oracle.area_weights(M, N, rho_hat, sup)
        loss_idx = (np.arange(M)[b.ly:b.ly + b.lh, None] * N
                    + np.arange(N)[None, b.lx:b.lx + b.lw]).reshape(-1)
        y, x = b.y0 + b.ly, b.x0 + b.lx
        got = out[b.img, y:y + b.lh, x:x + b.lw].reshape(-1)
        err, mg, ok = _check_block(i, s, w, phi, cls, cache, gamma, iters, sel[i], g[i],
                                   loss_idx, got, tol, delta, q14=q14)
        worst, margin, agree = max(worst, err), min(margin, mg), agree + int(ok)
    return dict(worst=worst, margin=margin, agree=agree, n=len(idx))


def oracle_check_video(frames, blocks, phi, T, M, N, rho_hat, gamma, iters, sel, g, out,
                       sample=None, tol=1e-3, delta=1e-3, q14=False):
    """oracle_check for areas of T consecutive frames (blocks with lt, ld;
    the model over the loss box in frames x rows x columns order).  Loss
    samples outside the frames are compared in the model only."""
    F, H, W = frames.shape
    lost = synth.video_lost_mask(F, H, W, blocks)
    cls = classes_of(phi)
    idx = list(range(len(blocks))) if sample is None else [int(i) for i in sample]
    cache = {}
    worst, margin, agree = 0.0, np.inf, 0
    for i in idx:
        b = blocks[i]
        s, sup = oracle.volume_signal(frames, lost, b.img, b.y0, b.x0, T, M, N)
        w = oracle.volume_weights(T, M, N, rho_hat, sup)
        tt, mm, nn = np.meshgrid(np.arange(b.lt, b.lt + b.ld), np.arange(b.ly, b.ly + b.lh),
                                 np.arange(b.lx, b.lx + b.lw), indexing="ij")
        loss_idx = ((tt * M + mm) * N + nn).reshape(-1)
        ff = (b.img + tt).reshape(-1)
        yy = (b.y0 + mm).reshape(-1)
        xx = (b.x0 + nn).reshape(-1)
        inside = (ff >= 0) & (ff < F) & (yy >= 0) & (yy < H) & (xx >= 0) & (xx < W)
        got = out[ff[inside], yy[inside], xx[inside]]
        err, mg, ok = _check_block(i, s, w, phi, cls, cache, gamma, iters, sel[i], g[i],
                                   loss_idx, got, tol, delta, pasted=inside, q14=q14)
        worst, margin, agree = max(worst, err), min(margin, mg), agree + int(ok)
    return dict(worst=worst, margin=margin, agree=agree, n=len(idx))
