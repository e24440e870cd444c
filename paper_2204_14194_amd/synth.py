"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module produces *inputs only*: 8-bit test images, loss layouts (which
pixels are lost and which extrapolation area belongs to each lost block) and
dictionaries of basis functions.  It contains no step of the extrapolation
itself: no weighting function, no scalar products, no selection.  Both the
FP64 oracle and the HIP path consume what it returns.

The paper measures on natural 8-bit images with 16x16 lost blocks
(Section "Results for Arbitrary Basis Functions", Table II); the generators
below are seeded stand-ins with smooth oscillating texture plus sharp edges.

Dictionary conventions (the paper allows arbitrary, even only numerically
defined, basis functions, Section II):
  * an atom is a length M*N vector over the extrapolation area, pixel (m, n)
    at index m*N + n; a dictionary is a (K, M*N) float64 array;
  * 2-D transform atoms are separable, index k = k1*N + k2 with k1 the
    vertical frequency;
  * DCT-II rows are orthonormal; Walsh-Hadamard rows are in natural
    (Sylvester) order with entries +-1/sqrt(M);
  * video areas of T frames: an atom is a length T*M*N vector, sample
    (tau, m, n) at index (tau*M + m)*N + n; 3-D transform atoms are
    separable, index (kt*M + k1)*N + k2;
  * the DCT-II rows 0 and M/2 take exactly the values +-1/sqrt(M) in exact
    arithmetic, the same as two Walsh-Hadamard rows.  Both dictionaries use
    the identical float64 constant for those entries and the same outer
    product, so the resulting parallel atoms in DCT u WHT unions are
    bit-identical ("twins").
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

__all__ = [
    "synth_image", "dct_rows", "wht_rows", "separable_atoms", "dct2_atoms",
    "wht2_atoms", "gaussian_atoms", "dictionary", "dictionary_parts", "Block", "grid_layout",
    "parity_lattice_layout", "lost_mask", "round_to_f32", "area32_inputs",
    "area48_inputs", "area64_inputs", "clustered_layout", "clustered_dictionaries",
    "clustered_dictionary_parts", "clustered_inputs", "frame_losses", "synth_video",
    "separable_atoms3", "video_dictionary", "video_dictionary_parts", "video_lost_mask",
    "video_grid_layout", "video_inputs",
]


# ----------------------------------------------------------------------------
# images
# ----------------------------------------------------------------------------
def synth_image(H: int, W: int, seed: int, n_cos: int = 20, n_rect: int = 6,
                amp_max: float = 40.0, step_max: float = 80.0,
                f_max: float = 1.0 / 8.0) -> np.ndarray:
    """Seeded uint8 image: 128 + sum of ``n_cos`` random 2-D cosines
    (amplitude U[0, amp_max], frequency U[-f_max, f_max] cycles/px per axis,
    phase U[0, 2 pi)) + ``n_rect`` axis-aligned rectangles with value steps
    U[-step_max, step_max]; clipped to [0, 255] and rounded half-to-even.

    Draw order (fixed): amplitudes, vertical freqs, horizontal freqs, phases,
    then per rectangle: height, width, top, left, step.
    """
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.0, amp_max, n_cos)
    fy = rng.uniform(-f_max, f_max, n_cos)
    fx = rng.uniform(-f_max, f_max, n_cos)
    ph = rng.uniform(0.0, 2.0 * np.pi, n_cos)
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    img = np.full((H, W), 128.0)
    for a, v, u, p in zip(amp, fy, fx, ph):
        img += a * np.cos(2.0 * np.pi * (v * y + u * x) + p)
    for _ in range(n_rect):
        h = rng.uniform(H / 16.0, H / 2.0)
        w = rng.uniform(W / 16.0, W / 2.0)
        top = rng.uniform(0.0, H - h)
        left = rng.uniform(0.0, W - w)
        step = rng.uniform(-step_max, step_max)
        y0, y1 = int(round(top)), int(round(top + h))
        x0, x1 = int(round(left)), int(round(left + w))
        img[y0:y1, x0:x1] += step
    return np.rint(np.clip(img, 0.0, 255.0)).astype(np.uint8)


# ----------------------------------------------------------------------------
# dictionaries
# ----------------------------------------------------------------------------
def _inv_sqrt(M: int) -> float:
    return 1.0 / np.sqrt(float(M))


def dct_rows(M: int) -> np.ndarray:
    """(M, M) orthonormal 1-D DCT-II rows, row k = alpha_k cos(pi (2m+1) k / 2M).
    Rows 0 and M/2 are set to +-1/sqrt(M) exactly (their exact values)."""
    m = np.arange(M, dtype=np.float64)
    k = np.arange(M, dtype=np.float64)[:, None]
    rows = np.sqrt(2.0 / M) * np.cos(np.pi * (2.0 * m + 1.0) * k / (2.0 * M))
    c = _inv_sqrt(M)
    rows[0, :] = c
    if M % 2 == 0:
        # cos(pi (2m+1)/4) is +sqrt(2)/2 for m = 0, 3 (mod 4), -sqrt(2)/2 else
        sign = np.where(np.isin(np.arange(M) % 4, (0, 3)), 1.0, -1.0)
        rows[M // 2, :] = sign * c
    return rows


def wht_rows(M: int) -> np.ndarray:
    """(M, M) Walsh-Hadamard rows in natural (Sylvester) order:
    row k, entry m = (-1)^popcount(m & k) / sqrt(M).  M must be a power of 2."""
    if M <= 0 or (M & (M - 1)) != 0:
        raise ValueError("Walsh-Hadamard rows need a power-of-two length")
    m = np.arange(M)
    k = np.arange(M)[:, None]
    parity = np.vectorize(lambda v: bin(int(v)).count("1") & 1)(m & k)
    return np.where(parity == 0, 1.0, -1.0) * _inv_sqrt(M)


def separable_atoms(rows_v: np.ndarray, rows_h: np.ndarray) -> np.ndarray:
    """2-D atoms phi_{k1*N+k2}[m*N+n] = rows_v[k1, m] * rows_h[k2, n]."""
    Kv, M = rows_v.shape
    Kh, N = rows_h.shape
    out = rows_v[:, None, :, None] * rows_h[None, :, None, :]
    return np.ascontiguousarray(out.reshape(Kv * Kh, M * N))


def dct2_atoms(M: int, N: int) -> np.ndarray:
    return separable_atoms(dct_rows(M), dct_rows(N))


def wht2_atoms(M: int, N: int) -> np.ndarray:
    return separable_atoms(wht_rows(M), wht_rows(N))


def gaussian_atoms(M: int, N: int, count: int, seed: int) -> np.ndarray:
    """``count`` numerically defined atoms: i.i.d. N(0,1) samples, each row
    scaled to unit L2 norm over the M x N area."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((count, M * N))
    return a / np.linalg.norm(a, axis=1, keepdims=True)


def _dft_phase(M: int, N: int):
    """Phase index q = (mu m N + eta n M) mod MN of the 2-D DFT atom
    (mu, eta) at pixel (m, n), atom mu*N + eta, pixel m*N + n: the atom is
    exp(j 2 pi q / MN)."""
    mu = np.arange(M)[:, None, None, None]
    eta = np.arange(N)[None, :, None, None]
    m = np.arange(M)[None, None, :, None]
    n = np.arange(N)[None, None, None, :]
    q = (mu * m * N + eta * n * M) % (M * N)
    return q.reshape(M * N, M * N)


def dft2_atoms(M: int, N: int) -> np.ndarray:
    """Complex 2-D DFT atoms exp(j 2 pi mu m / M) exp(j 2 pi eta n / N)
    (Section VI), scaled to unit norm over the M x N area; atom mu*N + eta."""
    q = _dft_phase(M, N)
    return np.exp(2j * np.pi * q / (M * N)) / np.sqrt(float(M * N))


def bdft2_atoms(M: int, N: int) -> np.ndarray:
    """Binarized 2-D DFT atoms: each of the real and imaginary parts of the
    DFT atom replaced by its sign (+1 where it is 0), scaled to unit norm.
    The signs are decided on the integer phase index, so no rounding enters."""
    q = _dft_phase(M, N)
    Q = M * N
    re = np.where((4 * q <= Q) | (4 * q >= 3 * Q), 1.0, -1.0)   # cos >= 0
    im = np.where(2 * q <= Q, 1.0, -1.0)                         # sin >= 0
    return (re + 1j * im) / np.sqrt(2.0 * Q)


def dictionary(M: int, N: int, parts: Sequence[str], seed: int = 101,
               n_gauss: int = 0) -> np.ndarray:
    """Union of sub-dictionaries, in the order given: 'dct', 'wht', 'gauss'
    (real), 'dft', 'bdft' (complex; the union is then complex)."""
    blocks = []
    for p in parts:
        if p == "dct":
            blocks.append(dct2_atoms(M, N))
        elif p == "wht":
            blocks.append(wht2_atoms(M, N))
        elif p == "gauss":
            blocks.append(gaussian_atoms(M, N, n_gauss, seed))
        elif p == "dft":
            blocks.append(dft2_atoms(M, N))
        elif p == "bdft":
            blocks.append(bdft2_atoms(M, N))
        else:
            raise ValueError(p)
    return np.ascontiguousarray(np.concatenate(blocks, axis=0))


def dictionary_parts(M: int, N: int, parts: Sequence[str], n_gauss: int = 0):
    """Where the transform sub-dictionaries of dictionary(M, N, parts, ...)
    start: a list of (name, first atom) for each 'dct', 'wht' and 'dft' part
    (binarized DFT and Gaussian atoms have no transform)."""
    out, first = [], 0
    for p in parts:
        if p in ("dct", "wht", "dft"):
            out.append((p, first))
        first += n_gauss if p == "gauss" else M * N
    return out


def round_to_f32(a: np.ndarray) -> np.ndarray:
    """Round to the nearest float32 and return float64 (complex64 ->
    complex128 for a complex array): the exact values a float32 device buffer
    holds, so both sides start from identical inputs."""
    if np.iscomplexobj(a):
        return np.asarray(a, dtype=np.complex64).astype(np.complex128)
    return np.asarray(a, dtype=np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# loss layouts
# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Block:
    """One lost block and its extrapolation area.

    img      : index of the image the block lies in
    y0, x0   : top-left corner of the M x N extrapolation area (image coords,
               may lie partly outside the image)
    ly, lx   : top-left corner of the loss rectangle, relative to the area
    lh, lw   : loss rectangle size
    lt, ld   : for areas of several video frames (img then the area's first
               frame): the loss covers frames lt .. lt+ld-1 of the area
    """
    img: int
    y0: int
    x0: int
    ly: int
    lx: int
    lh: int
    lw: int
    lt: int = 0
    ld: int = 1


def grid_layout(H: int, W: int, cell: int, loss: int, n_img: int = 1) -> List[Block]:
    """One centred ``loss`` x ``loss`` block in every ``cell`` x ``cell`` cell of
    each H x W image; the area is the cell itself."""
    off = (cell - loss) // 2
    out = []
    for i in range(n_img):
        for cy in range(H // cell):
            for cx in range(W // cell):
                out.append(Block(i, cy * cell, cx * cell, off, off, loss, loss))
    return out


def parity_lattice_layout(H: int, W: int, loss: int, area: int, seed: int,
                          margin: int, n_img: int = 1) -> List[Block]:
    """One loss per 2x2 group of the ``loss``-pixel block grid, all on one seeded
    parity lattice, so no area holds a second loss.  Coordinates are in a
    canvas that extends the H x W image by ``margin`` pixels on every side."""
    rng = np.random.default_rng(seed)
    py, px = (int(v) for v in rng.integers(0, 2, size=2))
    off = (area - loss) // 2
    out = []
    for i in range(n_img):
        for by in range(py, H // loss, 2):
            for bx in range(px, W // loss, 2):
                y = margin + by * loss
                x = margin + bx * loss
                out.append(Block(i, y - off, x - off, off, off, loss, loss))
    return out


def lost_mask(H: int, W: int, blocks: Sequence[Block], img: int = 0) -> np.ndarray:
    """uint8 mask, 1 where a pixel of image ``img`` is lost."""
    mask = np.zeros((H, W), dtype=np.uint8)
    for b in blocks:
        if b.img != img:
            continue
        y, x = b.y0 + b.ly, b.x0 + b.lx
        mask[max(y, 0):max(y + b.lh, 0), max(x, 0):max(x + b.lw, 0)] = 1
    return mask


# ----------------------------------------------------------------------------
# the workloads (one geometry each)
# ----------------------------------------------------------------------------
def area32_inputs(n_img: int = 1, seed0: int = 0):
    """128x128 images (seeds seed0..), 4x4 grid of 32x32 areas with centred
    8x8 losses (support width 12); K = 2048 (DCT-II 32^2 u WHT 32^2);
    rho_hat = 0.8, gamma = 0.5, I = 100."""
    imgs = np.stack([synth_image(128, 128, seed0 + i) for i in range(n_img)])
    blocks = grid_layout(128, 128, 32, 8, n_img)
    phi = dictionary(32, 32, ("dct", "wht"))
    return dict(images=imgs, blocks=blocks, phi=phi, M=32, N=32,
                tx_parts=dictionary_parts(32, 32, ("dct", "wht")),
                rho_hat=0.8, gamma=0.5, iters=100)


def dft32_inputs(n_img: int = 1, seed0: int = 0):
    """The 32x32-area layout of area32_inputs with the complex dictionary of
    the paper's Fig. 1 (bottom row): 2-D DFT 32^2 u binarized DFT 32^2
    (K = 2048); rho_hat = 0.8, gamma = 0.5, I = 100."""
    imgs = np.stack([synth_image(128, 128, seed0 + i) for i in range(n_img)])
    blocks = grid_layout(128, 128, 32, 8, n_img)
    phi = dictionary(32, 32, ("dft", "bdft"))
    return dict(images=imgs, blocks=blocks, phi=phi, M=32, N=32,
                tx_parts=dictionary_parts(32, 32, ("dft", "bdft")),
                rho_hat=0.8, gamma=0.5, iters=100)


def area48_inputs(n_img: int = 1, seed0: int = 1, layout_seed: int = 7):
    """512x512 image generated on a 544x544 canvas (areas read from the
    canvas); 256 isolated 16x16 losses on one parity lattice of the 16-px
    grid; area 48x48; K = 4096 (DCT 48^2 u 1792 seeded Gaussian atoms);
    rho_hat = 0.8, gamma = 0.5, I = 200."""
    imgs = np.stack([synth_image(544, 544, seed0 + i) for i in range(n_img)])
    blocks = parity_lattice_layout(512, 512, 16, 48, layout_seed, 16, n_img)
    phi = dictionary(48, 48, ("dct", "gauss"), seed=101, n_gauss=1792)
    return dict(images=imgs, blocks=blocks, phi=phi, M=48, N=48,
                tx_parts=dictionary_parts(48, 48, ("dct", "gauss"), 1792),
                rho_hat=0.8, gamma=0.5, iters=200)


def area64_inputs(n_img: int = 1, seed0: int = 300):
    """2048x2048 image, 1024 64x64 areas with centred 16x16 losses;
    K = 8192 (DCT 64^2 u WHT 64^2); rho_hat = 0.8, gamma = 0.5, I = 300."""
    imgs = np.stack([synth_image(2048, 2048, seed0 + i) for i in range(n_img)])
    blocks = grid_layout(2048, 2048, 64, 16, n_img)
    phi = dictionary(64, 64, ("dct", "wht"))
    return dict(images=imgs, blocks=blocks, phi=phi, M=64, N=64,
                tx_parts=dictionary_parts(64, 64, ("dct", "wht")),
                rho_hat=0.8, gamma=0.5, iters=300)


def clustered_layout(H: int, W: int, n_blocks: int, seed: int, img: int = 0,
                     n_centres=(3, 6), blob_sigma: float = 0.08,
                     burst_frac: float = 0.3, burst_len=(4, 16)):
    """Losses of a damaged frame: 8x8 and 16x16 lost blocks on the 8-pixel grid,
    partly clustered (Gaussian blobs around 3-6 seeded centres, sigma given as
    a fraction of the frame size) and partly in bursts (runs of 4-16 adjacent
    grid cells along a raster row).  Losses never overlap.  Each loss gets an
    extrapolation area centred on it: 8x8 -> 24 or 32, 16x16 -> 32 or 48
    (seeded).  Returns a list of Block (area coordinates may leave the
    frame)."""
    rng = np.random.default_rng(seed)
    gh, gw = H // 8, W // 8
    occ = np.zeros((gh, gw), dtype=bool)
    out: List[Block] = []
    centres = rng.uniform(0.1, 0.9, size=(int(rng.integers(n_centres[0], n_centres[1] + 1)), 2))

    def place(cy: int, cx: int, size: int) -> bool:
        c = size // 8
        if cy < 0 or cx < 0 or cy + c > gh or cx + c > gw or occ[cy:cy + c, cx:cx + c].any():
            return False
        occ[cy:cy + c, cx:cx + c] = True
        if size == 8:
            area = 24 if rng.random() < 0.5 else 32
        else:
            area = 32 if rng.random() < 0.5 else 48
        off = (area - size) // 2
        out.append(Block(img, cy * 8 - off, cx * 8 - off, off, off, size, size))
        return True

    tries = 0
    while len(out) < n_blocks and tries < 200 * n_blocks:
        tries += 1
        size = 16 if rng.random() < 0.4 else 8
        if rng.random() < burst_frac:
            cy = int(rng.integers(0, gh))
            cx = int(rng.integers(0, gw))
            run = int(rng.integers(burst_len[0], burst_len[1] + 1))
            for k in range(run):
                if len(out) >= n_blocks:
                    break
                if not place(cy, cx + k * (size // 8), size):
                    break
        else:
            c = centres[int(rng.integers(0, len(centres)))]
            y = int(rng.normal(c[0], blob_sigma) * gh)
            x = int(rng.normal(c[1], blob_sigma) * gw)
            if size == 16:
                y, x = y - y % 2, x - x % 2
            place(y, x, size)
    return out


def clustered_dictionaries():
    """Dictionary per area size for the uneven workload: DCT u WHT for 32x32
    (K = 2048), DCT u seeded Gaussian atoms for 24x24 and 48x48 (no Sylvester
    Walsh-Hadamard exists there), K = 2 * area pixels."""
    return {24: dictionary(24, 24, ("dct", "gauss"), seed=124, n_gauss=576),
            32: dictionary(32, 32, ("dct", "wht")),
            48: dictionary(48, 48, ("dct", "gauss"), seed=148, n_gauss=2304)}


def clustered_dictionary_parts():
    """The transform ranges of clustered_dictionaries(), per area size."""
    return {24: dictionary_parts(24, 24, ("dct", "gauss"), 576),
            32: dictionary_parts(32, 32, ("dct", "wht")),
            48: dictionary_parts(48, 48, ("dct", "gauss"), 2304)}


def clustered_inputs(n_img: int = 8, blocks_per_img: int = 500, seed0: int = 200,
                iter_range=(100, 200)):
    """8 seeded 1024x1024 frames with clustered/burst losses, 500 blocks each;
    per-block iteration counts I ~ U{100..200}; rho_hat = 0.8, gamma = 0.5."""
    imgs = np.stack([synth_image(1024, 1024, seed0 + i) for i in range(n_img)])
    blocks: List[Block] = []
    for i in range(n_img):
        blocks += clustered_layout(1024, 1024, blocks_per_img, seed=seed0 + 1000 + i, img=i)
    rng = np.random.default_rng(seed0 + 99)
    iters = rng.integers(iter_range[0], iter_range[1] + 1, size=len(blocks))
    return dict(images=imgs, blocks=blocks, iters=iters, dicts=clustered_dictionaries(),
                tx_parts=clustered_dictionary_parts(), rho_hat=0.8, gamma=0.5)


def frame_losses(H: int, W: int, coverage: float, seed: int, p16: float = 0.5,
                 p64: float = 0.5):
    """Lost blocks of one frame for serving: 8x8 and 16x16 losses on the
    8-pixel grid, placed uniformly at random without overlap until
    ``coverage`` of the frame is lost.  Returns (y, x, h, w, basis) tuples
    with basis 0 for 8x8 losses (32x32 areas), and 1 (48x48) or 2 (64x64)
    for 16x16 losses."""
    rng = np.random.default_rng(seed)
    gh, gw = H // 8, W // 8
    occ = np.zeros((gh, gw), dtype=bool)
    out = []
    lost = 0
    target = coverage * H * W
    tries = 0
    while lost < target and tries < 100000:
        tries += 1
        big = rng.random() < p16
        c = 2 if big else 1
        cy = int(rng.integers(0, gh - c + 1))
        cx = int(rng.integers(0, gw - c + 1))
        if big:
            cy, cx = cy - cy % 2, cx - cx % 2
        if occ[cy:cy + c, cx:cx + c].any():
            continue
        occ[cy:cy + c, cx:cx + c] = True
        s = 8 * c
        basis = 0 if not big else (2 if rng.random() < p64 else 1)
        out.append((cy * 8, cx * 8, s, s, basis))
        lost += s * s
    return out


# ----------------------------------------------------------------------------
# video: areas of T consecutive frames
# ----------------------------------------------------------------------------
def synth_video(F: int, H: int, W: int, seed: int, max_speed: int = 2) -> np.ndarray:
    """Seeded uint8 video of F frames of H x W: one synthetic image (seed
    ``seed + 1``) on a canvas larger by the whole motion, seen through a
    window that moves by a seeded integer velocity (vy, vx), each component
    uniform in [-max_speed, max_speed] pixels per frame (global translation,
    as in a camera pan).  Draw order: vy, vx."""
    rng = np.random.default_rng(seed)
    vy, vx = (int(v) for v in rng.integers(-max_speed, max_speed + 1, size=2))
    R = max_speed * max(F - 1, 0)
    canvas = synth_image(H + 2 * R, W + 2 * R, seed + 1)
    frames = [canvas[R + vy * f:R + vy * f + H, R + vx * f:R + vx * f + W] for f in range(F)]
    return np.ascontiguousarray(np.stack(frames))


def separable_atoms3(rows_t: np.ndarray, rows_v: np.ndarray, rows_h: np.ndarray) -> np.ndarray:
    """3-D atoms phi_{(kt*Kv + k1)*Kh + k2}[(tau*M + m)*N + n] =
    (rows_t[kt, tau] * rows_v[k1, m]) * rows_h[k2, n]."""
    Kt, T = rows_t.shape
    Kv, M = rows_v.shape
    Kh, N = rows_h.shape
    tv = rows_t[:, None, :, None] * rows_v[None, :, None, :]          # (Kt, Kv, T, M)
    out = tv[:, :, None, :, :, None] * rows_h[None, None, :, None, None, :]
    return np.ascontiguousarray(out.reshape(Kt * Kv * Kh, T * M * N))


def video_dictionary(T: int, M: int, N: int, parts: Sequence[str] = ("dct", "wht")) -> np.ndarray:
    """Union of 3-D separable transform dictionaries over T x M x N areas, in
    the order given: 'dct' (DCT-II along every axis) and 'wht' (Walsh-Hadamard,
    powers of two).  Parallel atoms of the two halves are bit-identical (the
    same constants and the same product order)."""
    rows = {"dct": dct_rows, "wht": wht_rows}
    return np.ascontiguousarray(np.concatenate(
        [separable_atoms3(rows[p](T), rows[p](M), rows[p](N)) for p in parts], axis=0))


def video_dictionary_parts(T: int, M: int, N: int, parts: Sequence[str] = ("dct", "wht")):
    """Where the sub-dictionaries of video_dictionary(T, M, N, parts) start:
    (name, first atom) per part."""
    return [(p, i * T * M * N) for i, p in enumerate(parts)]


def video_lost_mask(F: int, H: int, W: int, blocks: Sequence[Block]) -> np.ndarray:
    """uint8 (F, H, W) mask, 1 on every lost sample (each block's loss box:
    frames img+lt .. img+lt+ld-1)."""
    mask = np.zeros((F, H, W), dtype=np.uint8)
    for b in blocks:
        f0 = b.img + b.lt
        y, x = b.y0 + b.ly, b.x0 + b.lx
        mask[max(f0, 0):max(f0 + b.ld, 0), max(y, 0):max(y + b.lh, 0),
             max(x, 0):max(x + b.lw, 0)] = 1
    return mask


def video_grid_layout(F: int, H: int, W: int, T: int, cell: int, loss: int,
                      lt: int) -> List[Block]:
    """Losses in every T-th frame: the areas span frames T j .. T j + T - 1
    (j = 0 .. F/T - 1) and every cell x cell cell of the frame, each with a
    centred loss x loss rectangle in frame lt of the area.  No area holds a
    second loss, so every block has the same weight pattern."""
    off = (cell - loss) // 2
    out = []
    for j in range(F // T):
        for cy in range(H // cell):
            for cx in range(W // cell):
                out.append(Block(j * T, cy * cell, cx * cell, off, off, loss, loss, lt, 1))
    return out


def video_inputs(n_videos: int = 1, frames: int = 8, seed0: int = 500):
    """``n_videos`` seeded videos of ``frames`` 128x128 frames each, stacked
    into one batch of frames; areas of T = 4 frames x 16 x 16 pixels, one
    centred 8x8 loss in frame 2 of every area (two frames before it, one
    after), every 16x16 cell of every fourth frame; K = 2048 (3-D DCT-II
    4x16x16 u 3-D WHT 4x16x16); rho_hat = 0.8, gamma = 0.5, I = 100."""
    T, M, N = 4, 16, 16
    vids = [synth_video(frames, 128, 128, seed0 + 10 * v) for v in range(n_videos)]
    blocks: List[Block] = []
    for v in range(n_videos):
        for b in video_grid_layout(frames, 128, 128, T, 16, 8, 2):
            blocks.append(dataclasses.replace(b, img=b.img + v * frames))
    return dict(frames=np.concatenate(vids, axis=0), blocks=blocks,
                phi=video_dictionary(T, M, N), T=T, M=M, N=N,
                tx_parts=video_dictionary_parts(T, M, N),
                rho_hat=0.8, gamma=0.5, iters=100)
