"""ctypes binding of libsefase (include/se.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the method runs in the library's HIP kernels.  There is
no fallback: if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsefase.so")

SE_OK, SE_EINVAL, SE_ENOMEM, SE_EHIP, SE_EAGAIN, SE_EBUSY, SE_ENUMERIC, SE_ECANCELED = (
    0, -1, -2, -3, -4, -5, -6, -7)
SE_FP32, SE_BF16X3 = 0, 1
SE_DIAG_AUTO, SE_DIAG_FP64, SE_DIAG_FP32 = 0, 1, 2
SE_ROWS_Q14 = 1   # se_params.flags: the loop reads the fixed-point class rows
SE_ROWS_BF16X3 = 2   # se_params.flags: rows on demand from split-BF16 products
SE_INVARIANT = 4     # se_params.flags: products in one pass, independent of the batch
SE_PART_DCT2, SE_PART_WHT2, SE_PART_DFT2 = 1, 2, 3

# every symbol include/se.h declares
EXPORTED = (
    "se_last_error", "se_version", "se_area_weights_ws_bytes", "se_area_weights",
    "se_volume_weights",
    "se_weighted_gram_ws_bytes", "se_weighted_gram", "se_extrapolate_batch_ws_bytes",
    "se_extrapolate_batch", "se_extrapolate_plain", "se_blocks_upload", "se_project_ws_bytes",
    "se_project", "se_iterate", "se_extrapolate_device_ws_bytes", "se_extrapolate_device",
    "se_table_ld", "se_tables_tx_bytes",
    "se_extrapolate_ondemand_ws_bytes", "se_extrapolate_ondemand",
    "se_extrapolate_batch_static",
)

# bytes of the library's static scratch (se_extrapolate_batch_static)
SE_STATIC_SCRATCH_BYTES = 16 << 20


class SEError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsefase error {code}: {msg}")
        self.code = code


class se_part(C.Structure):
    _fields_ = [("kind", C.c_int32), ("first", C.c_int32)]


class se_basis(C.Structure):
    _fields_ = [("M", C.c_int32), ("N", C.c_int32), ("K", C.c_int32), ("phi", C.c_void_p),
                ("n_parts", C.c_int32), ("parts", se_part * 2), ("phi_im", C.c_void_p),
                ("T", C.c_int32)]


_PART_NAMES = {"dct": SE_PART_DCT2, "wht": SE_PART_WHT2, "dft": SE_PART_DFT2}


def _parts_arg(parts) -> tuple:
    """(kind, first) pairs; kind an SE_PART_* value or 'dct' / 'wht' / 'dft'."""
    parts = tuple((_PART_NAMES[k] if isinstance(k, str) else int(k), int(f)) for k, f in parts)
    if len(parts) > 2:
        raise ValueError("at most two transform parts")
    return parts


def _part_array(parts):
    arr = (se_part * 2)()
    for i, (k, f) in enumerate(parts):
        arr[i] = se_part(k, f)
    return arr


def make_basis(M: int, N: int, K: int, phi_ptr, parts=(), phi_im_ptr=None, T: int = 1) -> se_basis:
    """se_basis for a dictionary at device address ``phi_ptr``; ``parts`` is a
    sequence of (SE_PART_*, first atom) transform ranges; ``phi_im_ptr`` the
    imaginary parts of a complex dictionary (None for a real one); ``T`` the
    frames per area (atoms over T*M*N samples)."""
    parts = _parts_arg(parts)
    return se_basis(M, N, K, phi_ptr, len(parts), _part_array(parts), phi_im_ptr, int(T))


class se_block(C.Structure):
    _fields_ = [(n, C.c_int32)
                for n in ("img", "y0", "x0", "ly", "lx", "lh", "lw", "geom", "lt", "ld")]


BLOCK_INTS = 10   # int32 fields of se_block


class se_tables(C.Structure):
    _fields_ = [("M", C.c_int32), ("N", C.c_int32), ("K", C.c_int32), ("ldG", C.c_int32),
                ("G", C.c_void_p), ("D", C.c_void_p), ("Y", C.c_void_p),
                ("sqrtw", C.c_void_p), ("phi", C.c_void_p), ("info", C.c_void_p),
                ("precision", C.c_int32), ("Yhi", C.c_void_p), ("Ylo", C.c_void_p),
                ("n_parts", C.c_int32), ("parts", se_part * 2), ("tx", C.c_void_p),
                ("G_im", C.c_void_p), ("phi_im", C.c_void_p), ("T", C.c_int32),
                ("Gc", C.c_void_p), ("cls", C.c_void_p), ("n_classes", C.c_int32),
                ("Gq", C.c_void_p), ("Gq_rows", C.c_void_p)]


class se_params(C.Structure):
    _fields_ = [("gamma", C.c_float), ("iters", C.c_int32), ("flags", C.c_uint32)]


_lib = None


def lib():
    """Open libsefase.so (once).  Raises if it is missing: there is no other
    implementation to fall back to."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                           "`python -m paper_2204_14194_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, f32, sz = C.c_void_p, C.c_int32, C.c_float, C.c_size_t
    L.se_last_error.restype = C.c_char_p
    L.se_version.restype = i32
    L.se_table_ld.restype = i32
    L.se_table_ld.argtypes = [i32]
    L.se_tables_tx_bytes.restype = sz
    L.se_tables_tx_bytes.argtypes = [i32, i32, i32]
    L.se_area_weights_ws_bytes.restype = sz
    L.se_area_weights_ws_bytes.argtypes = [i32]
    L.se_area_weights.restype = i32
    L.se_area_weights.argtypes = [i32, i32, f32, vp, i32, i32, i32, vp, i32, vp, vp, sz, vp]
    L.se_volume_weights.restype = i32
    L.se_volume_weights.argtypes = [i32, i32, i32, f32, vp, i32, i32, i32, vp, i32, vp, vp, sz, vp]
    L.se_weighted_gram_ws_bytes.restype = sz
    L.se_weighted_gram_ws_bytes.argtypes = [C.POINTER(se_basis), i32]
    L.se_weighted_gram.restype = i32
    L.se_weighted_gram.argtypes = [C.POINTER(se_basis), vp, i32, C.c_uint32,
                                   C.POINTER(se_tables), vp, sz, vp]
    L.se_extrapolate_batch_ws_bytes.restype = sz
    L.se_extrapolate_batch_ws_bytes.argtypes = [C.POINTER(se_tables), i32]
    for name in ("se_extrapolate_batch", "se_extrapolate_plain"):
        f = getattr(L, name)
        f.restype = i32
        f.argtypes = [C.POINTER(se_tables), vp, i32, i32, i32, vp, i32, se_params, vp, vp, vp,
                      i32, vp, sz, vp]
    L.se_extrapolate_batch_static.restype = i32
    L.se_extrapolate_batch_static.argtypes = [C.POINTER(se_tables), vp, i32, i32, i32, vp, i32,
                                              se_params, vp, vp, vp, i32, vp]
    L.se_blocks_upload.restype = i32
    L.se_blocks_upload.argtypes = [C.POINTER(se_tables), i32, i32, i32, vp, i32, vp,
                                   C.POINTER(C.c_int32), vp]
    L.se_project_ws_bytes.restype = sz
    L.se_project_ws_bytes.argtypes = [C.POINTER(se_tables), i32]
    L.se_project.restype = i32
    L.se_project.argtypes = [C.POINTER(se_tables), vp, i32, i32, i32, vp, i32, vp, i32, vp, sz,
                             vp]
    L.se_iterate.restype = i32
    L.se_iterate.argtypes = [C.POINTER(se_tables), vp, i32, vp, i32, i32, i32, vp, i32,
                             se_params, vp, vp, vp, i32, vp]
    L.se_extrapolate_device_ws_bytes.restype = sz
    L.se_extrapolate_device_ws_bytes.argtypes = [C.POINTER(se_tables), i32]
    L.se_extrapolate_device.restype = i32
    L.se_extrapolate_device.argtypes = [C.POINTER(se_tables), vp, i32, i32, i32, vp, i32,
                                        se_params, vp, vp, vp, i32, vp, sz, vp]
    L.se_extrapolate_ondemand_ws_bytes.restype = sz
    L.se_extrapolate_ondemand_ws_bytes.argtypes = [C.POINTER(se_basis), i32, i32]
    L.se_extrapolate_ondemand.restype = i32
    L.se_extrapolate_ondemand.argtypes = [C.POINTER(se_basis), vp, vp, i32, i32, i32, vp, i32,
                                          se_params, vp, vp, vp, vp, i32, vp, sz, vp]
    L.se_ondemand_prepare.restype = i32
    L.se_ondemand_prepare.argtypes = [C.POINTER(se_basis), C.c_uint32, C.POINTER(vp), vp]
    L.se_ondemand_release.restype = None
    L.se_ondemand_release.argtypes = [vp]
    L.se_ondemand_plan_ws_bytes.restype = sz
    L.se_ondemand_plan_ws_bytes.argtypes = [vp, i32, i32, i32]
    L.se_ondemand_plan_create.restype = i32
    L.se_ondemand_plan_create.argtypes = [vp, i32, i32, i32, vp, i32, se_params, vp, i32, vp, sz,
                                          vp, C.POINTER(vp)]
    L.se_ondemand_plan_info.restype = i32
    L.se_ondemand_plan_info.argtypes = [vp, vp, vp, vp]
    L.se_ondemand_run.restype = i32
    L.se_ondemand_run.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp]
    L.se_ondemand_plan_release.restype = None
    L.se_ondemand_plan_release.argtypes = [vp]
    L.se_autotune_ondemand.restype = i32
    L.se_autotune_ondemand.argtypes = [vp, vp, vp, i32, vp, vp]
    L.se_ondemand_extrapolate.restype = i32
    L.se_ondemand_extrapolate.argtypes = [vp, vp, vp, i32, i32, i32, vp, i32, se_params, vp, vp,
                                          vp, vp, i32, i32, vp, sz, vp]
    _lib = L
    return L


def _check(code: int):
    if code != SE_OK:
        raise SEError(code, lib().se_last_error().decode())


class SENumericError(SEError):
    """SE_ENUMERIC from a concealment call: the call finished every other
    block, but some blocks had no available sample in their area (they
    report sel = -1 and keep their loss).  ``results`` holds the outputs the
    call would have returned."""

    def __init__(self, code: int, msg: str, results):
        super().__init__(code, msg)
        self.results = results


def _check_results(code: int, results):
    """_check for concealment calls: their outputs travel with SE_ENUMERIC."""
    if code == SE_ENUMERIC:
        raise SENumericError(code, lib().se_last_error().decode(), results)
    _check(code)
    return results


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def blocks_array(blocks: Sequence) -> C.Array:
    """Host array of se_block from objects with img, y0, x0, ly, lx, lh, lw
    (and optionally geom, and lt, ld for a loss over several frames)."""
    arr = (se_block * max(len(blocks), 1))()
    for i, b in enumerate(blocks):
        arr[i] = se_block(b.img, b.y0, b.x0, b.ly, b.lx, b.lh, b.lw, getattr(b, "geom", 0),
                          getattr(b, "lt", 0), getattr(b, "ld", 1))
    return arr


def loss_size(b) -> int:
    """Samples in a block's loss (frames x rows x columns)."""
    return max(int(getattr(b, "ld", 1)), 1) * b.lh * b.lw


def version() -> int:
    return int(lib().se_version())


def table_ld(K: int) -> int:
    """se_table_ld: row stride of the table and of projection buffers."""
    ld = int(lib().se_table_ld(int(K)))
    if ld <= 0:
        raise ValueError(f"unsupported dictionary size K={K}")
    return ld


# ---------------------------------------------------------------------------
def area_weights(M: int, N: int, rho_hat: float, lost: torch.Tensor, blocks: Sequence,
                 stream=None, T: Optional[int] = None) -> torch.Tensor:
    """se_area_weights: per-block weights (n_blk, M*N) float32 on the device;
    with ``T``, se_volume_weights over T x M x N areas of consecutive frames
    (n_blk, T*M*N)."""
    L = lib()
    if not (lost.is_cuda and lost.dtype == torch.uint8 and lost.dim() == 3 and lost.is_contiguous()):
        raise ValueError("lost must be a contiguous (n_img, H, W) uint8 CUDA tensor")
    n_img, H, W = lost.shape
    n = len(blocks)
    F = 1 if T is None else int(T)
    w = torch.empty((n, F * M * N), dtype=torch.float32, device=lost.device)
    nb = L.se_area_weights_ws_bytes(n)
    ws = _workspace(nb, lost.device)
    arr = blocks_array(blocks)
    if T is None:
        _check(L.se_area_weights(M, N, float(rho_hat), _ptr(lost), n_img, H, W, arr, n, _ptr(w),
                                 _ptr(ws), nb, _stream(stream)))
    else:
        _check(L.se_volume_weights(F, M, N, float(rho_hat), _ptr(lost), n_img, H, W, arr, n,
                                   _ptr(w), _ptr(ws), nb, _stream(stream)))
    return w


@dataclass
class Tables:
    """Device tables of one weight pattern and the ctypes struct describing them."""
    M: int
    N: int
    K: int
    ldG: int
    G: torch.Tensor
    D: torch.Tensor
    Y: torch.Tensor
    sqrtw: torch.Tensor
    phi: torch.Tensor
    info: torch.Tensor
    precision: int
    Yhi: Optional[torch.Tensor] = None
    Ylo: Optional[torch.Tensor] = None
    parts: tuple = ()
    tx: Optional[torch.Tensor] = None
    G_im: Optional[torch.Tensor] = None
    phi_im: Optional[torch.Tensor] = None
    T: int = 1
    Gc: Optional[torch.Tensor] = None
    cls: Optional[torch.Tensor] = None
    n_classes: int = 0
    Gq: Optional[torch.Tensor] = None
    Gq_rows: Optional[torch.Tensor] = None

    @property
    def complex(self) -> bool:
        return self.phi_im is not None

    @property
    def ldR(self) -> int:
        """Row length of R (real parts, then imaginary parts for a complex
        dictionary)."""
        return (2 if self.complex else 1) * self.ldG

    def struct(self) -> se_tables:
        return se_tables(self.M, self.N, self.K, self.ldG, self.G.data_ptr(), self.D.data_ptr(),
                         self.Y.data_ptr(), self.sqrtw.data_ptr(), self.phi.data_ptr(),
                         self.info.data_ptr(), self.precision,
                         self.Yhi.data_ptr() if self.Yhi is not None else None,
                         self.Ylo.data_ptr() if self.Ylo is not None else None,
                         len(self.parts), _part_array(self.parts),
                         self.tx.data_ptr() if self.tx is not None else None,
                         self.G_im.data_ptr() if self.G_im is not None else None,
                         self.phi_im.data_ptr() if self.phi_im is not None else None, self.T,
                         self.Gc.data_ptr() if self.Gc is not None else None,
                         self.cls.data_ptr() if self.cls is not None else None, self.n_classes,
                         self.Gq.data_ptr() if self.Gq is not None else None,
                         self.Gq_rows.data_ptr() if self.Gq_rows is not None else None)

    def nbytes(self) -> int:
        parts = [self.G, self.D, self.Y, self.sqrtw]
        parts += [x for x in (self.Yhi, self.Ylo, self.G_im, self.Gc, self.cls, self.Gq,
                              self.Gq_rows) if x is not None]
        return sum(t.numel() * t.element_size() for t in parts)


def weighted_gram(phi: torch.Tensor, w: torch.Tensor, M: int, N: int,
                  precision: int = SE_FP32, flags: int = SE_DIAG_AUTO, stream=None,
                  parts=(), phi_im: Optional[torch.Tensor] = None, T: int = 1,
                  classes: bool = True, fixed_point: bool = False,
                  fixed_point_rows: bool = False) -> Tables:
    """se_weighted_gram (Algorithm 2) for dictionary ``phi`` (K, T*M*N) and
    weight pattern ``w`` (T*M*N,).  ``parts``: declared transform ranges, as
    (SE_PART_*, first atom) pairs (verified by the library).  ``phi_im``: the
    imaginary parts of a complex dictionary (``phi`` then holds the real
    parts); the tables are then complex (G, G_im).  ``T``: frames per area
    (1: two-dimensional areas).  ``classes``: offer buffers for the parity
    class tables (used when the library finds the class structure; then
    ``n_classes`` is 4).  ``fixed_point``: also offer the buffer of the class
    rows as 16-bit words with 14 fraction bits (``Gq``, kept only with class
    tables), which loops called with ``rows_q14=True`` read.
    ``fixed_point_rows``: also write every whole row of G in those words
    (``Gq_rows``, real dictionaries), which the loop over whole rows reads
    when called with ``rows_q14=True``."""
    L = lib()
    _dev_f32(phi, "phi")
    _dev_f32(w, "w")
    K = phi.shape[0]
    P = int(T) * M * N
    if phi.shape[1] != P or w.numel() != P:
        raise ValueError("phi must be (K, T*M*N) and w (T*M*N,)")
    if phi_im is not None:
        _dev_f32(phi_im, "phi_im")
        if tuple(phi_im.shape) != tuple(phi.shape):
            raise ValueError("phi_im must have the shape of phi")
    ldG = table_ld(K)
    dev = phi.device
    y_rows = 2 * K if phi_im is not None else K
    t = Tables(M, N, K, ldG,
               torch.empty((K, ldG), dtype=torch.float32, device=dev),
               torch.empty(K, dtype=torch.float32, device=dev),
               torch.empty((y_rows, P), dtype=torch.float32, device=dev),
               torch.empty(P, dtype=torch.float32, device=dev),
               phi, torch.zeros(1, dtype=torch.int32, device=dev), int(precision), T=int(T))
    if phi_im is not None:
        t.phi_im = phi_im
        t.G_im = torch.empty((K, ldG), dtype=torch.float32, device=dev)
    if precision == SE_BF16X3:
        t.Yhi = torch.empty((K, P), dtype=torch.int16, device=dev)
        t.Ylo = torch.empty((K, P), dtype=torch.int16, device=dev)
    t.parts = _parts_arg(parts)
    if t.parts:
        nb_tx = int(L.se_tables_tx_bytes(int(T) * M, N, len(t.parts)))
        if nb_tx == 0:
            raise ValueError(f"no transform parts for a {T}x{M}x{N} area")
        t.tx = torch.empty(nb_tx // 4, dtype=torch.float32, device=dev)
    if (classes and len(t.parts) == 2 and phi_im is None and M % 2 == 0 and N % 2 == 0
            and K % 1024 == 0 and ldG == K):
        t.Gc = torch.empty((K, K // 4), dtype=torch.float32, device=dev)
        t.cls = torch.empty((K, 2), dtype=torch.int32, device=dev)
        if fixed_point:
            t.Gq = torch.empty((K, K // 4), dtype=torch.int16, device=dev)
    if fixed_point_rows and phi_im is None:
        t.Gq_rows = torch.empty((K, ldG), dtype=torch.int16, device=dev)
    b = make_basis(M, N, K, phi.data_ptr(), t.parts,
                   phi_im.data_ptr() if phi_im is not None else None, int(T))
    nb = L.se_weighted_gram_ws_bytes(C.byref(b), int(precision))
    ws = _workspace(nb, dev)
    st = t.struct()
    _check(L.se_weighted_gram(C.byref(b), _ptr(w), int(precision), int(flags), C.byref(st),
                              _ptr(ws), nb, _stream(stream)))
    t.n_classes = int(st.n_classes)
    if t.n_classes == 0:
        t.Gc = t.cls = t.Gq = None
    return t


def extrapolate_batch_ws_bytes(t: Tables, n_blk: int) -> int:
    st = t.struct()
    return int(lib().se_extrapolate_batch_ws_bytes(C.byref(st), n_blk))


def _extrapolate(name: str, t: Tables, images: torch.Tensor, blocks: Sequence, gamma: float,
                 iters: int, want_sel: bool, want_coef: bool, want_g: bool,
                 ws: Optional[torch.Tensor], stream, blocks_arr=None, flags: int = 0):
    L = lib()
    if not (images.is_cuda and images.dtype == torch.uint8 and images.dim() == 3
            and images.is_contiguous()):
        raise ValueError("images must be a contiguous (n_img, H, W) uint8 CUDA tensor")
    n_img, H, W = images.shape
    n = len(blocks)
    dev = images.device
    sel = torch.empty((n, iters), dtype=torch.int32, device=dev) if want_sel else None
    # complex tables: (real, imaginary) pairs per iteration
    coef = (torch.empty((n, iters * (2 if t.complex else 1)), dtype=torch.float32, device=dev)
            if want_coef else None)
    gld = max([loss_size(b) for b in blocks] + [1])
    g = torch.zeros((n, gld), dtype=torch.float32, device=dev) if want_g else None
    st = t.struct()
    nb = L.se_extrapolate_batch_ws_bytes(C.byref(st), n)
    if ws is None:
        ws = _workspace(nb, dev)
    elif ws.numel() < nb:
        raise ValueError(f"workspace of {ws.numel()} bytes < {nb}")
    arr = blocks_arr if blocks_arr is not None else blocks_array(blocks)
    prm = se_params(float(gamma), int(iters), int(flags))
    return _check_results(getattr(L, name)(C.byref(st), _ptr(images), n_img, H, W, arr, n, prm,
                                           _ptr(sel), _ptr(coef), _ptr(g), gld, _ptr(ws),
                                           ws.numel(), _stream(stream)), (sel, coef, g))


def extrapolate_batch(t: Tables, images: torch.Tensor, blocks: Sequence, gamma: float,
                      iters: int, want_sel=True, want_coef=True, want_g=True, ws=None,
                      stream=None, blocks_arr=None, rows_q14: bool = False,
                      invariant: bool = False):
    """se_extrapolate_batch (Algorithm 3, batched).  ``images`` is modified in
    place (each loss replaced).  Returns (sel, coef, g_loss) device tensors
    (None where not requested).  ``rows_q14``: the loop reads fixed-point
    words (SE_ROWS_Q14: the class rows on the one-launch route, the whole
    rows Gq_rows on the loop over whole rows); ``invariant``: SE_INVARIANT."""
    return _extrapolate("se_extrapolate_batch", t, images, blocks, gamma, iters, want_sel,
                        want_coef, want_g, ws, stream, blocks_arr,
                        (SE_ROWS_Q14 if rows_q14 else 0) | (SE_INVARIANT if invariant else 0))


def extrapolate_batch_static(t: Tables, images: torch.Tensor, blocks: Sequence, gamma: float,
                             iters: int, want_sel=True, want_coef=True, want_g=True,
                             stream=None, blocks_arr=None, rows_q14: bool = False):
    """se_extrapolate_batch_static: se_extrapolate_batch with the library's
    static scratch as workspace (no workspace is allocated; the output
    tensors requested here are).  Results as extrapolate_batch."""
    L = lib()
    if not (images.is_cuda and images.dtype == torch.uint8 and images.dim() == 3
            and images.is_contiguous()):
        raise ValueError("images must be a contiguous (n_img, H, W) uint8 CUDA tensor")
    n_img, H, W = images.shape
    n = len(blocks)
    dev = images.device
    sel = torch.empty((n, iters), dtype=torch.int32, device=dev) if want_sel else None
    coef = (torch.empty((n, iters * (2 if t.complex else 1)), dtype=torch.float32, device=dev)
            if want_coef else None)
    gld = max([loss_size(b) for b in blocks] + [1])
    g = torch.zeros((n, gld), dtype=torch.float32, device=dev) if want_g else None
    st = t.struct()
    arr = blocks_arr if blocks_arr is not None else blocks_array(blocks)
    prm = se_params(float(gamma), int(iters), SE_ROWS_Q14 if rows_q14 else 0)
    return _check_results(L.se_extrapolate_batch_static(C.byref(st), _ptr(images), n_img, H, W,
                                                        arr, n, prm, _ptr(sel), _ptr(coef),
                                                        _ptr(g), gld, _stream(stream)),
                          (sel, coef, g))


def extrapolate_plain(t: Tables, images: torch.Tensor, blocks: Sequence, gamma: float,
                      iters: int, want_sel=True, want_coef=True, want_g=True, ws=None,
                      stream=None, blocks_arr=None, rows_q14: bool = False):
    """se_extrapolate_plain: same results, one block at a time.  ``rows_q14``:
    the loop reads the whole-row words Gq_rows (SE_ROWS_Q14)."""
    return _extrapolate("se_extrapolate_plain", t, images, blocks, gamma, iters, want_sel,
                        want_coef, want_g, ws, stream, blocks_arr,
                        flags=SE_ROWS_Q14 if rows_q14 else 0)


# ---------------------------------------------------------------------------
# stage calls
# ---------------------------------------------------------------------------
class DeviceBlocks:
    """Validated block descriptors resident on the device (se_blocks_upload)."""

    def __init__(self, t: Tables, images: torch.Tensor, blocks: Sequence, stream=None):
        L = lib()
        n_img, H, W = images.shape
        self.n = len(blocks)
        self.buf = torch.empty((max(self.n, 1), BLOCK_INTS), dtype=torch.int32,
                               device=images.device)
        mx = C.c_int32(0)
        st = t.struct()
        code = L.se_blocks_upload(C.byref(st), n_img, H, W, blocks_array(blocks), self.n,
                                  _ptr(self.buf), C.byref(mx), _stream(stream))
        # SE_ENUMERIC: uploaded, with the blocks that have no available sample
        # marked (the loop reports sel = -1 for them)
        self.degenerate = code == SE_ENUMERIC
        if not self.degenerate:
            _check(code)
        self.max_loss = int(mx.value)


def project(t: Tables, images: torch.Tensor, dblocks: DeviceBlocks, R: torch.Tensor,
            ws: torch.Tensor, stream=None):
    """se_project: R[b, k] = D_k R_k^(0) for every block (eq. 12)."""
    L = lib()
    n_img, H, W = images.shape
    st = t.struct()
    _check(L.se_project(C.byref(st), _ptr(images), n_img, H, W, _ptr(dblocks.buf), dblocks.n,
                        _ptr(R), R.shape[1], _ptr(ws), ws.numel(), _stream(stream)))


def project_ws_bytes(t: Tables, n_blk: int) -> int:
    st = t.struct()
    return int(lib().se_project_ws_bytes(C.byref(st), n_blk))


def iterate(t: Tables, R: torch.Tensor, images: torch.Tensor, dblocks: DeviceBlocks,
            gamma: float, iters: int, sel=None, coef=None, g_loss=None, stream=None,
            rows_q14: bool = False):
    """se_iterate: the iteration loop and the paste, from R.  ``rows_q14``:
    the loop reads the whole-row words Gq_rows (SE_ROWS_Q14)."""
    L = lib()
    n_img, H, W = images.shape
    st = t.struct()
    gld = g_loss.shape[1] if g_loss is not None else 0
    prm = se_params(float(gamma), int(iters), SE_ROWS_Q14 if rows_q14 else 0)
    _check(L.se_iterate(C.byref(st), _ptr(R), R.shape[1], _ptr(images), n_img, H, W,
                        _ptr(dblocks.buf), dblocks.n, prm, _ptr(sel), _ptr(coef), _ptr(g_loss),
                        gld, _stream(stream)))


def extrapolate_device_ws_bytes(t: Tables, n_blk: int) -> int:
    st = t.struct()
    return int(lib().se_extrapolate_device_ws_bytes(C.byref(st), n_blk))


def extrapolate_device(t: Tables, images: torch.Tensor, dblocks: DeviceBlocks, gamma: float,
                       iters: int, ws=None, sel=None, coef=None, g_loss=None, stream=None,
                       rows_q14: bool = False):
    """se_extrapolate_device: projections and loop for device descriptors (one
    launch when every atom lies in a transform part; ``ws`` of
    extrapolate_device_ws_bytes bytes otherwise).  ``rows_q14`` as for
    extrapolate_batch."""
    L = lib()
    n_img, H, W = images.shape
    st = t.struct()
    gld = g_loss.shape[1] if g_loss is not None else 0
    _check(L.se_extrapolate_device(C.byref(st), _ptr(images), n_img, H, W, _ptr(dblocks.buf),
                                   dblocks.n,
                                   se_params(float(gamma), int(iters),
                                             SE_ROWS_Q14 if rows_q14 else 0), _ptr(sel),
                                   _ptr(coef), _ptr(g_loss), gld, _ptr(ws),
                                   ws.numel() if ws is not None else 0, _stream(stream)))


def extrapolate_ondemand(phi: torch.Tensor, M: int, N: int, w: torch.Tensor,
                         images: torch.Tensor, blocks: Sequence, gamma: float, iters,
                         want_sel=True, want_coef=True, want_g=True, ws=None, stream=None,
                         parts=(), rows_bf16: bool = False, invariant: bool = False):
    """se_extrapolate_ondemand: per-block weights ``w`` (n_blk, M*N); ``iters``
    an int or a per-block sequence.  ``rows_bf16``: the dense atoms' row
    products from split-BF16 operands (SE_ROWS_BF16X3); ``invariant``:
    SE_INVARIANT.  Returns (sel, coef, g_loss)."""
    L = lib()
    _dev_f32(phi, "phi")
    _dev_f32(w, "w")
    n_img, H, W = images.shape
    n = len(blocks)
    dev = images.device
    per = None
    if isinstance(iters, int):
        imax = iters
    else:
        per = (C.c_int32 * max(n, 1))(*[int(v) for v in iters])
        imax = max([int(v) for v in iters] + [0])
    sel = torch.empty((n, imax), dtype=torch.int32, device=dev) if want_sel else None
    coef = torch.empty((n, imax), dtype=torch.float32, device=dev) if want_coef else None
    gld = max([loss_size(b) for b in blocks] + [1])
    g = torch.zeros((n, gld), dtype=torch.float32, device=dev) if want_g else None
    bas = make_basis(M, N, phi.shape[0], phi.data_ptr(), parts)
    nb = L.se_extrapolate_ondemand_ws_bytes(C.byref(bas), n, gld)
    if ws is None:
        ws = _workspace(nb, dev)
    elif ws.numel() < nb:
        raise ValueError(f"workspace of {ws.numel()} bytes < {nb}")
    prm = se_params(float(gamma), int(imax), (SE_ROWS_BF16X3 if rows_bf16 else 0) |
                    (SE_INVARIANT if invariant else 0))
    return _check_results(L.se_extrapolate_ondemand(C.byref(bas), _ptr(w), _ptr(images), n_img,
                                                    H, W, blocks_array(blocks), n, prm, per,
                                                    _ptr(sel), _ptr(coef), _ptr(g), gld,
                                                    _ptr(ws), ws.numel(), _stream(stream)),
                          (sel, coef, g))


class se_tune_rows_result(C.Structure):
    _fields_ = [("row_tile", C.c_int32), ("row_split", C.c_int32), ("run_ms", C.c_float)]


class OnDemandDict:
    """se_ondemand_prepare: a dictionary prepared once for rows on demand
    (parts verified, phi squared and, with ``rows_bf16``, the split copy kept
    on the device).  ``phi`` is kept referenced while the object lives."""

    def __init__(self, phi: torch.Tensor, M: int, N: int, parts=(), rows_bf16: bool = False,
                 stream=None):
        L = lib()
        _dev_f32(phi, "phi")
        self.phi, self.M, self.N, self.K = phi, M, N, phi.shape[0]
        self.rows_bf16 = rows_bf16
        self._bas = make_basis(M, N, self.K, phi.data_ptr(), parts)
        h = C.c_void_p()
        _check(L.se_ondemand_prepare(C.byref(self._bas), SE_ROWS_BF16X3 if rows_bf16 else 0,
                                     C.byref(h), _stream(stream)))
        self.handle = h

    def extrapolate(self, w: torch.Tensor, images: torch.Tensor, blocks: Sequence, gamma: float,
                    iters, want_sel=True, want_coef=True, want_g=True, stream=None,
                    rows_bf16: bool = False, invariant: bool = False, row_slots: int = 0):
        """se_ondemand_extrapolate: extrapolate_ondemand on this prepared
        dictionary (no synchronisation), caching ``row_slots`` table rows per
        block.  Returns (sel, coef, g_loss)."""
        L = lib()
        _dev_f32(w, "w")
        n_img, H, W = images.shape
        n = len(blocks)
        dev = images.device
        per = None
        if isinstance(iters, int):
            imax = iters
        else:
            per = (C.c_int32 * max(n, 1))(*[int(v) for v in iters])
            imax = max([int(v) for v in iters] + [0])
        sel = torch.empty((n, imax), dtype=torch.int32, device=dev) if want_sel else None
        coef = torch.empty((n, imax), dtype=torch.float32, device=dev) if want_coef else None
        gld = max([loss_size(b) for b in blocks] + [1])
        g = torch.zeros((n, gld), dtype=torch.float32, device=dev) if want_g else None
        ws = _workspace(L.se_ondemand_plan_ws_bytes(self.handle, n, gld, int(row_slots)), dev)
        prm = se_params(float(gamma), int(imax), (SE_ROWS_BF16X3 if rows_bf16 else 0) |
                        (SE_INVARIANT if invariant else 0))
        return _check_results(L.se_ondemand_extrapolate(self.handle, _ptr(w), _ptr(images), n_img,
                                                        H, W, blocks_array(blocks), n, prm, per,
                                                        _ptr(sel), _ptr(coef), _ptr(g), gld,
                                                        int(row_slots), _ptr(ws), ws.numel(),
                                                        _stream(stream)),
                              (sel, coef, g))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().se_ondemand_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class OnDemandPlan:
    """se_ondemand_plan_create: the blocks of one batch ordered, checked and
    uploaded once, with their own workspace (``row_slots`` cached table rows
    per block; None caches every row).  ``run`` launches kernels only and
    may be captured in a graph."""

    def __init__(self, d: OnDemandDict, images: torch.Tensor, blocks: Sequence, gamma: float,
                 iters, row_slots=None, rows_bf16: bool = False, invariant: bool = False,
                 stream=None):
        L = lib()
        self.d = d
        n_img, H, W = images.shape
        n = len(blocks)
        self.n = n
        if isinstance(iters, int):
            per, imax = None, iters
        else:
            per = (C.c_int32 * max(n, 1))(*[int(v) for v in iters])
            imax = max([int(v) for v in iters] + [0])
        self.gld = max([loss_size(b) for b in blocks] + [1])
        slots = imax if row_slots is None else int(row_slots)
        nb = L.se_ondemand_plan_ws_bytes(d.handle, n, self.gld, slots)
        self.ws = _workspace(nb, images.device)
        prm = se_params(float(gamma), int(imax), (SE_ROWS_BF16X3 if rows_bf16 else 0) |
                        (SE_INVARIANT if invariant else 0))
        h = C.c_void_p()
        _check(L.se_ondemand_plan_create(d.handle, n_img, H, W, blocks_array(blocks), n, prm, per,
                                         slots, _ptr(self.ws), self.ws.numel(), _stream(stream),
                                         C.byref(h)))
        self.handle = h
        im, ml, rs = C.c_int32(), C.c_int32(), C.c_int32()
        L.se_ondemand_plan_info(h, C.byref(im), C.byref(ml), C.byref(rs))
        self.iters_max, self.max_loss, self.row_slots = im.value, ml.value, rs.value

    def outputs(self, device, want_sel=True, want_coef=True, want_g=True):
        n, im = self.n, self.iters_max
        sel = torch.empty((n, im), dtype=torch.int32, device=device) if want_sel else None
        coef = torch.empty((n, im), dtype=torch.float32, device=device) if want_coef else None
        g = torch.zeros((n, self.gld), dtype=torch.float32, device=device) if want_g else None
        return sel, coef, g

    def run(self, w: torch.Tensor, images: torch.Tensor, sel=None, coef=None, g=None,
            stream=None):
        """se_ondemand_run into the given outputs (None: not written)."""
        _dev_f32(w, "w")
        return _check_results(lib().se_ondemand_run(self.handle, _ptr(w), _ptr(images), _ptr(sel),
                                                    _ptr(coef), _ptr(g), self.gld,
                                                    _stream(stream)), (sel, coef, g))

    def autotune(self, w: torch.Tensor, images: torch.Tensor, reps: int = 2, stream=None):
        out = se_tune_rows_result()
        _check(lib().se_autotune_ondemand(self.handle, _ptr(w), _ptr(images), int(reps),
                                          _stream(stream), C.byref(out)))
        return out.row_tile, out.row_split, out.run_ms

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().se_ondemand_plan_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
class se_serve_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("frame_H", C.c_int32), ("frame_W", C.c_int32),
                ("max_slots", C.c_int32), ("max_queue", C.c_int32), ("n_streams", C.c_int32),
                ("rho_hat", C.c_float), ("hbm_budget_bytes", C.c_size_t)]


class se_loss(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("y", "x", "h", "w", "basis")]


class se_request(C.Structure):
    _fields_ = [("frame", C.c_void_p), ("H", C.c_int32), ("W", C.c_int32),
                ("losses", C.c_void_p), ("n_losses", C.c_int32), ("prm", se_params)]


class se_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_blocks", C.c_int32), ("n_isolated", C.c_int32),
                ("n_ondemand", C.c_int32), ("t_submit_ns", C.c_uint64),
                ("t_admit_ns", C.c_uint64), ("t_done_ns", C.c_uint64)]


class se_serve_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "completed", "batches", "table_hits",
                                          "table_builds", "table_evictions",
                                          "degraded_blocks")] + \
               [(n, C.c_size_t) for n in ("bytes_tables", "bytes_slots", "bytes_scratch")]


def _serve_lib():
    L = lib()
    if getattr(L, "_serve_ready", False):
        return L
    vp, i32 = C.c_void_p, C.c_int32
    L.se_serve_create.restype = i32
    L.se_serve_create.argtypes = [C.POINTER(se_serve_config), vp, i32, C.POINTER(vp)]
    L.se_serve_submit.restype = i32
    L.se_serve_submit.argtypes = [vp, C.POINTER(se_request), C.POINTER(C.c_uint64)]
    for name in ("se_serve_poll", "se_serve_wait"):
        f = getattr(L, name)
        f.restype = i32
        f.argtypes = [vp, C.c_uint64, C.POINTER(se_result)]
    L.se_serve_stats_get.restype = i32
    L.se_serve_stats_get.argtypes = [vp, C.POINTER(se_serve_stats)]
    L.se_serve_destroy.restype = i32
    L.se_serve_destroy.argtypes = [vp]
    L._serve_ready = True
    return L


SERVE_EXPORTED = ("se_serve_create", "se_serve_submit", "se_serve_poll", "se_serve_wait",
                  "se_serve_stats_get", "se_serve_destroy")
TUNE_EXPORTED = ("se_autotune_batch", "se_tune_export", "se_tune_import", "se_tune_clear",
                 "se_autotune_ondemand")
PLAN_EXPORTED = ("se_ondemand_prepare", "se_ondemand_release", "se_ondemand_plan_ws_bytes",
                 "se_ondemand_plan_create", "se_ondemand_plan_info", "se_ondemand_run",
                 "se_ondemand_plan_release", "se_ondemand_extrapolate")
EXPORTED = EXPORTED + SERVE_EXPORTED + TUNE_EXPORTED + PLAN_EXPORTED


class Server:
    """se_serve_*: a continuous-batching concealment server.  ``bases`` is a
    list of (phi (K, M*N) float32 CUDA tensor, M, N) or (phi, M, N, parts); the
    tensors must stay alive as long as the server."""

    def __init__(self, bases, frame_H: int, frame_W: int, max_slots: int = 8,
                 max_queue: int = 64, n_streams: int = 4, rho_hat: float = 0.8,
                 hbm_budget_bytes: int = 8 << 30, device: int = 0):
        L = _serve_lib()
        self._bases = [b[0] for b in bases]
        arr = (se_basis * len(bases))()
        for i, b in enumerate(bases):
            phi, M, N = b[:3]
            _dev_f32(phi, "phi")
            arr[i] = make_basis(M, N, phi.shape[0], phi.data_ptr(), b[3] if len(b) > 3 else ())
        cfg = se_serve_config(device, frame_H, frame_W, max_slots, max_queue, n_streams,
                              float(rho_hat), int(hbm_budget_bytes))
        h = C.c_void_p()
        _check(L.se_serve_create(C.byref(cfg), arr, len(bases), C.byref(h)))
        self._h = h
        self.frame_H, self.frame_W = frame_H, frame_W

    def submit(self, frame: torch.Tensor, losses, gamma: float, iters: int):
        """Queue a frame (device uint8 H x W, modified in place when done)
        with ``losses`` = [(y, x, h, w, basis), ...].  Returns the ticket, or
        raises SEError (code SE_EBUSY when the queue is full)."""
        L = _serve_lib()
        n = len(losses)
        arr = (se_loss * max(n, 1))()
        for i, l in enumerate(losses):
            arr[i] = se_loss(*[int(v) for v in l])
        req = se_request(frame.data_ptr(), frame.shape[0], frame.shape[1],
                         C.cast(arr, C.c_void_p), n, se_params(float(gamma), int(iters), 0))
        t = C.c_uint64()
        _check(L.se_serve_submit(self._h, C.byref(req), C.byref(t)))
        return int(t.value)

    def poll(self, ticket: int):
        """The se_result once done, else None."""
        res = se_result()
        r = _serve_lib().se_serve_poll(self._h, ticket, C.byref(res))
        if r == SE_EAGAIN:
            return None
        _check(r)
        return res

    def wait(self, ticket: int):
        res = se_result()
        _check(_serve_lib().se_serve_wait(self._h, ticket, C.byref(res)))
        return res

    def stats(self):
        st = se_serve_stats()
        _check(_serve_lib().se_serve_stats_get(self._h, C.byref(st)))
        return {n: getattr(st, n) for n, _ in se_serve_stats._fields_}

    def close(self):
        if self._h:
            _check(_serve_lib().se_serve_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# autotuning
# ---------------------------------------------------------------------------
class se_tune_result(C.Structure):
    _fields_ = [("loop_waves", C.c_int32), ("loop_vpl", C.c_int32), ("proj_tile", C.c_int32),
                ("loop_ms", C.c_float), ("proj_ms", C.c_float)]


def _tune_lib():
    L = lib()
    if getattr(L, "_tune_ready", False):
        return L
    vp, i32 = C.c_void_p, C.c_int32
    L.se_autotune_batch.restype = i32
    L.se_autotune_batch.argtypes = [C.POINTER(se_tables), vp, i32, i32, i32, vp, i32, se_params,
                                    vp, i32, vp, C.c_size_t, i32, vp, C.POINTER(se_tune_result)]
    L.se_tune_export.restype = i32
    L.se_tune_export.argtypes = [C.c_char_p, i32]
    L.se_tune_import.restype = i32
    L.se_tune_import.argtypes = [C.c_char_p]
    L.se_tune_clear.restype = None
    L.se_tune_clear.argtypes = []
    L._tune_ready = True
    return L


def autotune_batch(t: Tables, images: torch.Tensor, dblocks: "DeviceBlocks", R: torch.Tensor,
                   ws: torch.Tensor, gamma: float, iters: int, reps: int = 3, stream=None):
    """se_autotune_batch: returns dict(loop_waves, loop_vpl, proj_tile, loop_ms, proj_ms)."""
    L = _tune_lib()
    n_img, H, W = images.shape
    st = t.struct()
    out = se_tune_result()
    _check(L.se_autotune_batch(C.byref(st), _ptr(images), n_img, H, W, _ptr(dblocks.buf),
                               dblocks.n, se_params(float(gamma), int(iters), 0), _ptr(R),
                               R.shape[1], _ptr(ws), ws.numel(), int(reps), _stream(stream),
                               C.byref(out)))
    return {n: getattr(out, n) for n, _ in se_tune_result._fields_}


def tune_export() -> str:
    L = _tune_lib()
    n = L.se_tune_export(None, 0)
    buf = C.create_string_buffer(n + 1)
    L.se_tune_export(buf, n + 1)
    return buf.value.decode()


def tune_import(text: str) -> None:
    _check(_tune_lib().se_tune_import(text.encode()))


def tune_clear() -> None:
    _tune_lib().se_tune_clear()
