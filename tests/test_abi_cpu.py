"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments on the host before touching
a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2204_14194_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "se.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(se_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_what_binding_lists():
    assert _header_symbols() == sorted(B.EXPORTED)


def test_library_exports_every_symbol():
    L = B.lib()
    for name in _header_symbols():
        assert hasattr(L, name), name
    assert B.version() == 100


def test_no_gpu_code_in_python_fallback():
    src = open(os.path.join(ROOT, "paper_2204_14194_amd", "binding.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


def _tables_struct(K=64, M=8, N=8, ldG=None, fake=0x1000):
    ldG = B.table_ld(K) if ldG is None else ldG
    return B.se_tables(M, N, K, ldG, fake, fake, fake, fake, fake, 0, 0, None, None)


def test_rejects_bad_arguments_on_host():
    L = B.lib()
    t = _tables_struct()
    blk = (B.se_block * 1)(B.se_block(0, 0, 0, 6, 6, 4, 4, 0))   # loss leaves the area
    fake = C.c_void_p(0x1000)
    prm = B.se_params(0.5, 10, 0)
    r = L.se_extrapolate_batch(C.byref(t), fake, 1, 32, 32, blk, 1, prm, None, None, None, 0,
                               fake, 1 << 20, None)
    assert r == B.SE_EINVAL
    assert b"loss rectangle" in L.se_last_error()
    # gamma outside (0, 1]
    blk[0] = B.se_block(0, 0, 0, 2, 2, 4, 4, 0)
    r = L.se_extrapolate_batch(C.byref(t), fake, 1, 32, 32, blk, 1, B.se_params(1.5, 10, 0),
                               None, None, None, 0, fake, 1 << 20, None)
    assert r == B.SE_EINVAL
    # ldG below the padded row length
    t2 = _tables_struct(K=63, ldG=64)
    r = L.se_extrapolate_batch(C.byref(t2), fake, 1, 32, 32, blk, 1, prm, None, None, None, 0,
                               fake, 1 << 20, None)
    assert r == B.SE_EINVAL
    # image index out of range
    blk[0] = B.se_block(3, 0, 0, 2, 2, 4, 4, 0)
    r = L.se_extrapolate_batch(C.byref(t), fake, 1, 32, 32, blk, 1, prm, None, None, None, 0,
                               fake, 1 << 20, None)
    assert r == B.SE_EINVAL
    # loss larger than the per-lane capacity of the loop (K <= 2048: 256 px)
    tb = _tables_struct(K=64, M=32, N=32)
    blk[0] = B.se_block(0, 0, 0, 0, 0, 17, 16, 0)
    r = L.se_extrapolate_batch(C.byref(tb), fake, 1, 64, 64, blk, 1, prm, None, None, None, 0,
                               fake, 1 << 20, None)
    assert r == B.SE_EINVAL
    # workspace too small
    blk[0] = B.se_block(0, 0, 0, 2, 2, 4, 4, 0)
    r = L.se_extrapolate_batch(C.byref(t), fake, 1, 32, 32, blk, 1, prm, None, None, None, 0,
                               fake, 16, None)
    assert r == B.SE_ENOMEM
    # weights: rho_hat outside (0, 1]
    r = L.se_area_weights(8, 8, 1.5, fake, 1, 32, 32, blk, 1, fake, fake, 1 << 20, None)
    assert r == B.SE_EINVAL
    # table generation: unknown precision, NULL basis
    bas = B.se_basis(8, 8, 64, 0x1000)
    r = L.se_weighted_gram(C.byref(bas), fake, 7, 0, C.byref(t), fake, 1 << 20, None)
    assert r == B.SE_EINVAL
    bas0 = B.se_basis(8, 8, 64, 0)
    r = L.se_weighted_gram(C.byref(bas0), fake, 0, 0, C.byref(t), fake, 1 << 20, None)
    assert r == B.SE_EINVAL


def test_rejects_bad_transform_parts_on_host():
    """Declared transform parts (Section VI) are validated before any device
    work: known kind, inside the dictionary, disjoint, M, N <= 64, powers of
    two for Walsh-Hadamard."""
    L = B.lib()
    fake = C.c_void_p(0x1000)
    t = _tables_struct(K=2048, M=32, N=32)
    cases = [
        ((9, 0),), ((B.SE_PART_DCT2, -1),), ((B.SE_PART_DCT2, 1025),),
        ((B.SE_PART_DFT2, 0),),            # a DFT part needs a complex dictionary
        ((B.SE_PART_DCT2, 0), (B.SE_PART_WHT2, 1000)),
        ((B.SE_PART_DCT2, 0), (B.SE_PART_WHT2, 1024), (B.SE_PART_DCT2, 0)),
    ]
    for parts in cases:
        bas = B.se_basis(32, 32, 2048, 0x1000, len(parts), B._part_array(parts[:2]))
        r = L.se_weighted_gram(C.byref(bas), fake, 0, 0, C.byref(t), fake, 1 << 20, None)
        assert r == B.SE_EINVAL, parts
    # a complex dictionary declares one DFT part and nothing else
    for parts, what in ((((B.SE_PART_DCT2, 0),), b"DFT parts only"),
                        (((B.SE_PART_DFT2, 0), (B.SE_PART_DFT2, 1024)), b"at most one part"),
                        (((B.SE_PART_DFT2, 1025),), b"outside")):
        bas = B.make_basis(32, 32, 2048, 0x1000, parts, phi_im_ptr=0x2000)
        r = L.se_weighted_gram(C.byref(bas), fake, 0, 0, C.byref(t), fake, 1 << 20, None)
        assert r == B.SE_EINVAL and what in L.se_last_error(), parts
    # Walsh-Hadamard needs power-of-two sides; transforms need sides <= 64
    t48 = _tables_struct(K=4096, M=48, N=48)
    bas = B.make_basis(48, 48, 4096, 0x1000, [(B.SE_PART_WHT2, 0)])
    assert L.se_weighted_gram(C.byref(bas), fake, 0, 0, C.byref(t48), fake, 1 << 20,
                              None) == B.SE_EINVAL
    assert b"power-of-two" in L.se_last_error()
    t80 = _tables_struct(K=6400, M=80, N=80)
    bas = B.make_basis(80, 80, 6400, 0x1000, [(B.SE_PART_DCT2, 0)])
    assert L.se_weighted_gram(C.byref(bas), fake, 0, 0, C.byref(t80), fake, 1 << 20,
                              None) == B.SE_EINVAL
    # hand-built tables with an overlapping declaration are refused by the loop calls
    tb = _tables_struct(K=2048, M=32, N=32)
    tb.n_parts = 2
    tb.parts[0] = B.se_part(B.SE_PART_DCT2, 0)
    tb.parts[1] = B.se_part(B.SE_PART_DCT2, 512)
    tb.tx = 0x1000
    blk = (B.se_block * 1)(B.se_block(0, 0, 0, 2, 2, 4, 4, 0))
    r = L.se_extrapolate_batch(C.byref(tb), fake, 1, 64, 64, blk, 1, B.se_params(0.5, 10, 0),
                               None, None, None, 0, fake, 1 << 30, None)
    assert r == B.SE_EINVAL and b"overlap" in L.se_last_error()
    # declared parts need the operand buffer
    tb.parts[1] = B.se_part(B.SE_PART_WHT2, 1024)
    tb.tx = None
    r = L.se_extrapolate_batch(C.byref(tb), fake, 1, 64, 64, blk, 1, B.se_params(0.5, 10, 0),
                               None, None, None, 0, fake, 1 << 30, None)
    assert r == B.SE_EINVAL and b"tx" in L.se_last_error()
    # its size: fragments of A, B (per transform), D (per transform) and w, 1 KiB per
    # 16 x 16 tile, room for two transforms (a DFT part is a real and an imaginary one),
    # then A, B and D of both transforms once more in class order
    assert L.se_tables_tx_bytes(32, 32, 2) == (2 * 4 + 2 * 4 + 2 * 4 + 4 + 2 * (4 + 4 + 4)) * 1024
    assert L.se_tables_tx_bytes(32, 32, 1) == L.se_tables_tx_bytes(32, 32, 2)
    assert L.se_tables_tx_bytes(7, 5, 1) == (7 + 6) * 1024
    assert L.se_tables_tx_bytes(32, 32, 0) == 0 and L.se_tables_tx_bytes(65, 8, 1) == 0


def test_table_ld_is_padded_row_length():
    assert B.table_ld(2048) == 2048
    assert B.table_ld(2000) == 2048
    assert B.table_ld(4096) == 4096
    assert B.table_ld(8192) == 8192
    assert B.table_ld(4608) == 6144
    assert B.table_ld(1) == 512
    assert B.lib().se_table_ld(0) == 0 and B.lib().se_table_ld(40000) == 0
    for K in (1, 100, 513, 1025, 3000, 12000, 32768):
        ld = B.table_ld(K)
        assert ld >= K and ld % 64 == 0


def test_workspace_sizes_grow_with_work():
    L = B.lib()
    t = _tables_struct(K=2048, M=32, N=32)
    a = L.se_extrapolate_batch_ws_bytes(C.byref(t), 16)
    b = L.se_extrapolate_batch_ws_bytes(C.byref(t), 4096)
    assert 0 < a < b
    assert b >= 4096 * (2048 + 1024) * 4
    tb = _tables_struct(K=2048, M=32, N=32)
    tb.precision = B.SE_BF16X3
    tb.Yhi = tb.Ylo = 0x1000
    assert L.se_project_ws_bytes(C.byref(tb), 64) >= 64 * 1024 * 4
    # BF16X3 tables without their split dictionary are rejected
    tb.Ylo = None
    blk = (B.se_block * 1)(B.se_block(0, 0, 0, 2, 2, 4, 4, 0))
    fake = C.c_void_p(0x1000)
    r = L.se_extrapolate_batch(C.byref(tb), fake, 1, 64, 64, blk, 1, B.se_params(0.5, 10, 0),
                               None, None, None, 0, fake, 1 << 30, None)
    assert r == B.SE_EINVAL


def test_tune_records_roundtrip_and_validation():
    B.tune_clear()
    assert B.tune_export() == ""
    B.tune_import("2048 1024 12 2 16 128\n4096 2304 8 4 16 64\n")
    text = B.tune_export()
    assert "2048 1024 12 2 16 128" in text and "4096 2304 8 4 16 64" in text
    with pytest.raises(B.SEError):
        B.tune_import("2048 1024 12 3 16 128\n")      # 3 x 16 has another row length
    with pytest.raises(B.SEError):
        B.tune_import("2048 1024 12 2 16 96\n")       # unknown tile
    with pytest.raises(B.SEError):
        B.tune_import("garbage")
    B.tune_clear()
    assert B.tune_export() == ""
    # row-product records of rows on demand
    B.tune_import("rows 2304 2304 10 64 4\n2048 1024 12 2 16 128\nrows 576 576 9 12864 2\n")
    text = B.tune_export()
    assert "rows 2304 2304 10 64 4" in text and "2048 1024 12 2 16 128" in text
    assert "rows 576 576 9 12864 2" in text           # 128 atoms x 64 blocks, 2 slices
    for bad in ("rows 2304 2304 10 96 1\n",     # unknown tile
                "rows 2304 2304 10 64 3\n",     # unknown split
                "rows 2304 2304 10 128 2\n",    # the wide tile does not split
                "rows 2304 2304\n"):
        with pytest.raises(B.SEError):
            B.tune_import(bad)
    B.tune_clear()
    assert B.tune_export() == ""


def test_rejects_bad_ondemand_plans_on_host():
    """The prepared-dictionary and plan calls check their arguments before
    any device work: NULL handles, complex or multi-frame dictionaries,
    unknown flags."""
    L = B.lib()
    h = C.c_void_p()
    bas = B.make_basis(24, 24, 1152, 0x1000)
    assert L.se_ondemand_prepare(None, 0, C.byref(h), None) == B.SE_EINVAL
    assert L.se_ondemand_prepare(C.byref(bas), 0, None, None) == B.SE_EINVAL
    assert L.se_ondemand_prepare(C.byref(bas), 4, C.byref(h), None) == B.SE_EINVAL
    assert b"unknown flags" in L.se_last_error()
    cplx = B.make_basis(24, 24, 1152, 0x1000, phi_im_ptr=0x2000)
    assert L.se_ondemand_prepare(C.byref(cplx), 0, C.byref(h), None) == B.SE_EINVAL
    assert b"real dictionaries" in L.se_last_error()
    vol = B.make_basis(16, 16, 2048, 0x1000, T=4)
    assert L.se_ondemand_prepare(C.byref(vol), 0, C.byref(h), None) == B.SE_EINVAL
    assert not h.value
    assert L.se_ondemand_plan_ws_bytes(None, 10, 64, 0) == 0
    blk = (B.se_block * 1)(B.se_block(0, 0, 0, 8, 8, 8, 8, 0))
    prm = B.se_params(0.5, 10, 0)
    p = C.c_void_p()
    assert L.se_ondemand_plan_create(None, 1, 64, 64, blk, 1, prm, None, 0, None, 0, None,
                                     C.byref(p)) == B.SE_EINVAL
    fake = C.c_void_p(0x1000)
    assert L.se_ondemand_run(None, fake, fake, None, None, None, 0, None) == B.SE_EINVAL
    assert L.se_ondemand_plan_info(None, None, None, None) == -1
    assert L.se_autotune_ondemand(None, fake, fake, 1, None, None) == B.SE_EINVAL
    L.se_ondemand_release(None)
    L.se_ondemand_plan_release(None)


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets of
    the C declaration (compiled here with the host compiler)."""
    structs = [B.se_part, B.se_basis, B.se_block, B.se_tables, B.se_params, B.se_serve_config,
               B.se_loss, B.se_request, B.se_result, B.se_serve_stats, B.se_tune_result,
               B.se_tune_rows_result]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "se.h"', "int main(void) {"]
    for S in structs:
        name = S.__name__
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in S._fields_:
            lines.append(f'  printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for S in structs:
        name = S.__name__
        assert got[(name, "size")] == C.sizeof(S), name
        for f in S._fields_:
            assert got[(name, f[0])] == getattr(S, f[0]).offset, (name, f[0])


def test_rejects_bad_video_areas_on_host():
    """Areas of several frames: the area's frames must exist in the batch,
    the loss box must lie in the area's frames, T >= 1 for the weights, no
    transform parts, and the calls limited to two-dimensional areas refuse."""
    L = B.lib()
    fake = C.c_void_p(0x1000)
    prm = B.se_params(0.5, 10, 0)
    t = _tables_struct(K=2048, M=16, N=16)
    t.T = 4
    blk = (B.se_block * 1)(B.se_block(0, 0, 0, 4, 4, 8, 8, 0, 2, 1))

    def batch(n_img, ws_bytes=16):
        # a workspace too small for any batch: descriptors that pass every
        # check end in SE_ENOMEM before anything touches a device
        return L.se_extrapolate_batch(C.byref(t), fake, n_img, 64, 64, blk, 1, prm, None, None,
                                      None, 0, fake, ws_bytes, None)
    assert batch(3) == B.SE_EINVAL and b"frames" in L.se_last_error()   # frames 0..3 of 3
    blk[0] = B.se_block(1, 0, 0, 4, 4, 8, 8, 0, 2, 2)                    # loss frames 2..3
    assert batch(5) == B.SE_ENOMEM
    blk[0] = B.se_block(1, 0, 0, 4, 4, 8, 8, 0, 3, 2)                    # loss frames 3..4
    assert batch(5) == B.SE_EINVAL and b"loss frames" in L.se_last_error()
    blk[0] = B.se_block(1, 0, 0, 4, 4, 8, 8, 0, -1, 1)
    assert batch(5) == B.SE_EINVAL
    blk[0] = B.se_block(1, 0, 0, 0, 0, 16, 16, 0, 0, 2)                  # 512 > 256 samples
    assert batch(5) == B.SE_EINVAL and b"exceeds" in L.se_last_error()
    # a two-dimensional table accepts only lt = 0 and ld <= 1
    t2 = _tables_struct(K=2048, M=16, N=16)
    blk[0] = B.se_block(0, 0, 0, 4, 4, 8, 8, 0, 0, 2)
    assert L.se_extrapolate_batch(C.byref(t2), fake, 4, 64, 64, blk, 1, prm, None, None, None,
                                  0, fake, 16, None) == B.SE_EINVAL
    # weights
    blk[0] = B.se_block(2, 0, 0, 4, 4, 8, 8, 0, 0, 1)
    assert L.se_volume_weights(0, 8, 8, 0.8, fake, 4, 32, 32, blk, 1, fake, fake, 1 << 20,
                               None) == B.SE_EINVAL
    assert L.se_volume_weights(3, 8, 8, 0.8, fake, 4, 32, 32, blk, 1, fake, fake, 1 << 20,
                               None) == B.SE_EINVAL                      # frames 2..4 of 4
    # transform parts of areas of several frames: the stacked frames T M <= 64
    # rows, M a power of two
    t4 = _tables_struct(K=4096, M=16, N=16)
    bas = B.make_basis(16, 16, 4096, 0x1000, [(B.SE_PART_DCT2, 0)], T=8)
    assert L.se_weighted_gram(C.byref(bas), fake, 0, 0, C.byref(t4), fake, 1 << 20,
                              None) == B.SE_EINVAL
    assert b"T M, N <= 64" in L.se_last_error()
    bas = B.make_basis(12, 16, 2048, 0x1000, [(B.SE_PART_DCT2, 0)], T=4)
    assert L.se_weighted_gram(C.byref(bas), fake, 0, 0, C.byref(t4), fake, 1 << 20,
                              None) == B.SE_EINVAL
    assert b"power-of-two M" in L.se_last_error()
    # rows on demand take two-dimensional areas
    bas = B.make_basis(16, 16, 2048, 0x1000, T=4)
    r = L.se_extrapolate_ondemand(C.byref(bas), fake, fake, 8, 64, 64, blk, 1, prm, None,
                                  None, None, None, 0, fake, 16, None)
    assert r == B.SE_EINVAL and b"two-dimensional" in L.se_last_error()
    # the server takes two-dimensional areas (refused before any device call)
    SL = B._serve_lib()
    cfg = B.se_serve_config(0, 64, 64, 1, 1, 1, 0.8, 1 << 30)
    sets = (B.se_basis * 1)(B.make_basis(16, 16, 2048, 0x1000, T=4))
    out = C.c_void_p()
    assert SL.se_serve_create(C.byref(cfg), sets, 1, C.byref(out)) == B.SE_EINVAL
    assert b"two-dimensional" in L.se_last_error()


def test_rejects_fixed_point_rows_on_host():
    """SE_ROWS_Q14 is taken by the one-launch calls on class tables with
    fixed-point class rows and by the loop over whole rows on tables with
    whole-row words, SE_ROWS_BF16X3 only by rows on demand; unknown flags,
    the other cases and misaligned words are refused before any device
    work."""
    L = B.lib()
    fake = C.c_void_p(0x1000)
    t = _tables_struct(K=2048, M=32, N=32)          # no parts, no class tables
    blk = (B.se_block * 1)(B.se_block(0, 0, 0, 12, 12, 8, 8, 0))
    q14 = B.se_params(0.5, 10, B.SE_ROWS_Q14)

    def call(name, prm):
        return getattr(L, name)(C.byref(t), fake, 1, 64, 64, blk, 1, prm, None, None, None, 0,
                                fake, 16, None)
    assert call("se_extrapolate_batch", B.se_params(0.5, 10, 0)) == B.SE_ENOMEM
    assert call("se_extrapolate_batch", B.se_params(0.5, 10, 8)) == B.SE_EINVAL
    assert b"unknown flags" in L.se_last_error()
    # SE_INVARIANT is accepted by every call (here it reaches the workspace check)
    assert call("se_extrapolate_batch", B.se_params(0.5, 10, B.SE_INVARIANT)) == B.SE_ENOMEM
    for name in ("se_extrapolate_batch", "se_extrapolate_plain"):
        assert call(name, q14) == B.SE_EINVAL and b"SE_ROWS_Q14" in L.se_last_error()
    r = L.se_iterate(C.byref(t), fake, t.ldG, fake, 1, 64, 64, fake, 1, q14, None, None, None,
                     0, None)
    assert r == B.SE_EINVAL and b"SE_ROWS_Q14" in L.se_last_error()
    bas = B.make_basis(32, 32, 2048, 0x1000)
    r = L.se_extrapolate_ondemand(C.byref(bas), fake, fake, 1, 64, 64, blk, 1, q14, None,
                                  None, None, None, 0, fake, 16, None)
    assert r == B.SE_EINVAL and b"no fixed-point rows" in L.se_last_error()
    # split-BF16 rows belong to rows on demand
    bf = B.se_params(0.5, 10, B.SE_ROWS_BF16X3)
    assert call("se_extrapolate_batch", bf) == B.SE_EINVAL
    assert b"rows on demand" in L.se_last_error()
    r = L.se_extrapolate_ondemand(C.byref(bas), fake, fake, 1, 64, 64, blk, 1, bf, None,
                                  None, None, None, 0, fake, 16, None)
    assert r == B.SE_ENOMEM
    t.Gq = 0x1002
    assert L.se_weighted_gram(C.byref(bas), fake, 0, 0, C.byref(t), fake, 1 << 20,
                              None) == B.SE_EINVAL
    assert b"Gq" in L.se_last_error()
    t.Gq = None
    t.Gq_rows = 0x1002
    assert L.se_weighted_gram(C.byref(bas), fake, 0, 0, C.byref(t), fake, 1 << 20,
                              None) == B.SE_EINVAL
    assert b"Gq_rows" in L.se_last_error()
    # whole-row words: the loop over whole rows (these tables have no
    # one-launch form) takes SE_ROWS_Q14 and reaches the workspace check
    t.Gq_rows = 0x2000
    for name in ("se_extrapolate_batch", "se_extrapolate_plain"):
        assert call(name, q14) == B.SE_ENOMEM, name


def test_rejects_overlapping_losses_on_host():
    """Each block writes its loss in place: losses sharing a pixel are
    refused; adjacent losses, losses in different images and losses that
    meet only outside the image are accepted (checked up to the workspace
    test, SE_ENOMEM, before any device work)."""
    L = B.lib()
    fake = C.c_void_p(0x1000)
    prm = B.se_params(0.5, 10, 0)
    t = _tables_struct(K=2048, M=32, N=32)

    def batch(pairs, n_img=2, H=100, W=100):
        blk = (B.se_block * len(pairs))(*[B.se_block(*p) for p in pairs])
        return L.se_extrapolate_batch(C.byref(t), fake, n_img, H, W, blk, len(pairs), prm, None,
                                      None, None, 0, fake, 16, None)
    # (img, y0, x0, ly, lx, lh, lw)
    a = (0, 10, 10, 12, 12, 8, 8)                     # loss rows 22..29, cols 22..29
    assert batch([a, (0, 10, 17, 12, 12, 8, 8)]) == B.SE_EINVAL   # shares column 29
    assert b"overlap" in L.se_last_error()
    assert batch([a, (0, 10, 18, 12, 12, 8, 8)]) == B.SE_ENOMEM   # adjacent
    assert batch([a, (1, 10, 10, 12, 12, 8, 8)]) == B.SE_ENOMEM   # another image
    # losses that meet only above the image (rows < 0) write nothing there
    assert batch([(0, -20, 0, 12, 12, 8, 8), (0, -20, 4, 12, 12, 8, 8)]) == B.SE_ENOMEM
    assert batch([(0, -16, 0, 12, 12, 8, 8), (0, -16, 4, 12, 12, 8, 8)]) == B.SE_EINVAL
    # many disjoint losses across cell borders, one duplicate at the end
    grid = [(0, y, x, 12, 12, 8, 8) for y in range(-12, 80, 8) for x in range(-12, 80, 8)]
    assert batch(grid) == B.SE_ENOMEM
    assert batch(grid + [grid[57]]) == B.SE_EINVAL
    # rows on demand check the same
    bas = B.make_basis(32, 32, 2048, 0x1000)
    blk = (B.se_block * 2)(B.se_block(*a), B.se_block(0, 10, 17, 12, 12, 8, 8))
    r = L.se_extrapolate_ondemand(C.byref(bas), fake, fake, 2, 100, 100, blk, 2, prm, None,
                                  None, None, None, 0, fake, 16, None)
    assert r == B.SE_EINVAL and b"overlap" in L.se_last_error()


def test_blocks_without_support_are_reported_on_host():
    """Blocks whose area holds no available sample (eq. 17 undefined for every
    atom): an area wholly outside the image, and a loss covering every
    in-image sample of its area.  The host finds them before any launch; with
    every block such and no output requested there is nothing to compute and
    the call returns SE_ENUMERIC without touching a device."""
    L = B.lib()
    t = _tables_struct(K=64, M=8, N=8)
    fake = C.c_void_p(0x1000)
    prm = B.se_params(0.5, 10, 0)
    blk = (B.se_block * 3)(B.se_block(0, 40, 0, 2, 2, 4, 4, 0),    # area below the image
                           B.se_block(0, -8, -8, 2, 2, 4, 4, 0),   # above and left of it
                           B.se_block(0, -4, -4, 4, 4, 4, 4, 0))   # loss = the in-image quarter
    r = L.se_extrapolate_batch(C.byref(t), fake, 1, 32, 32, blk, 3, prm, None, None, None, 0,
                               fake, 1 << 20, None)
    assert r == B.SE_ENUMERIC
    assert b"3 block(s) have no available sample" in L.se_last_error()
    r = L.se_extrapolate_batch_static(C.byref(t), fake, 1, 32, 32, blk, 3, prm, None, None,
                                      None, 0, None)
    assert r == B.SE_ENUMERIC
    # one sample of the last area left outside its loss: not such a block
    # (the call would then launch, which needs a device: only the message of
    # the first two is checked through a call with two blocks)
    r = L.se_extrapolate_batch(C.byref(t), fake, 1, 32, 32, blk, 2, prm, None, None, None, 0,
                               fake, 1 << 20, None)
    assert r == B.SE_ENUMERIC
    assert b"2 block(s)" in L.se_last_error()
