"""Projections and loop in one launch (se_extrapolate_device) for tables whose
atoms all lie in declared transform parts: every output must equal the
two-launch route (se_project + se_iterate) bit for bit, for every loop shape
of the row length, for areas inside the image (16-byte pixel segments) and
across its border (single pixels), and the route must agree with the FP64
oracle.  Tables with dense atoms take the two-launch route inside the call.
(The tables here carry no parity-class tables, with which the one-launch
route streams class rows instead; tests/test_gpu_classes.py covers those.)"""
import numpy as np
import pytest
import torch

from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth

from test_gpu_parity import TOL_FP32, check_against_oracle, dev, say, shared_tables, upload_phi


pytestmark = pytest.mark.gpu


def _bucket(n):
    b = 0
    while (1 << b) < n:
        b += 1
    return b


def _two_stage(t, images, blocks, gamma, iters, gld):
    img = torch.from_numpy(images).to(dev())
    db = B.DeviceBlocks(t, img, blocks)
    n = len(blocks)
    R = torch.empty((n, t.ldG), dtype=torch.float32, device=dev())
    ws = torch.empty(max(1, B.project_ws_bytes(t, n)), dtype=torch.uint8, device=dev())
    sel = torch.full((n, iters), -7, dtype=torch.int32, device=dev())
    coef = torch.zeros((n, iters), dtype=torch.float32, device=dev())
    g = torch.zeros((n, gld), dtype=torch.float32, device=dev())
    B.project(t, img, db, R, ws)
    B.iterate(t, R, img, db, gamma, iters, sel, coef, g)
    torch.cuda.synchronize()
    return [x.cpu() for x in (sel, coef, g, img)]


def _fused(t, images, blocks, gamma, iters, gld):
    img = torch.from_numpy(images).to(dev())
    db = B.DeviceBlocks(t, img, blocks)
    n = len(blocks)
    nb = B.extrapolate_device_ws_bytes(t, n)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev()) if nb else None
    sel = torch.full((n, iters), -7, dtype=torch.int32, device=dev())
    coef = torch.zeros((n, iters), dtype=torch.float32, device=dev())
    g = torch.zeros((n, gld), dtype=torch.float32, device=dev())
    B.extrapolate_device(t, img, db, gamma, iters, ws, sel, coef, g)
    torch.cuda.synchronize()
    return nb, [x.cpu() for x in (sel, coef, g, img)]


def _assert_same(a, b):
    for name, x, y in zip(("sel", "coef", "g_loss", "image"), a, b):
        assert torch.equal(x, y), f"{name} differs between the fused and two-launch routes"


@pytest.mark.parametrize("shape", [(1, 32), (2, 16), (4, 8)])
def test_fused_equals_two_stage_area32(shape):
    d = synth.area32_inputs(8)
    w, v = shape
    say(f"fused vs two launches: 32x32 areas, 128 blocks, K=2048, I=100, shape {w}x{v}")
    phi = upload_phi(synth.round_to_f32(d["phi"]))
    t, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8, parts=d["tx_parts"],
                            classes=False)
    B.tune_clear()
    B.tune_import(f"2048 1024 {_bucket(len(d['blocks']))} {w} {v} 64\n")
    try:
        ref = _two_stage(t, d["images"], d["blocks"], 0.5, 100, 64)
        nb, got = _fused(t, d["images"], d["blocks"], 0.5, 100, 64)
    finally:
        B.tune_clear()
    assert nb == 0
    _assert_same(ref, got)


def test_fused_border_areas_and_oracle():
    """Areas that leave the image (pixels outside read as 0, single-pixel
    loads) next to areas on the 16-byte grid; parity with the oracle."""
    M = N = 32
    H, W = 3 * M + 8, 3 * N + 16
    images = np.stack([synth.synth_image(H, W, seed=40 + s) for s in range(2)])
    blocks = [synth.Block(i, y, x, 12, 12, 8, 8)
              for i in range(2) for (y, x) in ((-12, -12), (0, 16), (40, 48), (H - 20, W - 20))]
    say("fused route: 8 blocks of 32x32 areas, 4 crossing the image border")
    phi_np = synth.round_to_f32(synth.dictionary(M, N, ("dct", "wht")))
    t, _, _ = shared_tables(images, blocks, upload_phi(phi_np), M, N, 0.8,
                            parts=synth.dictionary_parts(M, N, ("dct", "wht")), ref_block=1,
                            classes=False)
    # every block's own weights differ at the border: compare the two
    # routes, which share the tables, bit for bit
    ref = _two_stage(t, images, blocks, 0.5, 100, 64)
    nb, got = _fused(t, images, blocks, 0.5, 100, 64)
    assert nb == 0
    _assert_same(ref, got)
    # the blocks whose weights equal the tables' (inside the image) against
    # the oracle
    inner = [1, 2, 5, 6]
    sel, coef, g, out = (x.numpy() for x in got)
    check_against_oracle(images, [blocks[i] for i in inner], phi_np.astype(np.float64), M, N,
                         0.8, 0.5, 100, sel[inner], coef[inner], g[inner], out,
                         tol=TOL_FP32, tables=t)


@pytest.mark.parametrize("shape", [(4, 32), (8, 16)])
def test_fused_equals_two_stage_area64(shape):
    d = synth.area64_inputs(1)
    blocks = d["blocks"][:96]
    w, v = shape
    say(f"fused vs two launches: 64x64 areas, 96 blocks, K=8192, I=300, shape {w}x{v}")
    phi = upload_phi(synth.round_to_f32(d["phi"]))
    t, _, _ = shared_tables(d["images"], blocks, phi, 64, 64, 0.8, parts=d["tx_parts"],
                            classes=False)
    B.tune_clear()
    B.tune_import(f"8192 4096 {_bucket(len(blocks))} {w} {v} 64\n")
    try:
        ref = _two_stage(t, d["images"], blocks, 0.5, 300, 256)
        nb, got = _fused(t, d["images"], blocks, 0.5, 300, 256)
    finally:
        B.tune_clear()
    assert nb == 0
    _assert_same(ref, got)


def test_dense_tables_take_two_launches():
    d = synth.area32_inputs(2)
    say("extrapolate_device on tables without parts: workspace route")
    phi = upload_phi(synth.round_to_f32(d["phi"]))
    t, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8)
    ref = _two_stage(t, d["images"], d["blocks"], 0.5, 100, 64)
    nb, got = _fused(t, d["images"], d["blocks"], 0.5, 100, 64)
    assert nb > 0
    _assert_same(ref, got)
    # too small a workspace is refused before anything runs
    img = torch.from_numpy(d["images"]).to(dev())
    db = B.DeviceBlocks(t, img, d["blocks"])
    small = torch.empty(16, dtype=torch.uint8, device=dev())
    with pytest.raises(B.SEError) as e:
        B.extrapolate_device(t, img, db, 0.5, 100, small)
    assert e.value.code == B.SE_ENOMEM
