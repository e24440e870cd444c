"""Areas of T consecutive video frames on the GPU (the three-dimensional model
the paper's closing section extends the method to): the weights, the tables
and the loop over T*M*N samples against the FP64 oracle, every route of the
library bit for bit against the others, losses over several frames and areas
that leave the frame."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth

from helpers import describe, oracle_check_video
from test_gpu_parity import TOL_FP32, dev, say, upload_phi

pytestmark = pytest.mark.gpu

TOL_BF16X3 = 1e-2


def _tables(phi32, frames, blocks, T, M, N, ref_block=0, precision=B.SE_FP32, parts=(),
            classes=True, fixed_point=False):
    F, H, W = frames.shape
    lost = torch.from_numpy(synth.video_lost_mask(F, H, W, blocks)).to(dev())
    w = B.area_weights(M, N, 0.8, lost, [blocks[ref_block]], T=T)
    return B.weighted_gram(upload_phi(phi32), w[0].contiguous(), M, N, precision, T=T,
                           parts=parts, classes=classes, fixed_point=fixed_point)


def _batch(t, frames, blocks, iters, plain=False):
    img = torch.from_numpy(frames).to(dev())
    fn = B.extrapolate_plain if plain else B.extrapolate_batch
    sel, coef, g = fn(t, img, blocks, 0.5, iters)
    torch.cuda.synchronize()
    return sel.cpu().numpy(), coef.cpu().numpy(), g.cpu().numpy(), img.cpu().numpy()


def test_volume_weights_match_oracle():
    F, H, W = 6, 40, 44
    T, M, N = 3, 12, 10
    blocks = [synth.Block(0, -4, 3, 5, 4, 4, 3, 1, 1), synth.Block(2, 10, 20, 4, 4, 5, 5, 0, 2),
              synth.Block(3, 12, 24, 2, 2, 4, 4, 2, 1), synth.Block(1, 30, 38, 3, 3, 6, 5, 1, 1)]
    say(f"volume weights: {len(blocks)} areas of {T}x{M}x{N}, across the border and "
        "holding other losses")
    lost = synth.video_lost_mask(F, H, W, blocks)
    w = B.area_weights(M, N, 0.8, torch.from_numpy(lost).to(dev()), blocks, T=T).cpu().numpy()
    assert w.shape == (len(blocks), T * M * N)
    for i, b in enumerate(blocks):
        _, sup = oracle.volume_signal(np.zeros((F, H, W), np.uint8), lost, b.img, b.y0, b.x0,
                                      T, M, N)
        ref = oracle.volume_weights(T, M, N, 0.8, sup)
        np.testing.assert_array_equal(w[i] == 0, ref == 0)
        np.testing.assert_allclose(w[i], ref, rtol=2e-6, atol=0)
    # one frame: the two-dimensional call, bit for bit
    w1 = B.area_weights(M, N, 0.8, torch.from_numpy(lost).to(dev()), blocks, T=1).cpu().numpy()
    w2 = B.area_weights(M, N, 0.8, torch.from_numpy(lost).to(dev()), blocks).cpu().numpy()
    np.testing.assert_array_equal(w1, w2)


def test_video_gram_matches_oracle():
    T, M, N = 4, 16, 16
    say("video tables: 3-D DCT u WHT 4x16x16 (K=2048), one loss box")
    phi = synth.round_to_f32(synth.video_dictionary(T, M, N))
    sup = np.ones((T, M, N), bool)
    sup[2, 4:12, 4:12] = False
    w_ref = oracle.volume_weights(T, M, N, 0.8, sup).astype(np.float32).astype(np.float64)
    t = B.weighted_gram(upload_phi(phi), torch.from_numpy(w_ref.astype(np.float32)).to(dev()),
                        M, N, T=T)
    torch.cuda.synchronize()
    K = phi.shape[0]
    G = t.G.cpu().numpy()[:, :K].astype(np.float64)
    np.testing.assert_array_equal(G, G.T)
    C_ref, D_ref = oracle.table_generation(phi, w_ref)
    np.testing.assert_allclose(t.D.cpu().numpy(), D_ref, rtol=2e-6)
    err = np.abs(G - D_ref[:, None] * C_ref * D_ref[None, :]).max()
    print(f"max |G - G_oracle| = {err:.3g}")
    assert err < 2e-5


def test_video_batch_parity():
    d = synth.video_inputs(1, frames=8)
    T, M, N = d["T"], d["M"], d["N"]
    say(f"video batch: {len(d['blocks'])} areas of {T}x{M}x{N}, K=2048, I=100")
    phi = synth.round_to_f32(d["phi"])
    t = _tables(phi, d["frames"], d["blocks"], T, M, N)
    sel, coef, g, out = _batch(t, d["frames"], d["blocks"], 100)
    st = oracle_check_video(d["frames"], d["blocks"], phi, T, M, N, 0.8, 0.5, 100, sel, g, out,
                            tol=TOL_FP32, coef=coef, tables=t)
    print(describe(st))
    assert st["worst"] <= TOL_FP32
    # frames without losses are untouched
    lost = synth.video_lost_mask(*d["frames"].shape, d["blocks"])
    np.testing.assert_array_equal(out[lost == 0], d["frames"][lost == 0])


def test_video_routes_agree():
    """Batched, two-stage and device-descriptor calls give the same bits;
    the per-block call (its projections a matrix-vector product, summed in
    another order) the same selections and the model within the FP32 bar;
    split-BF16 tables stay within their bar."""
    d = synth.video_inputs(1, frames=8)
    T, M, N = d["T"], d["M"], d["N"]
    blocks = d["blocks"][:48]
    say(f"video routes: {len(blocks)} areas of {T}x{M}x{N}")
    phi = synth.round_to_f32(d["phi"])
    t = _tables(phi, d["frames"], blocks, T, M, N)
    sel0, coef0, g0, out0 = _batch(t, d["frames"], blocks, 60)
    sel1, coef1, g1, out1 = _batch(t, d["frames"], blocks[:6], 60, plain=True)
    np.testing.assert_array_equal(sel1, sel0[:6])
    assert np.abs(g1 - g0[:6]).max() <= TOL_FP32
    n = len(blocks)
    img = torch.from_numpy(d["frames"]).to(dev())
    db = B.DeviceBlocks(t, img, blocks)
    R = torch.empty((n, t.ldR), dtype=torch.float32, device=dev())
    ws = torch.empty(max(1, B.project_ws_bytes(t, n)), dtype=torch.uint8, device=dev())
    sel = torch.zeros((n, 60), dtype=torch.int32, device=dev())
    g = torch.zeros((n, g0.shape[1]), dtype=torch.float32, device=dev())
    B.project(t, img, db, R, ws)
    B.iterate(t, R, img, db, 0.5, 60, sel, None, g)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(sel.cpu().numpy(), sel0)
    np.testing.assert_array_equal(g.cpu().numpy(), g0)
    np.testing.assert_array_equal(img.cpu().numpy(), out0)
    img2 = torch.from_numpy(d["frames"]).to(dev())
    db2 = B.DeviceBlocks(t, img2, blocks)
    nb = B.extrapolate_device_ws_bytes(t, n)
    assert nb > 0
    g2 = torch.zeros_like(g)
    B.extrapolate_device(t, img2, db2, 0.5, 60, torch.empty(nb, dtype=torch.uint8, device=dev()),
                         None, None, g2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g2.cpu().numpy(), g0)
    # split-BF16 tables and projections
    tb = _tables(phi, d["frames"], blocks, T, M, N, precision=B.SE_BF16X3)
    selb, _, gb, outb = _batch(tb, d["frames"], blocks, 60)
    st = oracle_check_video(d["frames"], blocks, phi, T, M, N, 0.8, 0.5, 60, selb, gb, outb,
                            sample=range(0, n, 6), tol=TOL_BF16X3, tables=tb)
    print(f"bf16x3: {describe(st)}")


def test_video_loss_boxes_and_border_areas():
    """Losses over two frames with more samples than the workgroup has lanes,
    losses in the first and last frame of the area, and areas that leave the
    frame (each block concealed with the tables of its own weights)."""
    T, M, N = 2, 8, 8
    F, H, W = 6, 30, 34
    frames = synth.synth_video(F, H, W, seed=77)
    blocks = [synth.Block(0, -3, -2, 1, 0, 6, 8, 0, 2),      # 96 samples, across the corner
              synth.Block(2, 10, 12, 2, 2, 4, 5, 1, 1),     # loss in the last frame
              synth.Block(4, 24, 28, 0, 1, 5, 4, 0, 1),     # across the far border
              synth.Block(3, 14, 2, 3, 3, 2, 2, 0, 2)]
    say(f"video loss boxes: {len(blocks)} areas of {T}x{M}x{N}, K=256, per-block tables")
    phi = synth.round_to_f32(synth.video_dictionary(T, M, N))
    lost = torch.from_numpy(synth.video_lost_mask(F, H, W, blocks)).to(dev())
    w = B.area_weights(M, N, 0.8, lost, blocks, T=T)
    out = frames.copy()
    sels, gs = [], []
    for i, b in enumerate(blocks):
        t = B.weighted_gram(upload_phi(phi), w[i].contiguous(), M, N, T=T)
        img = torch.from_numpy(out).to(dev())
        sel, _, g = B.extrapolate_batch(t, img, [b], 0.5, 40)
        torch.cuda.synchronize()
        out = img.cpu().numpy()
        sels.append(sel.cpu().numpy()[0])
        gs.append(g.cpu().numpy()[0])
    gl = max(len(x) for x in gs)
    g_all = np.stack([np.pad(x, (0, gl - len(x))) for x in gs])
    st = oracle_check_video(frames, blocks, phi, T, M, N, 0.8, 0.5, 40, np.stack(sels), g_all,
                            out, tol=TOL_FP32)
    print(describe(st))
    assert st["worst"] <= TOL_FP32
    # samples outside every loss are untouched
    keep = synth.video_lost_mask(F, H, W, blocks) == 0
    np.testing.assert_array_equal(out[keep], frames[keep])


@pytest.mark.parametrize("precision", [B.SE_FP32, B.SE_BF16X3])
def test_video_transform_parts(precision):
    """3-D DCT and WHT halves declared as transform parts: the projections
    are separable transforms of the stacked frames (vertical matrix the
    Kronecker product of the frame and row transforms) and the table rows
    over the part columns transforms of the weighted atoms.  Both must match
    the dense route, and the loop must match the oracle."""
    d = synth.video_inputs(1, frames=8)
    T, M, N = d["T"], d["M"], d["N"]
    blocks = d["blocks"]
    say(f"video transform parts: {len(blocks)} areas of {T}x{M}x{N}, precision {precision}")
    phi = synth.round_to_f32(d["phi"])
    tp = _tables(phi, d["frames"], blocks, T, M, N, precision=precision, parts=d["tx_parts"])
    td = _tables(phi, d["frames"], blocks, T, M, N, precision=precision)
    torch.cuda.synchronize()
    K = phi.shape[0]
    Gp, Gd = tp.G.cpu().numpy()[:, :K], td.G.cpu().numpy()[:, :K]
    np.testing.assert_array_equal(Gp, Gp.T)
    assert np.abs(Gp - Gd).max() < (2e-5 if precision == B.SE_FP32 else 2e-4)
    n = len(blocks)
    img = torch.from_numpy(d["frames"]).to(dev())
    R = {}
    for name, t in (("parts", tp), ("dense", td)):
        db = B.DeviceBlocks(t, img, blocks)
        R[name] = torch.full((n, t.ldR), float("nan"), dtype=torch.float32, device=dev())
        ws = torch.empty(max(1, B.project_ws_bytes(t, n)), dtype=torch.uint8, device=dev())
        B.project(t, img, db, R[name], ws)
    torch.cuda.synchronize()
    Rp, Rd = R["parts"].cpu().numpy(), R["dense"].cpu().numpy()
    assert np.all(Rp[:, K:] == 0)
    scale = np.abs(Rd[:, :K]).max()
    err = np.abs(Rp[:, :K] - Rd[:, :K]).max()
    print(f"max |R_parts - R_dense| = {err:.3g} (scale {scale:.3g})")
    assert err <= (2e-6 if precision == B.SE_FP32 else 2e-4) * scale
    sel, _, g, out = _batch(tp, d["frames"], blocks, 100)
    tol = TOL_FP32 if precision == B.SE_FP32 else TOL_BF16X3
    sample = None if precision == B.SE_FP32 else range(0, n, 8)
    st = oracle_check_video(d["frames"], blocks, phi, T, M, N, 0.8, 0.5, 100, sel, g, out,
                            sample=sample, tol=tol, tables=tp)
    print(describe(st))
    assert st["worst"] <= tol


def test_video_part_declaration_is_verified():
    """A 3-D part is the transform along every axis: a dictionary of 2-D
    atoms of the 64 x 16 stack (a 64-point DCT down the stacked rows) is not
    it, and declaring it is refused."""
    T, M, N = 4, 16, 16
    wrong = synth.round_to_f32(np.concatenate([synth.dct2_atoms(T * M, N),
                                               synth.wht2_atoms(T * M, N)]))
    w = torch.ones(T * M * N, dtype=torch.float32, device=dev())
    say("video part verification: 64-point DCT rows declared as a 3-D part")
    with pytest.raises(B.SEError) as e:
        B.weighted_gram(upload_phi(wrong), w, M, N, T=T,
                        parts=synth.video_dictionary_parts(T, M, N))
    assert e.value.code == B.SE_EINVAL
    # the Walsh-Hadamard half alone is the same either way (Sylvester order
    # is a Kronecker power), so it is accepted
    B.weighted_gram(upload_phi(wrong), w, M, N, T=T, parts=[("wht", T * M * N)])


def _two_stage_and_one_launch(t, frames, blocks, iters):
    n = len(blocks)
    outs = []
    for one in (False, True):
        img = torch.from_numpy(frames).to(dev())
        db = B.DeviceBlocks(t, img, blocks)
        sel = torch.full((n, iters), -7, dtype=torch.int32, device=dev())
        coef = torch.zeros((n, iters), dtype=torch.float32, device=dev())
        g = torch.zeros((n, 64), dtype=torch.float32, device=dev())
        if one:
            nb = B.extrapolate_device_ws_bytes(t, n)
            assert nb == 0
            B.extrapolate_device(t, img, db, 0.5, iters, None, sel, coef, g)
        else:
            R = torch.empty((n, t.ldR), dtype=torch.float32, device=dev())
            ws = torch.empty(max(1, B.project_ws_bytes(t, n)), dtype=torch.uint8, device=dev())
            B.project(t, img, db, R, ws)
            B.iterate(t, R, img, db, 0.5, iters, sel, coef, g)
        torch.cuda.synchronize()
        outs.append([x.cpu() for x in (sel, coef, g, img)])
    for name, x, y in zip(("sel", "coef", "g_loss", "frames"), *outs):
        assert torch.equal(x, y), f"{name} differs between one launch and two"


def test_video_one_launch_equals_two_stage():
    """Areas of four 16 x 16 frames with transform parts take one launch
    (the frames stacked into a 64 x 16 transform inside each block's
    workgroup): the same bits as the projection launch and the loop launch,
    for areas on the 16-byte grid and across the frame border."""
    d = synth.video_inputs(1, frames=8)
    T, M, N = d["T"], d["M"], d["N"]
    say(f"video one launch vs two: {len(d['blocks'])} areas of {T}x{M}x{N}")
    phi = synth.round_to_f32(d["phi"])
    t = _tables(phi, d["frames"], d["blocks"], T, M, N, parts=d["tx_parts"], classes=False)
    _two_stage_and_one_launch(t, d["frames"], d["blocks"], 100)
    border = [synth.Block(0, -5, -3, 4, 4, 8, 8, 2, 1), synth.Block(4, 120, 118, 4, 4, 8, 8, 2, 1),
              synth.Block(0, 40, 7, 4, 4, 8, 8, 1, 2)]
    _two_stage_and_one_launch(t, d["frames"], border, 60)


def test_video_class_tables():
    """Areas of four frames with a centred loss in one frame: the weights are
    mirror-symmetric in every frame's rows and columns (not in time), so the
    3-D DCT u WHT table is block diagonal in the spatial parities; the class
    route's one launch against the whole-row two launches and the oracle."""
    d = synth.video_inputs(1, frames=8)
    T, M, N = d["T"], d["M"], d["N"]
    say(f"video class tables: {len(d['blocks'])} areas of {T}x{M}x{N}")
    phi = synth.round_to_f32(d["phi"])
    tc = _tables(phi, d["frames"], d["blocks"], T, M, N, parts=d["tx_parts"])
    assert tc.n_classes == 4
    K, Kc = 2048, 512
    cls = tc.cls.cpu().numpy()
    G = tc.G.cpu().numpy()[:, :K]
    Gc = tc.Gc.cpu().numpy()
    order = cls[:, 0]
    assert sorted(order.tolist()) == list(range(K))
    # the class of an atom from its own rows: spatial parities of (k1, k2)
    rows = {"dct": synth.dct_rows(M), "wht": synth.wht_rows(M)}
    def parity(r):
        return 0 if np.allclose(r[::-1], r, atol=1e-12) else 1
    cls_of = np.zeros(K, int)
    for name, first in d["tx_parts"]:
        for k in range(T * M * N):
            k1, k2 = (k // N) % M, k % N
            cls_of[first + k] = 2 * parity(rows[name][k1]) + parity(rows[name][k2])
    for c in range(4):
        blk = order[c * Kc:(c + 1) * Kc]
        assert np.all(cls_of[blk] == c)
        assert np.all(np.diff(blk[:Kc // 2]) > 0) and np.all(np.diff(blk[Kc // 2:]) > 0)
        np.testing.assert_array_equal(Gc[c * Kc:(c + 1) * Kc], G[np.ix_(blk, blk)])
    worst = np.abs(G[cls_of[:, None] != cls_of[None, :]]).max()
    print(f"max |G| between classes = {worst:.3g}")
    assert worst < 1e-6
    sel, _, g, out = _batch(tc, d["frames"], d["blocks"], 100)
    tf = _tables(phi, d["frames"], d["blocks"], T, M, N, parts=d["tx_parts"], classes=False)
    self_, _, gf, _ = _batch(tf, d["frames"], d["blocks"], 100)
    dg = np.abs(g - gf).max()
    print(f"class vs whole rows: identical selections "
          f"{int(np.all(sel == self_, axis=1).sum())}/{len(sel)}, max|dg|={dg:.3g}")
    assert dg <= TOL_FP32
    st = oracle_check_video(d["frames"], d["blocks"], phi, T, M, N, 0.8, 0.5, 100, sel, g, out,
                            tol=TOL_FP32, tables=tc)
    print(f"class route vs oracle: {describe(st)}")
    assert st["worst"] <= TOL_FP32
