"""Blocks with nothing to extrapolate from (eq. 17 undefined for every atom:
no available sample in the area, or every atom of zero weighted norm).
Such a block reports sel = -1 in every iteration, zero coefficients and a
zero model, and keeps its loss; the call finishes every other block.  The
host finds the blocks without an available sample by their geometry (the
call then ends with SE_ENUMERIC); the device finds the rest (every D_k = 0),
which asynchronous calls report through sel only and the server through the
request's status."""
import numpy as np
import pytest
import torch

from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth

from test_gpu_parity import dev, say, shared_tables, upload_phi

pytestmark = pytest.mark.gpu


def _run(fn, t, images, blocks, iters):
    img = torch.from_numpy(images).to(dev())
    try:
        sel, coef, g = fn(t, img, blocks, 0.5, iters)
        code = B.SE_OK
    except B.SENumericError as e:
        (sel, coef, g), code = e.results, e.code
    torch.cuda.synchronize()
    return code, sel.cpu().numpy(), coef.cpu().numpy(), g.cpu().numpy(), img.cpu().numpy()


def _assert_degenerate(sel, coef, g, out, images, b, n):
    assert (sel[n] == -1).all() and (coef[n] == 0).all() and (g[n] == 0).all()
    np.testing.assert_array_equal(out, images)          # the loss (and all else) untouched


@pytest.mark.parametrize("route", ["one_launch", "two_launch", "plain", "static"])
def test_block_without_available_sample(route):
    """A block whose loss covers every in-image sample of its area, added to
    the 16 blocks of a 128 x 128 image: SE_ENUMERIC, the 16 blocks exactly as
    without it, the extra block sel = -1 with its loss kept."""
    say(f"block without an available sample: 32x32 areas, 16 + 1 blocks, {route} route")
    d = synth.area32_inputs(1)
    phi = synth.round_to_f32(d["phi"])
    t, _, _ = shared_tables(d["images"], d["blocks"], upload_phi(phi), 32, 32, 0.8,
                            parts=d["tx_parts"] if route == "one_launch" else ())
    fn = {"one_launch": B.extrapolate_batch, "two_launch": B.extrapolate_batch,
          "plain": B.extrapolate_plain, "static": B.extrapolate_batch_static}[route]
    extra = synth.Block(0, -24, -24, 24, 24, 8, 8)       # loss = image rows/columns 0..7
    code0, sel0, coef0, g0, out0 = _run(fn, t, d["images"], d["blocks"], 100)
    code, sel, coef, g, out = _run(fn, t, d["images"], d["blocks"] + [extra], 100)
    assert code0 == B.SE_OK and code == B.SE_ENUMERIC
    np.testing.assert_array_equal(sel[:16], sel0)
    np.testing.assert_array_equal(coef[:16], coef0)
    np.testing.assert_array_equal(g[:16], g0)
    assert (sel[16] == -1).all() and (coef[16] == 0).all() and (g[16] == 0).all()
    np.testing.assert_array_equal(out, out0)             # rows/columns 0..7 kept
    assert (sel0 >= 0).all()


@pytest.mark.parametrize("parts", [False, True])
def test_tables_of_an_empty_support(parts):
    """Tables built from an all-zero weight pattern have D = 0 for every atom:
    every block using them is found on the device (the call returns SE_OK)."""
    say(f"tables of an all-zero weight pattern, parts {parts}")
    d = synth.area32_inputs(1)
    phi = synth.round_to_f32(d["phi"])
    w = torch.zeros(1024, dtype=torch.float32, device=dev())
    t = B.weighted_gram(upload_phi(phi), w, 32, 32, parts=d["tx_parts"] if parts else ())
    torch.cuda.synchronize()
    assert (t.D.cpu().numpy() == 0).all()
    code, sel, coef, g, out = _run(B.extrapolate_batch, t, d["images"], d["blocks"], 20)
    assert code == B.SE_OK
    assert (sel == -1).all() and (coef == 0).all() and (g == 0).all()
    np.testing.assert_array_equal(out, d["images"])


def _cluster():
    """A 3 x 3 cluster of 8 x 8 losses covering [16, 40)^2 of a 64 x 64 image:
    the 24 x 24 area of the centre loss (rows and columns 24 .. 31) is
    covered by the nine losses."""
    img = synth.synth_image(64, 64, seed=4)[None]
    blocks = [synth.Block(0, 16 + 8 * i - 8, 16 + 8 * j - 8, 8, 8, 8, 8)
              for i in range(3) for j in range(3)]
    return img, blocks


def test_ondemand_block_whose_area_is_lost():
    say("rows on demand: the centre of a 3x3 cluster of losses has no available sample")
    img, blocks = _cluster()
    phi = synth.round_to_f32(synth.dictionary(24, 24, ("dct", "gauss"), seed=7, n_gauss=576))
    lost = torch.from_numpy(synth.lost_mask(64, 64, blocks)[None]).to(dev())
    w = B.area_weights(24, 24, 0.8, lost, blocks)
    assert (w[4] == 0).all() and (w.sum(dim=1)[[0, 1, 2, 3, 5, 6, 7, 8]] > 0).all()
    img_d = torch.from_numpy(img).to(dev())
    sel, coef, g = B.extrapolate_ondemand(upload_phi(phi), 24, 24, w, img_d, blocks, 0.5, 30)
    torch.cuda.synchronize()
    sel, coef, g, out = (x.cpu().numpy() for x in (sel, coef, g, img_d))
    assert (sel[4] == -1).all() and (coef[4] == 0).all() and (g[4] == 0).all()
    np.testing.assert_array_equal(out[0, 24:32, 24:32], img[0, 24:32, 24:32])
    for i in (0, 1, 2, 3, 5, 6, 7, 8):
        assert (sel[i] >= 0).all()
        b = blocks[i]
        y, x = b.y0 + b.ly, b.x0 + b.lx
        np.testing.assert_array_equal(out[0, y:y + 8, x:x + 8],
                                      np.clip(np.rint(g[i, :64]), 0, 255).reshape(8, 8))


def test_served_request_with_such_a_block():
    say("server: a request whose 5x5 cluster of losses leaves one block without samples")
    phi = synth.round_to_f32(synth.dictionary(32, 32, ("dct", "wht"))).astype(np.float32)
    srv = B.Server([(torch.from_numpy(phi).cuda(), 32, 32, ())], 64, 64, max_slots=1,
                   max_queue=2, n_streams=1)
    img = synth.synth_image(64, 64, seed=4)
    # 8x8 losses covering the square [8, 48)^2: the 32x32 area of the loss at
    # (24, 24), rows and columns 12 .. 43, lies inside it
    losses = [(y, x, 8, 8, 0) for y in range(8, 48, 8) for x in range(8, 48, 8)]
    fr = torch.from_numpy(img.copy()).cuda()
    res = srv.wait(srv.submit(fr, losses, 0.5, 20))
    assert res.status == B.SE_ENUMERIC and res.n_blocks == 25
    out = fr.cpu().numpy()
    np.testing.assert_array_equal(out[24:32, 24:32], img[24:32, 24:32])
    assert not np.array_equal(out[32:40, 32:40], img[32:40, 32:40])
    # a request without such a block on the same server
    fr2 = torch.from_numpy(img.copy()).cuda()
    assert srv.wait(srv.submit(fr2, losses[:3], 0.5, 20)).status == B.SE_OK
    srv.close()
