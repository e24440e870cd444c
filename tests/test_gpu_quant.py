"""Fixed-point rows (Section III: the loop of Algorithm 3 has no division,
so its tables suit fixed-point words; the bit depth is open).  Class rows:
the device's 16-bit words against the oracle's quantisation of its own FP64
table, the fixed-point route against the oracle run on those words, the
exactness of the word arithmetic (the fixed-point route equals the FP32
route on the dequantised rows bit for bit, eager and replayed from a graph),
both loop shapes, areas of four frames and 64 x 64 areas.  Whole rows (the
loop over whole rows, tables without parts): the same three checks."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth

from helpers import describe, oracle_check, oracle_check_video
from test_gpu_classes import expected_class_order, _bucket
from test_gpu_parity import dev, say, shared_tables, upload_phi
from test_gpu_video import _tables as video_tables

pytestmark = pytest.mark.gpu

# The device's words are those of its FP32 table (FP32 weights, FP32 products),
# so a word whose exact value lies within that table's rounding of a half
# step can differ from the oracle's by one (about 1 in 10^4 words).  One such
# word shifts R~_k by gamma |R~_u| 2^-14 (3e-2 at |R~_u| ~ 10^3) each time u
# is selected, which reaches the model, when k is selected later, at ~1e-3
# per event: the fixed-point route is held to 1e-2 (the FP32 route's 1e-3
# holds where no word differs: the exact-arithmetic test below).
TOL_Q14 = 1e-2


def _run(t, images, blocks, iters, q14, n=None):
    img = torch.from_numpy(images).to(dev())
    bl = blocks if n is None else blocks[:n]
    sel, coef, g = B.extrapolate_batch(t, img, bl, 0.5, iters, rows_q14=q14)
    torch.cuda.synchronize()
    return [x.cpu() for x in (sel, coef, g, img)]


def _dequantised_twin(t):
    """The same tables with Gc replaced by the words times 2^-14 (FP32,
    exact): the FP32 class route on them must equal the fixed-point route."""
    twin = B.Tables(t.M, t.N, t.K, t.ldG, t.G, t.D, t.Y, t.sqrtw, t.phi, t.info, t.precision,
                    Yhi=t.Yhi, Ylo=t.Ylo, parts=t.parts, tx=t.tx, T=t.T,
                    Gc=t.Gq.float() * 2.0 ** -14, cls=t.cls, n_classes=t.n_classes)
    return twin


def test_fixed_point_words_match_oracle():
    d = synth.area32_inputs(2)
    say("fixed-point words: 32x32 areas, centred 8x8 loss, K=2048")
    phi32 = synth.round_to_f32(d["phi"])
    t, w, lost = shared_tables(d["images"], d["blocks"], upload_phi(phi32), 32, 32, 0.8,
                               parts=d["tx_parts"], fixed_point=True)
    torch.cuda.synchronize()
    assert t.n_classes == 4 and t.Gq is not None and t.Gq.dtype == torch.int16
    b = d["blocks"][0]
    _, sup = oracle.area_signal(d["images"][b.img], lost[b.img], b.y0, b.x0, 32, 32)
    C, D = oracle.table_generation(phi32, oracle.area_weights(32, 32, 0.8, sup))
    G = oracle.unit_table(C, D)
    q_ref = oracle.quantise_table(G).astype(np.int32)
    order, _ = expected_class_order(32, 32, d["tx_parts"])
    Gq = t.Gq.cpu().numpy().astype(np.int32)
    Kc = 512
    worst, near_only = 0, True
    for c in range(4):
        blk = order[c * Kc:(c + 1) * Kc]
        ref = q_ref[np.ix_(blk, blk)]
        diff = np.abs(Gq[c * Kc:(c + 1) * Kc] - ref)
        worst = max(worst, int(diff.max()))
        # a word may differ by one only where the FP64 entry lies within the
        # FP32 table's rounding of a half-step boundary
        x = G[np.ix_(blk, blk)] * 2.0 ** 14
        near_only &= bool((np.abs(np.abs(x - np.floor(x)) - 0.5)[diff > 0] < 1e-2).all())
    n_diff = sum(int((Gq[c * Kc:(c + 1) * Kc] != q_ref[np.ix_(order[c * Kc:(c + 1) * Kc],
                                                             order[c * Kc:(c + 1) * Kc])]).sum())
                 for c in range(4))
    print(f"words differing from the oracle's: {n_diff} of {2048 * 512} (by at most {worst})")
    assert worst <= 1 and near_only
    diag = Gq[np.arange(2048), np.arange(2048) % Kc]
    assert (diag == 16384).all()


def test_fixed_point_route_matches_oracle():
    d = synth.area32_inputs(8)
    say("fixed-point route: 128 blocks, K=2048, I=100, against the oracle on its words")
    phi32 = synth.round_to_f32(d["phi"])
    t, _, _ = shared_tables(d["images"], d["blocks"], upload_phi(phi32), 32, 32, 0.8,
                            parts=d["tx_parts"], fixed_point=True)
    sel, coef, g, img = [x.numpy() for x in _run(t, d["images"], d["blocks"], 100, True)]
    st = oracle_check(d["images"], d["blocks"], phi32, 32, 32, 0.8, 0.5, 100, sel, g, img,
                      tol=TOL_Q14, q14=True, coef=coef, tables=t)
    print(f"fixed-point route vs oracle on words: {describe(st)}")
    assert st["worst"] <= TOL_Q14
    # context: how far the words move the model from the FP32 rows
    _, _, gf, _ = [x.numpy() for x in _run(t, d["images"], d["blocks"], 100, False)]
    print(f"fixed-point vs FP32 rows: max|dg|={np.abs(g - gf).max():.3g}, "
          f"median {np.median(np.abs(g - gf)):.3g}")


def test_fixed_point_route_is_exact_word_arithmetic():
    """R~ -= (tc 2^-14) q rounds as R~ -= tc (q 2^-14): the fixed-point route
    equals the FP32 class route on the dequantised rows bit for bit, through
    se_extrapolate_batch, se_extrapolate_device and graph replays."""
    d = synth.area32_inputs(8)
    say("fixed-point route == FP32 route on dequantised rows (batch, device call, graph)")
    t, _, _ = shared_tables(d["images"], d["blocks"], upload_phi(synth.round_to_f32(d["phi"])),
                            32, 32, 0.8, parts=d["tx_parts"], fixed_point=True)
    q = _run(t, d["images"], d["blocks"], 100, True)
    f = _run(_dequantised_twin(t), d["images"], d["blocks"], 100, False)
    for name, x, y in zip(("sel", "coef", "g_loss", "image"), q, f):
        assert torch.equal(x, y), f"{name} differs"
    n = len(d["blocks"])
    img0 = torch.from_numpy(d["images"]).to(dev())
    img = img0.clone()
    db = B.DeviceBlocks(t, img, d["blocks"])
    sel = torch.zeros((n, 100), dtype=torch.int32, device=dev())
    coef = torch.zeros((n, 100), dtype=torch.float32, device=dev())
    g = torch.zeros((n, q[2].shape[1]), dtype=torch.float32, device=dev())

    def step(stream=None):
        B.extrapolate_device(t, img, db, 0.5, 100, None, sel, coef, g, stream=stream,
                             rows_q14=True)
    step()
    torch.cuda.synchronize()
    for x, y in zip((sel, coef, g, img), q):
        assert torch.equal(x.cpu(), y)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=side):
        step(side)
    torch.cuda.synchronize()
    for rep in range(3):
        for x in (sel, coef, g):
            x.zero_()
        img.copy_(img0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for x, y in zip((sel, coef, g, img), q):
            assert torch.equal(x.cpu(), y), f"replay {rep}"


def test_fixed_point_loop_shapes_agree():
    d = synth.area32_inputs(8)
    say("fixed-point route: loop shapes 1x32 and 2x16")
    t, _, _ = shared_tables(d["images"], d["blocks"], upload_phi(synth.round_to_f32(d["phi"])),
                            32, 32, 0.8, parts=d["tx_parts"], fixed_point=True)
    got = []
    for w, v in ((1, 32), (2, 16)):
        B.tune_clear()
        B.tune_import(f"2048 1024 {_bucket(len(d['blocks']))} {w} {v} 64\n")
        try:
            got.append(_run(t, d["images"], d["blocks"], 100, True))
        finally:
            B.tune_clear()
    for name, x, y in zip(("sel", "coef", "g_loss", "image"), *got):
        assert torch.equal(x, y), f"{name} differs between the loop shapes"


def test_fixed_point_video_areas():
    d = synth.video_inputs(1)
    T, M, N = 4, 16, 16
    say("fixed-point route: areas of 4 frames x 16x16, K=2048, I=100")
    phi = synth.round_to_f32(d["phi"])
    t = video_tables(phi, d["frames"], d["blocks"], T, M, N, parts=d["tx_parts"],
                     fixed_point=True)
    assert t.n_classes == 4 and t.Gq is not None
    q = _run(t, d["frames"], d["blocks"], 100, True)
    f = _run(_dequantised_twin(t), d["frames"], d["blocks"], 100, False)
    for name, x, y in zip(("sel", "coef", "g_loss", "image"), q, f):
        assert torch.equal(x, y), f"{name} differs"
    sel, _, g, out = [x.numpy() for x in q]
    sample = np.random.default_rng(1).choice(len(d["blocks"]), 24, replace=False)
    st = oracle_check_video(d["frames"], d["blocks"], phi, T, M, N, 0.8, 0.5, 100, sel, g, out,
                            sample=sample, tol=TOL_Q14, q14=True, tables=t)
    print(f"video fixed-point route vs oracle on words: {describe(st)}")
    assert st["worst"] <= TOL_Q14


def test_fixed_point_area64():
    """64 x 64 areas (K = 8192, four waves per block): the fixed-point route
    equals the FP32 route on the dequantised rows, on 64 blocks."""
    d = synth.area64_inputs(1)
    say("fixed-point route: 64x64 areas, K=8192, I=300, 64 blocks")
    t, _, _ = shared_tables(d["images"], d["blocks"], upload_phi(synth.round_to_f32(d["phi"])),
                            64, 64, 0.8, parts=d["tx_parts"], fixed_point=True)
    assert t.n_classes == 4
    q = _run(t, d["images"], d["blocks"], 300, True, n=64)
    f = _run(_dequantised_twin(t), d["images"], d["blocks"], 300, False, n=64)
    for name, x, y in zip(("sel", "coef", "g_loss", "image"), q, f):
        assert torch.equal(x, y), f"{name} differs"


def test_fixed_point_edge_cases():
    """An empty batch, zero iterations (the model is 0 and is pasted), and
    areas across the image border next to areas on the 16-byte grid: the
    fixed-point route equals the FP32 route on the dequantised rows bit for
    bit; tables without fixed-point words refuse the flag."""
    M = N = 32
    H, W = 3 * M + 8, 3 * N + 16
    images = np.stack([synth.synth_image(H, W, seed=40 + s) for s in range(2)])
    blocks = [synth.Block(i, y, x, 12, 12, 8, 8)
              for i in range(2) for (y, x) in ((-12, -12), (0, 16), (40, 48), (H - 20, W - 20))]
    say("fixed-point route: empty batch, I=0, 8 areas of which 4 cross the border")
    phi = upload_phi(synth.round_to_f32(synth.dictionary(M, N, ("dct", "wht"))))
    parts = synth.dictionary_parts(M, N, ("dct", "wht"))
    t, _, _ = shared_tables(images, blocks, phi, M, N, 0.8, parts=parts, ref_block=1,
                            fixed_point=True)
    assert t.n_classes == 4
    twin = _dequantised_twin(t)
    img = torch.from_numpy(images).to(dev())
    sel, coef, g = B.extrapolate_batch(t, img, [], 0.5, 100, rows_q14=True)
    torch.cuda.synchronize()
    assert sel.numel() == 0 and torch.equal(img.cpu(), torch.from_numpy(images))
    for iters in (0, 100):
        q = _run(t, images, blocks, iters, True)
        f = _run(twin, images, blocks, iters, False)
        for name, x, y in zip(("sel", "coef", "g_loss", "image"), q, f):
            assert torch.equal(x, y), f"{name} differs at I={iters}"
        if iters == 0:
            assert (q[2] == 0).all()
    # class tables without words: the flag is refused
    t2, _, _ = shared_tables(images, blocks, phi, M, N, 0.8, parts=parts, ref_block=1)
    assert t2.n_classes == 4 and t2.Gq is None
    with pytest.raises(RuntimeError, match="SE_ROWS_Q14"):
        B.extrapolate_batch(t2, torch.from_numpy(images).to(dev()), blocks, 0.5, 10,
                            rows_q14=True)


# ---------------------------------------------------------------------------
# whole-row words: the loop over whole rows (tables without the one-launch form)
# ---------------------------------------------------------------------------
def _dense_tables(d, M, n_img_blocks=None):
    phi32 = synth.round_to_f32(d["phi"])
    t, w, lost = shared_tables(d["images"], d["blocks"], upload_phi(phi32), M, M, 0.8,
                               fixed_point_rows=True)
    torch.cuda.synchronize()
    assert t.n_classes == 0 and t.Gq_rows is not None and t.Gq_rows.dtype == torch.int16
    return phi32, t, lost


def _row_twin(t):
    """The same tables with G replaced by the whole-row words times 2^-14
    (FP32, exact): the FP32 loop on them must equal the fixed-point loop."""
    return B.Tables(t.M, t.N, t.K, t.ldG, (t.Gq_rows.float() * 2.0 ** -14).contiguous(), t.D,
                    t.Y, t.sqrtw, t.phi, t.info, t.precision, Yhi=t.Yhi, Ylo=t.Ylo,
                    parts=t.parts, tx=t.tx, T=t.T)


def test_whole_row_words_match_oracle():
    d = synth.area32_inputs(2)
    say("whole-row words: 32x32 areas, no parts, K=2048")
    phi32, t, lost = _dense_tables(d, 32)
    b = d["blocks"][0]
    _, sup = oracle.area_signal(d["images"][b.img], lost[b.img], b.y0, b.x0, 32, 32)
    C, D = oracle.table_generation(phi32, oracle.area_weights(32, 32, 0.8, sup))
    G = oracle.unit_table(C, D)
    ref = oracle.quantise_table(G).astype(np.int32)
    Gq = t.Gq_rows.cpu().numpy().astype(np.int32)
    K = 2048
    diff = np.abs(Gq[:, :K] - ref)
    x = G * 2.0 ** 14
    near = np.abs(np.abs(x - np.floor(x)) - 0.5)[diff > 0]
    print(f"whole-row words differing from the oracle's: {int((diff > 0).sum())} of {K * K} "
          f"(by at most {int(diff.max())})")
    assert diff.max() <= 1 and (near < 1e-2).all()
    assert (Gq[np.arange(K), np.arange(K)] == 16384).all()
    assert (Gq[:, K:] == 0).all()


def test_whole_row_route_is_exact_word_arithmetic():
    """The loop over whole rows with SE_ROWS_Q14 equals the FP32 loop on the
    dequantised words bit for bit (batch call and plain per-block form)."""
    d = synth.area32_inputs(4)
    say("whole-row words: Q14 loop == FP32 loop on dequantised rows (batch, plain)")
    _, t, _ = _dense_tables(d, 32)
    q = _run(t, d["images"], d["blocks"], 100, True)
    f = _run(_row_twin(t), d["images"], d["blocks"], 100, False)
    for name, x, y in zip(("sel", "coef", "g_loss", "image"), q, f):
        assert torch.equal(x, y), f"{name} differs"
    img = torch.from_numpy(d["images"]).to(dev())
    bl = d["blocks"][:8]
    sel, coef, g = B.extrapolate_plain(t, img, bl, 0.5, 100, rows_q14=True)
    img2 = torch.from_numpy(d["images"]).to(dev())
    sel2, coef2, g2 = B.extrapolate_plain(_row_twin(t), img2, bl, 0.5, 100)
    torch.cuda.synchronize()
    assert torch.equal(sel, sel2) and torch.equal(coef, coef2) and torch.equal(g, g2)
    assert torch.equal(img, img2)


def test_whole_row_route_area64_against_oracle():
    """64 x 64 areas without declared parts (K = 8192, the loop over whole
    rows, four waves per block): the fixed-point loop against the oracle run
    on its own words, on a seeded sample of 16 of 256 blocks."""
    d = synth.area64_inputs(1)
    say("whole-row words: 64x64 areas, no parts, K=8192, I=300, 256 blocks")
    phi32, t, lost = _dense_tables(d, 64)
    n = 256
    sel, coef, g, img = [x.numpy() for x in _run(t, d["images"], d["blocks"], 300, True, n=n)]
    sample = sorted(np.random.default_rng(64).choice(n, 16, replace=False))
    st = oracle_check(d["images"], d["blocks"][:n], phi32, 64, 64, 0.8, 0.5, 300, sel, g, img,
                      sample=sample, tol=TOL_Q14, q14=True, tables=t,
                      lost=synth.lost_mask(2048, 2048, d["blocks"])[None])
    print(f"whole-row words area 64 vs oracle on words: {describe(st)}")
    assert st["worst"] <= TOL_Q14

