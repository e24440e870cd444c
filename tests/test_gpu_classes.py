"""Parity-class tables (DCT-II and Walsh-Hadamard atoms under a
mirror-symmetric weight pattern, eq. 16): the class order against one derived
here from the 1-D rows' own symmetry, the class rows against the full table,
the class form of the one-launch route against the full-row route and the
oracle, its graph replays, and the patterns that must not get class tables."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth

from helpers import describe, oracle_check
from test_gpu_parity import TOL_FP32, dev, say, shared_tables, upload_phi

pytestmark = pytest.mark.gpu


def _row_parity(r):
    """0 if the 1-D row is even about its centre, 1 if odd (checked)."""
    if np.allclose(r[::-1], r, rtol=0, atol=1e-12):
        return 0
    assert np.allclose(r[::-1], -r, rtol=0, atol=1e-12)
    return 1


def expected_class_order(M, N, parts):
    """Original atom index per position of the class order, derived from the
    rows' symmetry: class 2 pv + ph, then the parts by first atom, then
    (k1 // 2, k2 // 2)."""
    rows = {"dct": synth.dct_rows, "wht": synth.wht_rows}
    entries = []
    for qi, (name, first) in enumerate(sorted(parts, key=lambda p: p[1])):
        pv = [_row_parity(x) for x in rows[name](M)]
        ph = [_row_parity(x) for x in rows[name](N)]
        for k1 in range(M):
            for k2 in range(N):
                entries.append(((2 * pv[k1] + ph[k2], qi, k1 // 2, k2 // 2), first + k1 * N + k2))
    entries.sort()
    return np.array([o for _, o in entries]), np.array([e[0][0] for e in entries])


def test_class_tables_structure():
    d = synth.area32_inputs(2)
    say("class tables: 32x32 areas, centred 8x8 loss, DCT u WHT (K=2048)")
    phi = upload_phi(synth.round_to_f32(d["phi"]))
    t, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8, parts=d["tx_parts"])
    torch.cuda.synchronize()
    assert t.n_classes == 4
    K, Kc = 2048, 512
    order, cls_of = expected_class_order(32, 32, d["tx_parts"])
    cls = t.cls.cpu().numpy()
    np.testing.assert_array_equal(cls[:, 0], order)
    D = t.D.cpu().numpy()
    np.testing.assert_array_equal(cls[:, 1].view(np.float32), D[order])
    G = t.G.cpu().numpy()[:, :K]
    Gc = t.Gc.cpu().numpy()
    for c in range(4):
        blk = order[c * Kc:(c + 1) * Kc]
        np.testing.assert_array_equal(Gc[c * Kc:(c + 1) * Kc], G[np.ix_(blk, blk)])
    # every entry between atoms of different classes is 0 up to rounding
    cross = cls_of[np.argsort(order)]
    mask = cross[:, None] != cross[None, :]
    worst = np.abs(G[mask]).max()
    print(f"max |G| between classes = {worst:.3g}")
    assert worst < 1e-6


def test_class_route_matches_full_rows_and_oracle():
    d = synth.area32_inputs(8)
    say("class route: 128 blocks, K=2048, I=100, against full rows and the oracle")
    phi_np = synth.round_to_f32(d["phi"])
    phi = upload_phi(phi_np)
    tc, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8, parts=d["tx_parts"])
    tf, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8, parts=d["tx_parts"],
                             classes=False)
    assert tc.n_classes == 4 and tf.n_classes == 0
    out = {}
    for name, t in (("class", tc), ("full", tf)):
        img = torch.from_numpy(d["images"]).to(dev())
        sel, coef, g = B.extrapolate_batch(t, img, d["blocks"], 0.5, 100)
        torch.cuda.synchronize()
        out[name] = (sel.cpu().numpy(), coef.cpu().numpy(), g.cpu().numpy(), img.cpu().numpy())
    same = int(np.all(out["class"][0] == out["full"][0], axis=1).sum())
    dg = np.abs(out["class"][2] - out["full"][2]).max()
    print(f"class vs full rows: identical selections {same}/128, max|dg|={dg:.3g}")
    assert dg <= TOL_FP32
    sel, coef, g, img = out["class"]
    st = oracle_check(d["images"], d["blocks"], phi_np, 32, 32, 0.8, 0.5, 100, sel, g, img,
                      tol=TOL_FP32, coef=coef, tables=tc)
    print(f"class route vs oracle: {describe(st)}")
    assert st["agree"] == st["n"]
    assert st["worst"] <= TOL_FP32


def test_class_route_device_call_and_graph_replays():
    """se_extrapolate_device with class tables equals se_extrapolate_batch bit
    for bit, and a captured step replays to the same bits."""
    d = synth.area32_inputs(8)
    say("class route: one launch on device descriptors, eager and graph replays")
    phi = upload_phi(synth.round_to_f32(d["phi"]))
    t, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8, parts=d["tx_parts"])
    assert t.n_classes == 4
    n = len(d["blocks"])
    img_b = torch.from_numpy(d["images"]).to(dev())
    sel_b, coef_b, g_b = B.extrapolate_batch(t, img_b, d["blocks"], 0.5, 100)
    img0 = torch.from_numpy(d["images"]).to(dev())
    img = img0.clone()
    db = B.DeviceBlocks(t, img, d["blocks"])
    assert B.extrapolate_device_ws_bytes(t, n) == 0
    sel = torch.zeros((n, 100), dtype=torch.int32, device=dev())
    coef = torch.zeros((n, 100), dtype=torch.float32, device=dev())
    g = torch.zeros((n, g_b.shape[1]), dtype=torch.float32, device=dev())

    def step(stream=None):
        B.extrapolate_device(t, img, db, 0.5, 100, None, sel, coef, g, stream=stream)

    step()
    torch.cuda.synchronize()
    for x, y in ((sel, sel_b), (coef, coef_b), (g, g_b), (img, img_b)):
        assert torch.equal(x, y)
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
        for x, y in ((sel, sel_b), (coef, coef_b), (g, g_b), (img, img_b)):
            assert torch.equal(x, y), f"replay {rep}"


def test_no_class_tables_without_the_structure():
    """An off-centre loss (weights not mirror-symmetric) and a dictionary
    with dense atoms get no class tables; the route then streams full rows."""
    d = synth.area32_inputs(2)
    phi = upload_phi(synth.round_to_f32(d["phi"]))
    say("class tables refused: off-centre loss; dense atoms")
    off = [synth.Block(b.img, b.y0, b.x0, 10, 12, 8, 8) for b in d["blocks"]]
    t, _, _ = shared_tables(d["images"], off, phi, 32, 32, 0.8, parts=d["tx_parts"])
    assert t.n_classes == 0 and t.Gc is None
    mixed = synth.round_to_f32(synth.dictionary(32, 32, ("dct", "gauss"), n_gauss=1024))
    t2, _, _ = shared_tables(d["images"], d["blocks"], upload_phi(mixed), 32, 32, 0.8,
                             parts=synth.dictionary_parts(32, 32, ("dct", "gauss"), 1024))
    assert t2.n_classes == 0


def _bucket(n):
    b = 0
    while (1 << b) < n:
        b += 1
    return b


def test_class_route_shapes_agree():
    """The one-wave class loop (class maxima kept across iterations) and the
    two-wave one (the whole row scanned every iteration) select the same
    positions, so every output is the same bit for bit."""
    d = synth.area32_inputs(8)
    say("class route: loop shapes 1x32 (kept class maxima) and 2x16 (full scans)")
    phi = upload_phi(synth.round_to_f32(d["phi"]))
    t, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8, parts=d["tx_parts"])
    assert t.n_classes == 4
    got = []
    for w, v in ((1, 32), (2, 16)):
        B.tune_clear()
        B.tune_import(f"2048 1024 {_bucket(len(d['blocks']))} {w} {v} 64\n")
        try:
            img = torch.from_numpy(d["images"]).to(dev())
            sel, coef, g = B.extrapolate_batch(t, img, d["blocks"], 0.5, 100)
            torch.cuda.synchronize()
            got.append([x.cpu() for x in (sel, coef, g, img)])
        finally:
            B.tune_clear()
    for name, x, y in zip(("sel", "coef", "g_loss", "image"), *got):
        assert torch.equal(x, y), f"{name} differs between the loop shapes"


@pytest.mark.parametrize("M,N", [(64, 16), (64, 64)])
def test_class_route_exact_tie_between_classes(M, N):
    """An exact tie between atoms of two parity classes must go to the lower
    atom index (eq. 18 with ties to the lowest k), although the class order
    puts the other atom first.  Walsh-Hadamard atoms (1, 3) (class 2) and
    (3, 1) (class 1) of a 64 x 16 area (one wave per block) and of a 64 x 64
    area (four waves): with 0/1 weights and a signal built from the two
    atoms, every product and sum of the projections and of their table rows
    is a dyadic number computed exactly on both sides, so the scores are
    bit-identical on the device as in the oracle."""
    say(f"class route, exact tie between classes: {M}x{N} area, WHT atoms (1,3) and (3,1)")
    phi = synth.round_to_f32(synth.dictionary(M, N, ("dct", "wht")))
    P = M * N
    a, b = P + 1 * N + 3, P + 3 * N + 1            # classes 2 and 1 (lower position: b)
    sup = np.ones((M, N), bool)
    ly, lx = M // 2 - 8, N // 2 - 4
    sup[ly:ly + 16, lx:lx + 8] = False
    w = sup.reshape(-1).astype(np.float64)
    va, vb = np.sign(phi[a]), np.sign(phi[b])
    s = (96 + 40 * (va + vb)) * w
    img = s.reshape(1, M, N).astype(np.uint8)
    t = B.weighted_gram(upload_phi(phi), torch.from_numpy(w.astype(np.float32)).to(dev()), M, N,
                        parts=synth.dictionary_parts(M, N, ("dct", "wht")))
    assert t.n_classes == 4
    blk = [synth.Block(0, 0, 0, ly, lx, 16, 8)]
    img_d = torch.from_numpy(img).to(dev())
    sel, coef, g = B.extrapolate_batch(t, img_d, blk, 0.5, 8)
    torch.cuda.synchronize()
    sel = sel.cpu().numpy()[0]
    phi64 = phi.astype(np.float64)
    C, D = oracle.table_generation(phi64, w)
    res = oracle.fase(s, w, phi64, C, D, 0.5, 8, oracle.duplicate_classes(phi64))
    ties = np.nonzero(res.second == res.best)[0]
    print(f"device {sel.tolist()}, oracle {res.sel.tolist()}, exact ties at {ties.tolist()}")
    assert res.sel[2] == a and res.best[2] == res.second[2]    # the tie the test is built on
    np.testing.assert_array_equal(sel, res.sel)
    gref = res.g.reshape(M, N)[ly:ly + 16, lx:lx + 8].reshape(-1)
    assert np.abs(g.cpu().numpy()[0, :128] - gref).max() <= TOL_FP32
