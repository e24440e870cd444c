"""Transform parts (Section VI, eq. 21-23) on the GPU: the initial projections
of declared DCT-II / Walsh-Hadamard ranges are computed as separable
transforms of the weighted area signal; the results must match the FP64
oracle's direct scalar products, and declarations that do not match the
atoms must be refused."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth

from helpers import describe, oracle_check
from test_gpu_parity import TOL_BF16X3, TOL_FP32, dev, run_batch, say, shared_tables, upload_phi

pytestmark = pytest.mark.gpu


def _project(t, imgs, blocks):
    img_d = torch.from_numpy(imgs).to(dev())
    db = B.DeviceBlocks(t, img_d, blocks)
    R = torch.full((len(blocks), t.ldG), float("nan"), dtype=torch.float32, device=dev())
    ws = torch.empty(max(B.project_ws_bytes(t, len(blocks)), 1), dtype=torch.uint8,
                     device=dev())
    B.project(t, img_d, db, R, ws)
    torch.cuda.synchronize()
    return R.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("M,N,parts,n_gauss", [
    (32, 32, ("dct", "wht"), 0),          # every atom in a transform part
    (48, 48, ("dct", "gauss"), 300),      # transform, then a dense range
    (16, 8, ("gauss", "wht", "dct"), 70),  # dense range first, two parts after it
    (7, 5, ("dct", "gauss"), 13),         # odd sides: padded transform tiles
    (64, 64, ("wht", "dct"), 0),          # the largest area, WHT first
])
def test_project_with_parts_matches_oracle(M, N, parts, n_gauss):
    say(f"project with transform parts M={M} N={N} parts={parts}")
    phi = synth.round_to_f32(synth.dictionary(M, N, parts, seed=M + N, n_gauss=n_gauss))
    tx = synth.dictionary_parts(M, N, parts, n_gauss)
    K = phi.shape[0]
    H, W = 3 * M + 1, 3 * N + 2
    imgs = np.stack([synth.synth_image(H, W, seed=s) for s in range(2)])
    lh, lw = max(1, M // 3), max(1, N // 3)
    # one area leaves the image on the top left, one on the bottom right
    blocks = [synth.Block(i, y, x, (M - lh) // 2, (N - lw) // 2, lh, lw)
              for i in range(2) for (y, x) in ((-2, -3), (M, N), (2 * M + 3, 2 * N + 4))]
    t, w_d, lost = shared_tables(imgs, blocks, upload_phi(phi), M, N, 0.8, parts=tx)
    assert len(t.parts) == len(tx)
    Rh = _project(t, imgs, blocks)
    assert np.all(Rh[:, K:] == 0.0)
    w = w_d.cpu().numpy().astype(np.float64)
    _, D_ref = oracle.table_generation(phi, w)
    for i, b in enumerate(blocks):
        s, _ = oracle.area_signal(imgs[b.img], lost[b.img], b.y0, b.x0, M, N)
        ref = D_ref * (phi @ (w * s))
        scale = np.abs(ref).max()
        err = np.abs(Rh[i, :K] - ref).max()
        assert err <= 1e-5 * scale, f"block {i}: {err} vs scale {scale}"


@pytest.mark.parametrize("M,N,parts,n_gauss,precision", [
    (32, 32, ("dct", "wht"), 0, B.SE_FP32),        # every row from transforms
    (48, 48, ("dct", "gauss"), 300, B.SE_FP32),    # dense block after the part
    (16, 8, ("gauss", "wht", "dct"), 72, B.SE_FP32),  # dense block first
    (7, 5, ("dct", "gauss"), 13, B.SE_FP32),       # unaligned dense start: one product
    (32, 32, ("dct", "wht"), 0, B.SE_BF16X3),
    (48, 48, ("dct", "gauss"), 300, B.SE_BF16X3),
])
def test_gram_with_parts_matches_oracle(M, N, parts, n_gauss, precision):
    """Algorithm 2 with transform parts: rows over the part columns are
    transforms of the weighted atoms (Section VI), the dense block a product;
    the table must equal the oracle's D C D and be exactly symmetric."""
    say(f"weighted_gram with parts M={M} N={N} parts={parts} precision={precision}")
    phi = synth.round_to_f32(synth.dictionary(M, N, parts, seed=M * N, n_gauss=n_gauss))
    tx = synth.dictionary_parts(M, N, parts, n_gauss)
    K = phi.shape[0]
    sup = np.ones((M, N), bool)
    sup[M // 3:M // 3 + 3, N // 4:N // 4 + 2] = False
    sup[0, :] = False                      # a border row outside the image
    w_ref = oracle.area_weights(M, N, 0.8, sup)
    w_d = torch.from_numpy(w_ref.astype(np.float32)).to(dev())
    t = B.weighted_gram(upload_phi(phi), w_d, M, N, precision, parts=tx)
    torch.cuda.synchronize()
    G = t.G.cpu().numpy()[:, :K].astype(np.float64)
    assert np.all(t.G.cpu().numpy()[:, K:] == 0.0)
    D = t.D.cpu().numpy().astype(np.float64)
    C_ref, D_ref = oracle.table_generation(phi, w_ref.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(D, D_ref, rtol=2e-6)
    G_ref = D_ref[:, None] * C_ref * D_ref[None, :]
    tol = 2e-5 if precision == B.SE_FP32 else 2e-4
    err = np.abs(G - G_ref).max()
    print(f"max |G - G_oracle| = {err:.3g}")
    assert err < tol
    np.testing.assert_array_equal(G, G.T)


def test_parts_equal_dense_projection():
    """With and without the declaration the projections agree to FP32
    rounding (same tables, two routes to R)."""
    d = synth.area32_inputs(2)
    say("32x32 areas: projections with and without declared parts")
    phi = upload_phi(synth.round_to_f32(d["phi"]))
    t0, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8)
    t1, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8, parts=d["tx_parts"])
    R0 = _project(t0, d["images"], d["blocks"])
    R1 = _project(t1, d["images"], d["blocks"])
    scale = np.abs(R0).max()
    assert np.abs(R0 - R1).max() <= 2e-6 * scale


def test_wrong_declaration_is_refused():
    M = N = 16
    say("weighted_gram refuses declarations that do not match the atoms")
    phi_np = synth.round_to_f32(synth.dictionary(M, N, ("dct", "wht")))
    w = torch.ones(M * N, dtype=torch.float32, device=dev())
    phi = upload_phi(phi_np)
    # kinds swapped
    with pytest.raises(B.SEError) as e:
        B.weighted_gram(phi, w, M, N, parts=[("wht", 0), ("dct", 256)])
    assert e.value.code == B.SE_EINVAL
    # shifted by one atom
    with pytest.raises(B.SEError):
        B.weighted_gram(phi, w, M, N, parts=[("dct", 1)])
    # one atom changed by 1e-4 in one pixel
    bad = phi_np.copy()
    bad[300, 17] += 1e-4
    with pytest.raises(B.SEError):
        B.weighted_gram(upload_phi(bad), w, M, N, parts=[("dct", 0), ("wht", 256)])
    # the same dictionary, correctly declared, is accepted
    t = B.weighted_gram(phi, w, M, N, parts=[("dct", 0), ("wht", 256)])
    torch.cuda.synchronize()
    assert t.parts == ((B.SE_PART_DCT2, 0), (B.SE_PART_WHT2, 256))


def test_area32_batch_parity_with_parts():
    d = synth.area32_inputs(2)
    say("32x32 areas batched with transform parts: 2 images, 32 blocks, K=2048, I=100")
    phi = synth.round_to_f32(d["phi"])
    t, _, _ = shared_tables(d["images"], d["blocks"], upload_phi(phi), 32, 32, 0.8,
                            parts=d["tx_parts"])
    sel, coef, g, out = run_batch(t, d["images"], d["blocks"], 0.5, 100)
    st = oracle_check(d["images"], d["blocks"], phi, 32, 32, 0.8, 0.5, 100, sel, g, out,
                      tol=TOL_FP32, coef=coef, tables=t)
    print(describe(st))
    assert st["agree"] == st["n"]


@pytest.mark.parametrize("with_parts", [True, False])
def test_area48_batch_parity(with_parts):
    """The 512x512 workload: DCT 48^2 (declared as a transform part, or dense)
    followed by 1792 dense Gaussian atoms; 32 sampled blocks against the
    oracle, selections held to the derived window."""
    d = synth.area48_inputs(1)
    say(f"48x48 areas batched, DCT part declared {with_parts}: 256 blocks, K=4096, I=200")
    phi = synth.round_to_f32(d["phi"])
    t, _, _ = shared_tables(d["images"], d["blocks"], upload_phi(phi), 48, 48, 0.8,
                            parts=d["tx_parts"] if with_parts else ())
    sel, coef, g, out = run_batch(t, d["images"], d["blocks"], 0.5, 200)
    sample = np.random.default_rng(48).choice(256, 32, replace=False)
    st = oracle_check(d["images"], d["blocks"], phi, 48, 48, 0.8, 0.5, 200, sel, g, out,
                      sample=sample, tol=TOL_FP32, coef=coef, tables=t)
    print(f"48x48 parts {with_parts}: {describe(st)}")


@pytest.mark.parametrize("precision", [B.SE_FP32, B.SE_BF16X3])
def test_area64_parity_with_parts(precision):
    name = "FP32" if precision == B.SE_FP32 else "BF16X3"
    d = synth.area64_inputs(1)
    say(f"64x64 areas {name} with transform parts: 1024 blocks, K=8192, I=300")
    phi = synth.round_to_f32(d["phi"])
    t, _, _ = shared_tables(d["images"], d["blocks"], upload_phi(phi), 64, 64, 0.8, precision,
                            parts=d["tx_parts"])
    sel, coef, g, out = run_batch(t, d["images"], d["blocks"], 0.5, 300)
    tol = TOL_FP32 if precision == B.SE_FP32 else TOL_BF16X3
    sample = np.random.default_rng(65).choice(1024, 32, replace=False)
    st = oracle_check(d["images"], d["blocks"], phi, 64, 64, 0.8, 0.5, 300, sel, g, out,
                      sample=sample, tol=tol, coef=coef, tables=t)
    print(f"64x64 {name} with parts: {describe(st)}")
