"""Complex dictionaries on the GPU (the paper's general case with conjugated
atoms): the Hermitian tables, the complex initial projections and the loop
against the FP64 oracle, on the DFT and binarized-DFT atoms of the paper's
Fig. 1 scenario."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth

from helpers import describe, oracle_check
from test_gpu_parity import TOL_FP32, dev, say, upload_phi

pytestmark = pytest.mark.gpu


def _tables(phi, images, blocks, M, N, ref_block=0, parts=()):
    n_img, H, W = images.shape
    lost = np.stack([synth.lost_mask(H, W, blocks, i) for i in range(n_img)])
    w = B.area_weights(M, N, 0.8, torch.from_numpy(lost).to(dev()), [blocks[ref_block]])
    t = B.weighted_gram(upload_phi(phi.real), w[0].contiguous(), M, N,
                        phi_im=upload_phi(phi.imag), parts=parts)
    return t, w[0], lost


def test_complex_gram_matches_oracle():
    M = N = 16
    say("complex tables: DFT 16^2 u binarized DFT 16^2 (K=512), one loss in the area")
    phi = synth.round_to_f32(synth.dictionary(M, N, ("dft", "bdft")))
    sup = np.ones((M, N), bool)
    sup[5:9, 6:11] = False
    w_ref = oracle.area_weights(M, N, 0.8, sup).astype(np.float32).astype(np.float64)
    w_d = torch.from_numpy(w_ref.astype(np.float32)).to(dev())
    t = B.weighted_gram(upload_phi(phi.real), w_d, M, N, phi_im=upload_phi(phi.imag))
    torch.cuda.synchronize()
    K = phi.shape[0]
    Gr = t.G.cpu().numpy()[:, :K].astype(np.float64)
    Gi = t.G_im.cpu().numpy()[:, :K].astype(np.float64)
    assert np.all(t.G.cpu().numpy()[:, K:] == 0) and np.all(t.G_im.cpu().numpy()[:, K:] == 0)
    # Hermitian exactly (Algorithm 2's mirror)
    np.testing.assert_array_equal(Gr, Gr.T)
    np.testing.assert_array_equal(Gi, -Gi.T)
    C_ref, D_ref = oracle.table_generation(phi, w_ref)
    np.testing.assert_allclose(t.D.cpu().numpy(), D_ref, rtol=2e-6)
    G_ref = D_ref[:, None] * C_ref * D_ref[None, :]
    err = max(np.abs(Gr - G_ref.real).max(), np.abs(Gi - G_ref.imag).max())
    print(f"max |G - G_oracle| = {err:.3g}")
    assert err < 2e-5


def test_complex_project_matches_oracle():
    M = N = 16
    say("complex projections: DFT 16^2 u binarized DFT 16^2, 6 blocks, two across the border")
    phi = synth.round_to_f32(synth.dictionary(M, N, ("dft", "bdft")))
    H, W = 3 * M + 4, 3 * N + 8
    images = np.stack([synth.synth_image(H, W, seed=70 + s) for s in range(2)])
    blocks = [synth.Block(i, y, x, 5, 5, 6, 6)
              for i in range(2) for (y, x) in ((-3, -2), (M, N), (2 * M, 2 * N + 6))]
    t, w_d, lost = _tables(phi, images, blocks, M, N, ref_block=1)
    K = phi.shape[0]
    img = torch.from_numpy(images).to(dev())
    db = B.DeviceBlocks(t, img, blocks)
    R = torch.full((len(blocks), t.ldR), float("nan"), dtype=torch.float32, device=dev())
    ws = torch.empty(max(1, B.project_ws_bytes(t, len(blocks))), dtype=torch.uint8, device=dev())
    B.project(t, img, db, R, ws)
    torch.cuda.synchronize()
    Rh = R.cpu().numpy().astype(np.float64)
    L = t.ldG
    assert np.all(Rh[:, K:L] == 0) and np.all(Rh[:, L + K:] == 0)
    w = w_d.cpu().numpy().astype(np.float64)
    _, D_ref = oracle.table_generation(phi, w)
    for i, b in enumerate(blocks):
        s, _ = oracle.area_signal(images[b.img], lost[b.img], b.y0, b.x0, M, N)
        ref = D_ref * (np.conj(phi) @ (w * s))
        scale = np.abs(ref).max()
        err = max(np.abs(Rh[i, :K] - ref.real).max(), np.abs(Rh[i, L:L + K] - ref.imag).max())
        assert err <= 1e-5 * scale, f"block {i}: {err} vs scale {scale}"


@pytest.mark.parametrize("M,N,subs", [(16, 16, ("dft", "bdft")), (20, 12, ("bdft", "dft")),
                                      (16, 16, ("dft",))])
def test_dft_part_projections_match_oracle(M, N, subs):
    """A declared DFT part (Section VI's complex case): the projections of
    its atoms are 2-D DFTs of the weighted blocks (six real products on the
    matrix cores), the other atoms' the GEMM; against the oracle's conjugated
    scalar products (eq. 12), with blocks across the image border, an area
    whose sides are not multiples of 16, a part that does not start at atom
    0, and a dictionary that is only the part."""
    say(f"complex projections with a DFT part: {M}x{N}, {subs}")
    phi = synth.round_to_f32(synth.dictionary(M, N, subs))
    parts = synth.dictionary_parts(M, N, subs)
    assert [p for p, _ in parts] == ["dft"]
    H, W = 3 * M + 4, 3 * N + 8
    images = np.stack([synth.synth_image(H, W, seed=80 + s) for s in range(2)])
    blocks = [synth.Block(i, y, x, 5, 5, 6, 6)
              for i in range(2) for (y, x) in ((-3, -2), (M, N), (2 * M, 2 * N + 6))]
    t, w_d, lost = _tables(phi, images, blocks, M, N, ref_block=1, parts=parts)
    t0, _, _ = _tables(phi, images, blocks, M, N, ref_block=1)
    K = phi.shape[0]
    img = torch.from_numpy(images).to(dev())
    db = B.DeviceBlocks(t, img, blocks)
    Rs = []
    for tt in (t, t0):
        R = torch.full((len(blocks), tt.ldR), float("nan"), dtype=torch.float32, device=dev())
        ws = torch.empty(max(1, B.project_ws_bytes(tt, len(blocks))), dtype=torch.uint8,
                         device=dev())
        B.project(tt, img, db, R, ws)
        torch.cuda.synchronize()
        Rs.append(R.cpu().numpy().astype(np.float64))
    Rh, R0 = Rs
    L = t.ldG
    assert np.all(Rh[:, K:L] == 0) and np.all(Rh[:, L + K:] == 0)
    # the tables themselves do not depend on the declaration
    np.testing.assert_array_equal(t.G.cpu().numpy(), t0.G.cpu().numpy())
    np.testing.assert_array_equal(t.G_im.cpu().numpy(), t0.G_im.cpu().numpy())
    w = w_d.cpu().numpy().astype(np.float64)
    _, D_ref = oracle.table_generation(phi, w)
    first = parts[0][1]
    part = slice(first, first + M * N)
    for i, b in enumerate(blocks):
        s, _ = oracle.area_signal(images[b.img], lost[b.img], b.y0, b.x0, M, N)
        ref = D_ref * (np.conj(phi) @ (w * s))
        scale = np.abs(ref).max()
        err = max(np.abs(Rh[i, :K] - ref.real).max(), np.abs(Rh[i, L:L + K] - ref.imag).max())
        assert err <= 1e-5 * scale, f"block {i}: {err} vs scale {scale}"
        # outside the part both routes run the same GEMM
        out = np.ones(K, bool)
        out[part] = False
        np.testing.assert_array_equal(Rh[i, :K][out], R0[i, :K][out])
        np.testing.assert_array_equal(Rh[i, L:L + K][out], R0[i, L:L + K][out])


def test_dft_part_refused_when_it_does_not_match():
    """A DFT part is verified against the atoms given: declared over the
    binarized atoms it fails with SE_EINVAL."""
    M = N = 16
    say("complex tables: a DFT part over binarized DFT atoms is refused")
    phi = synth.round_to_f32(synth.dictionary(M, N, ("dft", "bdft")))
    with pytest.raises(RuntimeError, match="does not match"):
        B.weighted_gram(upload_phi(phi.real), torch.ones(M * N, device=dev()), M, N,
                        phi_im=upload_phi(phi.imag), parts=[("dft", M * N)])


def _batch(t, images, blocks, iters):
    img = torch.from_numpy(images).to(dev())
    sel, coef, g = B.extrapolate_batch(t, img, blocks, 0.5, iters)
    torch.cuda.synchronize()
    return sel.cpu().numpy(), coef.cpu().numpy(), g.cpu().numpy(), img.cpu().numpy()


@pytest.mark.parametrize("parts,n_img,declare", [(("dft",), 2, False),
                                                 (("dft", "bdft"), 2, False),
                                                 (("dft", "bdft"), 2, True)])
def test_complex_batch_parity(parts, n_img, declare):
    """Algorithm 3 with complex atoms: selections equal to the oracle's
    (modulo parallel atoms and near-ties) and the real part of the model
    within the FP32 bar.  For a real signal the DFT coefficients of
    frequencies (mu, eta) and (-mu, -eta) are conjugate, so their scores tie
    exactly and rounding decides which is taken first; the comparison takes
    such picks as ties (the oracle re-run along the device's choices, within
    the near-tie window, must give the same model)."""
    d = synth.dft32_inputs(n_img)
    say(f"complex batch: 32x32 areas, {parts}, DFT part declared: {declare}, "
        f"{len(d['blocks'])} blocks, I=100")
    phi = synth.round_to_f32(synth.dictionary(32, 32, parts))
    t, _, _ = _tables(phi, d["images"], d["blocks"], 32, 32,
                      parts=synth.dictionary_parts(32, 32, parts) if declare else ())
    sel, coef, g, out = _batch(t, d["images"], d["blocks"], 100)
    assert coef.shape[1] == 200
    st = oracle_check(d["images"], d["blocks"], phi, 32, 32, 0.8, 0.5, 100, sel, g, out,
                      tol=TOL_FP32, tables=t)
    print(describe(st))
    assert st["worst"] <= TOL_FP32


@pytest.mark.parametrize("declare", [False, True])
def test_complex_routes_agree_and_refusals(declare):
    """The batched call, the two stages and the device-descriptor call give
    the same bits (with and without the DFT half declared as a transform
    part); the per-block form, rows on demand and split-BF16 tables refuse
    complex dictionaries."""
    d = synth.dft32_inputs(1)
    say(f"complex tables: routes agree (DFT part declared: {declare}); unsupported calls refuse")
    phi = synth.round_to_f32(d["phi"])
    t, w_d, _ = _tables(phi, d["images"], d["blocks"], 32, 32,
                        parts=d["tx_parts"] if declare else ())
    sel0, coef0, g0, out0 = _batch(t, d["images"], d["blocks"], 60)
    n = len(d["blocks"])
    img = torch.from_numpy(d["images"]).to(dev())
    db = B.DeviceBlocks(t, img, d["blocks"])
    R = torch.empty((n, t.ldR), dtype=torch.float32, device=dev())
    ws = torch.empty(max(1, B.project_ws_bytes(t, n)), dtype=torch.uint8, device=dev())
    sel = torch.zeros((n, 60), dtype=torch.int32, device=dev())
    g = torch.zeros((n, 64), dtype=torch.float32, device=dev())
    B.project(t, img, db, R, ws)
    B.iterate(t, R, img, db, 0.5, 60, sel, None, g)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(sel.cpu().numpy(), sel0)
    np.testing.assert_array_equal(g.cpu().numpy(), g0[:, :64])
    np.testing.assert_array_equal(img.cpu().numpy(), out0)
    img2 = torch.from_numpy(d["images"]).to(dev())
    db2 = B.DeviceBlocks(t, img2, d["blocks"])
    nb = B.extrapolate_device_ws_bytes(t, n)
    assert nb > 0
    wsd = torch.empty(nb, dtype=torch.uint8, device=dev())
    g2 = torch.zeros((n, 64), dtype=torch.float32, device=dev())
    B.extrapolate_device(t, img2, db2, 0.5, 60, wsd, None, None, g2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g2.cpu().numpy(), g0[:, :64])
    # refusals
    with pytest.raises(B.SEError) as e:
        B.extrapolate_plain(t, img, d["blocks"][:1], 0.5, 10)
    assert e.value.code == B.SE_EINVAL
    with pytest.raises(B.SEError):
        B.weighted_gram(upload_phi(phi.real), w_d.contiguous(), 32, 32, B.SE_BF16X3,
                        phi_im=upload_phi(phi.imag))
    # R too short for the imaginary halves
    with pytest.raises(B.SEError):
        B.project(t, img, db, torch.empty((n, t.ldG), dtype=torch.float32, device=dev()), ws)
