"""Pins of the oracle's three-dimensional model (areas of T consecutive video
frames; the paper's closing section extends the method to three dimensions,
generated as in two).  Each test ties the 3-D functions to something other
than themselves: the pinned 2-D functions at T = 1, closed-form weights,
coordinate-encoded frames, exact recovery of a signal that is one atom, the
equality of Algorithm 1 and Algorithm 3, and the symmetry of an isotropic
model under a permutation of the three axes."""
import numpy as np

import oracle
from paper_2204_14194_amd import synth


def test_volume_weights_reduce_to_area_weights():
    rng = np.random.default_rng(3)
    sup = rng.random((9, 11)) > 0.2
    a = oracle.area_weights(9, 11, 0.8, sup)
    v = oracle.volume_weights(1, 9, 11, 0.8, sup[None])
    np.testing.assert_array_equal(a, v)


def test_volume_weights_closed_form():
    """T = 3, M = 3, N = 5, centre (1, 1, 2): weight 1 at the centre,
    rho at distance 1 along each axis, rho^sqrt(6) at the corner (0, 0, 0),
    0 on a masked sample; sample (tau, m, n) at (tau*3 + m)*5 + n."""
    rho = 0.8
    sup = np.ones((3, 3, 5), bool)
    sup[2, 0, 4] = False
    w = oracle.volume_weights(3, 3, 5, rho, sup)
    at = lambda t, m, n: w[(t * 3 + m) * 5 + n]
    assert at(1, 1, 2) == 1.0
    for p in ((0, 1, 2), (2, 1, 2), (1, 0, 2), (1, 2, 2), (1, 1, 1), (1, 1, 3)):
        assert abs(at(*p) - rho) < 1e-15, p
    assert abs(at(0, 0, 0) - rho ** np.sqrt(6.0)) < 1e-15
    assert abs(at(2, 2, 4) - rho ** np.sqrt(6.0)) < 1e-15
    assert abs(at(0, 1, 0) - rho ** np.sqrt(5.0)) < 1e-15
    assert at(2, 0, 4) == 0.0


def test_volume_signal_sample_order():
    """Frames whose values encode their coordinates: sample (tau, m, n) of the
    area must be frame t0+tau, row y0+m, column x0+n; samples outside the
    frames, the frame range or on a lost sample are 0 and not support."""
    F, H, W = 4, 6, 7
    f, y, x = np.meshgrid(np.arange(F), np.arange(H), np.arange(W), indexing="ij")
    frames = (40 * f + 6 * y + x).astype(np.uint8)
    lost = np.zeros((F, H, W), np.uint8)
    lost[2, 3, 4] = 1
    T, M, N, t0, y0, x0 = 3, 4, 5, 1, 2, 3
    s, sup = oracle.volume_signal(frames, lost, t0, y0, x0, T, M, N)
    for tau in range(T):
        for m in range(M):
            for n in range(N):
                k = (tau * M + m) * N + n
                ff, yy, xx = t0 + tau, y0 + m, x0 + n
                inside = yy < H and xx < W
                if inside and not lost[ff, yy, xx]:
                    assert s[k] == 40 * ff + 6 * yy + xx and sup[tau, m, n]
                else:
                    assert s[k] == 0 and not sup[tau, m, n]
    # an area that starts before the first frame
    s2, sup2 = oracle.volume_signal(frames, lost, -1, 0, 0, 2, 2, 2)
    assert not sup2[0].any() and (s2[:4] == 0).all()
    np.testing.assert_array_equal(s2[4:], frames[0, :2, :2].reshape(-1))


def test_conceal_video_with_one_frame_is_conceal():
    """T = 1 areas (each frame its own image) give exactly the 2-D result."""
    imgs = np.stack([synth.synth_image(40, 40, seed=s) for s in (1, 2)])
    blocks = [synth.Block(0, 4, 6, 6, 6, 4, 4), synth.Block(1, 20, 10, 5, 6, 5, 4),
              synth.Block(1, -4, 20, 7, 3, 4, 4)]
    M = N = 16
    phi = synth.dictionary(M, N, ("dct", "wht"))
    lost = np.stack([synth.lost_mask(40, 40, blocks, i) for i in range(2)])
    out3, per3 = oracle.conceal_video(imgs, lost, blocks, phi, 1, M, N, 0.8, 0.5, 25)
    for i in range(2):
        mine = [b for b in blocks if b.img == i]
        out2, per2 = oracle.conceal(imgs[i], lost[i], mine, phi, M, N, 0.8, 0.5, 25)
        np.testing.assert_array_equal(out3[i], out2)
        for b, (r2, g2) in zip(mine, per2):
            r3, g3 = per3[blocks.index(b)]
            np.testing.assert_array_equal(r3.sel, r2.sel)
            np.testing.assert_array_equal(g3[0], g2)


def test_single_atom_video_is_recovered_in_one_step():
    """A signal that equals one atom over the whole area: its weighted
    projection onto that atom is exact and no other atom scores higher
    (Cauchy-Schwarz in the weighted product), so with gamma = 1 one
    iteration of Algorithm 1 or 3 gives the atom itself over the loss box."""
    T, M, N = 4, 8, 8
    phi = synth.video_dictionary(T, M, N)
    j = (2 * M + 3) * N + 6                  # DCT atom (kt, k1, k2) = (2, 3, 6)
    F, H, W = 6, 12, 12
    t0, y0, x0 = 1, 2, 3
    vol = np.zeros((F, H, W))
    vol[t0:t0 + T, y0:y0 + M, x0:x0 + N] = 37.0 * phi[j].reshape(T, M, N)
    b = synth.Block(t0, y0, x0, 2, 3, 3, 4, 1, 2)      # loss: frames 1-2, 3x4 pixels
    lost = synth.video_lost_mask(F, H, W, [b])
    s, sup = oracle.volume_signal(vol, lost, t0, y0, x0, T, M, N)
    w = oracle.volume_weights(T, M, N, 0.8, sup)
    truth = 37.0 * phi[j].reshape(T, M, N)[1:3, 2:5, 3:7]
    for method in ("se", "fase"):
        if method == "se":
            res = oracle.se_original(s, w, phi, 1.0, 1)
        else:
            C, D = oracle.table_generation(phi, w)
            res = oracle.fase(s, w, phi, C, D, 1.0, 1)
        assert res.sel[0] == j
        g = res.g.reshape(T, M, N)[1:3, 2:5, 3:7]
        np.testing.assert_allclose(g, truth, atol=1e-10)
    # and through conceal_video (loss box placed in the right frames)
    _, per = oracle.conceal_video(vol, lost, [b], phi, T, M, N, 0.8, 1.0, 1)
    np.testing.assert_allclose(per[0][1], truth, atol=1e-10)


def test_video_algorithm1_equals_algorithm3():
    """FaSE reaches the result of SE exactly (up to rounding) in 3-D too."""
    T, M, N = 2, 8, 8
    phi = synth.video_dictionary(T, M, N)
    frames = synth.synth_video(6, 24, 24, seed=9)
    blocks = [synth.Block(1, 4, 6, 2, 2, 4, 4, 1, 1), synth.Block(3, 12, 10, 3, 1, 3, 5, 0, 2)]
    lost = synth.video_lost_mask(6, 24, 24, blocks)
    cls = oracle.duplicate_classes(phi)
    _, se = oracle.conceal_video(frames, lost, blocks, phi, T, M, N, 0.8, 0.5, 30, "se", cls)
    _, fa = oracle.conceal_video(frames, lost, blocks, phi, T, M, N, 0.8, 0.5, 30, "fase", cls)
    for (r1, g1), (r3, g3) in zip(se, fa):
        np.testing.assert_array_equal(cls[r1.sel], cls[r3.sel])
        np.testing.assert_allclose(g3, g1, atol=1e-8)


def test_video_model_is_symmetric_under_axis_permutation():
    """With T = M = N the weights are symmetric in the three axes and the
    3-D DCT u WHT dictionary maps onto itself when the axes are permuted, so
    concealing the permuted volume with the permuted loss box gives the
    permuted model.  A wrong temporal centre, or frames mixed up with rows
    in the sample order or the paste, breaks this."""
    T = M = N = 4
    phi = synth.video_dictionary(T, M, N)
    rng = np.random.default_rng(21)
    vol = rng.integers(0, 256, size=(4, 4, 4)).astype(np.uint8)
    box = dict(lt=1, ld=2, ly=2, lh=1, lx=0, lw=3)
    b = synth.Block(0, 0, 0, box["ly"], box["lx"], box["lh"], box["lw"], box["lt"], box["ld"])
    lost = synth.video_lost_mask(4, 4, 4, [b])
    cls = oracle.duplicate_classes(phi)
    _, per = oracle.conceal_video(vol, lost, [b], phi, T, M, N, 0.8, 0.5, 20, "se", cls)
    g = per[0][1]                                   # (ld, lh, lw) = frames x rows x columns
    for perm in ((1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)):
        volp = np.ascontiguousarray(vol.transpose(perm))
        start = (box["lt"], box["ly"], box["lx"])
        size = (box["ld"], box["lh"], box["lw"])
        sp, zp = [start[a] for a in perm], [size[a] for a in perm]
        bp = synth.Block(0, 0, 0, sp[1], sp[2], zp[1], zp[2], sp[0], zp[0])
        lostp = synth.video_lost_mask(4, 4, 4, [bp])
        np.testing.assert_array_equal(lostp, lost.transpose(perm))
        _, perp = oracle.conceal_video(volp, lostp, [bp], phi, T, M, N, 0.8, 0.5, 20, "se", cls)
        np.testing.assert_allclose(perp[0][1], g.transpose(perm), atol=1e-9)


def test_video_dictionary_structure():
    """The generator's 3-D atoms: each half orthonormal, a one-frame
    dictionary equal to the 2-D one, and atom (kt, k1, k2) the product of
    the three 1-D rows."""
    T, M, N = 4, 8, 8
    phi = synth.video_dictionary(T, M, N)
    P = T * M * N
    for h in range(2):
        half = phi[h * P:(h + 1) * P]
        np.testing.assert_allclose(half @ half.T, np.eye(P), atol=1e-12)
    np.testing.assert_array_equal(synth.separable_atoms3(np.ones((1, 1)), synth.dct_rows(8),
                                                         synth.dct_rows(8)),
                                  synth.dct2_atoms(8, 8))
    d4, d8 = synth.dct_rows(4), synth.dct_rows(8)
    kt, k1, k2 = 3, 5, 2
    ref = np.einsum("t,m,n->tmn", d4[kt], d8[k1], d8[k2]).reshape(-1)
    np.testing.assert_allclose(phi[(kt * M + k1) * N + k2], ref, atol=1e-15)
