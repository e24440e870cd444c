"""GPU tests of the serving loop (se_serve_*): results against the FP64
oracle, the same result alone and in a mix of concurrent requests, the HBM
budget forcing the on-demand path, queue limits and argument errors."""
import sys
import time

import numpy as np
import pytest
import torch

from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth


pytestmark = pytest.mark.gpu

H, W = 192, 256


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def bases(with64=True):
    b = [(synth.round_to_f32(synth.dictionary(32, 32, ("dct", "wht"))), 32, 32),
         (synth.round_to_f32(synth.dictionary(48, 48, ("dct", "gauss"), seed=101, n_gauss=1792)),
          48, 48)]
    if with64:
        b.append((synth.round_to_f32(synth.dictionary(64, 64, ("dct", "wht"))), 64, 64))
    return b


# the transform ranges of the dictionaries above (DCT first, then WHT or
# Gaussian atoms)
PARTS = {32: [("dct", 0), ("wht", 1024)], 48: [("dct", 0)], 64: [("dct", 0), ("wht", 4096)]}


def to_dev(bs, with_parts=False):
    return [(torch.from_numpy(p.astype(np.float32)).cuda(), M, N,
             PARTS[M] if with_parts else ()) for p, M, N in bs]


def losses_for(seed, coverage=0.03, with64=True):
    L = synth.frame_losses(H, W, coverage, seed, p64=0.5 if with64 else 0.0)
    return L


def blocks_of(losses, bs):
    out = []
    for (y, x, h, w, k) in losses:
        M, N = bs[k][1], bs[k][2]
        ly, lx = (M - h) // 2, (N - w) // 2
        out.append(synth.Block(0, y - ly, x - lx, ly, lx, h, w))
    return out


def check_frame(img, out, losses, bs, iters, tol=1e-3, per_basis=2):
    """The pasted pixels of a few blocks of each dictionary equal the rounded
    FP64 oracle model (except where that model lies within ``tol`` of a
    rounding boundary)."""
    import oracle
    all_blocks = blocks_of(losses, bs)
    lost = synth.lost_mask(H, W, all_blocks)
    for k in range(len(bs)):
        idx = [i for i, l in enumerate(losses) if l[4] == k][:per_basis]
        if not idx:
            continue
        phi, M, N = bs[k]
        cls = oracle.duplicate_classes(phi)
        sub = [all_blocks[i] for i in idx]
        _, per = oracle.conceal(img, lost, sub, phi, M, N, 0.8, 0.5, iters, classes=cls,
                                table_cache={})
        for b, (res, gref) in zip(sub, per):
            y, x = b.y0 + b.ly, b.x0 + b.lx
            got = out[y:y + b.lh, x:x + b.lw].astype(np.float64)
            near = np.abs(np.abs(gref - np.floor(gref)) - 0.5) < tol
            q = np.clip(np.rint(gref), 0, 255)
            assert ((got == q) | near).all(), f"dictionary {k}, block {b}"


@pytest.mark.parametrize("with_parts", [False, True])
def test_serve_single_frame_against_oracle(with_parts):
    say(f"serve: one 192x256 frame, 3 dictionaries, I=40, transform parts {with_parts}")
    bs = bases()
    srv = B.Server(to_dev(bs, with_parts), H, W, max_slots=2, max_queue=4, n_streams=2)
    img = synth.synth_image(H, W, seed=11)
    losses = losses_for(3)
    fr = torch.from_numpy(img.copy()).cuda()
    t = srv.submit(fr, losses, 0.5, 40)
    res = srv.wait(t)
    assert res.status == 0 and res.n_blocks == len(losses)
    assert res.n_isolated > 0 and res.n_ondemand > 0
    assert res.t_submit_ns <= res.t_admit_ns <= res.t_done_ns
    out = fr.cpu().numpy()
    mask = synth.lost_mask(H, W, blocks_of(losses, bs)).astype(bool)
    np.testing.assert_array_equal(out[~mask], img[~mask])
    check_frame(img, out, losses, bs, 40)
    st = srv.stats()
    assert st["completed"] == 1 and st["table_builds"] >= 1
    srv.close()


@pytest.mark.parametrize("with_parts", [False, True])
def test_serve_alone_equals_in_mix(with_parts):
    say(f"serve: the same frame alone and among 5 concurrent frames, parts {with_parts}")
    bs = bases()
    srv = B.Server(to_dev(bs, with_parts), H, W, max_slots=4, max_queue=16, n_streams=3)
    imgs = [synth.synth_image(H, W, seed=20 + i) for i in range(6)]
    losses = [losses_for(40 + i) for i in range(6)]
    a = torch.from_numpy(imgs[0].copy()).cuda()
    srv.wait(srv.submit(a, losses[0], 0.5, 60))
    alone = a.cpu().numpy()
    frames = [torch.from_numpy(im.copy()).cuda() for im in imgs]
    tickets = [srv.submit(f, L, 0.5, 60) for f, L in zip(frames, losses)]
    for t in tickets:
        assert srv.wait(t).status == 0
    np.testing.assert_array_equal(frames[0].cpu().numpy(), alone)
    # and every frame equals its own run alone
    for i in (3, 5):
        f = torch.from_numpy(imgs[i].copy()).cuda()
        srv.wait(srv.submit(f, losses[i], 0.5, 60))
        np.testing.assert_array_equal(frames[i].cpu().numpy(), f.cpu().numpy())
    st = srv.stats()
    assert st["table_hits"] > 0
    srv.close()


@pytest.mark.parametrize("with_parts", [False, True])
def test_serve_budget_degrades_to_ondemand(with_parts):
    say(f"serve: HBM budget too small for the 48x48 tables, parts {with_parts}")
    bs = bases(with64=False)
    losses = losses_for(7, with64=False)
    img = synth.synth_image(H, W, seed=5)
    srv = B.Server(to_dev(bs, with_parts), H, W, max_slots=1, max_queue=2, n_streams=1,
                   hbm_budget_bytes=110 << 20)
    fr = torch.from_numpy(img.copy()).cuda()
    res = srv.wait(srv.submit(fr, losses, 0.5, 40))
    assert res.status == 0
    st = srv.stats()
    assert st["degraded_blocks"] > 0
    assert st["bytes_tables"] + st["bytes_slots"] + st["bytes_scratch"] <= 110 << 20
    check_frame(img, fr.cpu().numpy(), losses, bs, 40)
    srv.close()


def test_serve_queue_limit_and_errors():
    say("serve: queue full, bad requests, unknown ticket")
    bs = bases(with64=False)
    srv = B.Server(to_dev(bs), H, W, max_slots=1, max_queue=2, n_streams=1)
    img = synth.synth_image(H, W, seed=9)
    losses = losses_for(9, coverage=0.08, with64=False)
    frames = [torch.from_numpy(img.copy()).cuda() for _ in range(12)]
    tickets, busy = [], 0
    for f in frames:
        try:
            tickets.append(srv.submit(f, losses, 0.5, 100))
        except B.SEError as e:
            assert e.code == B.SE_EBUSY
            busy += 1
    assert busy > 0
    for t in tickets:
        assert srv.wait(t).status == 0
    f = frames[0]
    with pytest.raises(B.SEError) as e:
        srv.submit(f, [(0, 0, 8, 8, 7)], 0.5, 10)            # unknown dictionary
    assert e.value.code == B.SE_EINVAL
    with pytest.raises(B.SEError):
        srv.submit(f, [(H - 4, 0, 8, 8, 0)], 0.5, 10)        # leaves the frame
    with pytest.raises(B.SEError):
        srv.submit(f, [(0, 0, 8, 8, 0), (4, 4, 8, 8, 0)], 0.5, 10)   # overlap
    with pytest.raises(B.SEError):
        srv.submit(torch.zeros((H, W + 8), dtype=torch.uint8, device="cuda"), [], 0.5, 10)
    with pytest.raises(B.SEError):
        srv.poll(123456789)
    srv.close()


def test_serve_full_hd_frames():
    """The serving workload's frame size: 1920x1080 frames with 8x8 and 16x16
    losses covering 5% of the frame (areas 32, 48, 64).  Each of two frames
    is the same alone and among others, bit for bit.  The served frame equals,
    bit for bit, the direct library calls on its blocks with SE_INVARIANT
    (the blocks of an isolated pattern with that pattern's tables, the others
    with rows on demand), and those calls' selections and models are held to
    the FP64 oracle on 16 sampled blocks per dictionary (half of each kind
    where the frame has them), with the window derived from the arithmetic."""
    from helpers import describe, oracle_check
    FH, FW = 1080, 1920
    say("serve: 1920x1080 frames, 5% lost, 3 dictionaries, I=100")
    bs = bases()
    dev_bases = to_dev(bs, True)
    srv = B.Server(dev_bases, FH, FW, max_slots=3, max_queue=8, n_streams=3,
                   hbm_budget_bytes=6 << 30)
    imgs = [synth.synth_image(FH, FW, seed=70 + i) for i in range(3)]
    losses = [synth.frame_losses(FH, FW, 0.05, 80 + i) for i in range(3)]
    frames = [torch.from_numpy(im.copy()).cuda() for im in imgs]
    tickets = [srv.submit(f, L, 0.5, 100) for f, L in zip(frames, losses)]
    for t in tickets:
        assert srv.wait(t).status == 0
    outs = [f.cpu().numpy() for f in frames]
    for i in (0, 2):
        f = torch.from_numpy(imgs[i].copy()).cuda()
        assert srv.wait(srv.submit(f, losses[i], 0.5, 100)).status == 0
        np.testing.assert_array_equal(f.cpu().numpy(), outs[i])
    srv.close()
    # frame 0: the direct calls on its blocks, then the oracle
    img, out, L = imgs[0], outs[0], losses[0]
    blocks = [(synth.Block(0, y - (bs[k][1] - h) // 2, x - (bs[k][2] - w) // 2,
                           (bs[k][1] - h) // 2, (bs[k][2] - w) // 2, h, w), k)
              for (y, x, h, w, k) in L]
    lost = synth.lost_mask(FH, FW, [b for b, _ in blocks])
    lost_d = torch.from_numpy(lost[None]).cuda()
    rng = np.random.default_rng(5)
    for k in range(len(bs)):
        phi, M, N = bs[k]
        phi_d, _, _, parts = dev_bases[k]
        mine = [b for b, kk in blocks if kk == k]
        inside = [b.y0 >= 0 and b.x0 >= 0 and b.y0 + M <= FH and b.x0 + N <= FW and
                  lost[b.y0:b.y0 + M, b.x0:b.x0 + N].sum() == b.lh * b.lw for b in mine]
        iso = [b for b, f in zip(mine, inside) if f]
        own = [b for b, f in zip(mine, inside) if not f]
        checked = 0
        if iso:
            w = B.area_weights(M, N, 0.8, lost_d, iso[:1])
            t = B.weighted_gram(phi_d, w[0].contiguous(), M, N, parts=parts)
            img_d = torch.from_numpy(img[None].copy()).cuda()
            sel, coef, g = B.extrapolate_batch(t, img_d, iso, 0.5, 100, invariant=True)
            torch.cuda.synchronize()
            sel, coef, g, o = (x.cpu().numpy() for x in (sel, coef, g, img_d))
            for b in iso:
                y, x = b.y0 + b.ly, b.x0 + b.lx
                np.testing.assert_array_equal(out[y:y + b.lh, x:x + b.lw],
                                              o[0, y:y + b.lh, x:x + b.lw])
            n = min(len(iso), 16 if not own else 8)
            sample = sorted(rng.choice(len(iso), n, replace=False))
            st = oracle_check(img[None], iso, phi, M, N, 0.8, 0.5, 100, sel, g, o, sample=sample,
                              tol=1e-3, coef=coef, tables=t, lost=lost[None])
            print(f"dictionary {k} ({M}x{N}), isolated pattern: {len(iso)} blocks, "
                  f"{describe(st)}")
            checked += n
            del t
        if own:
            w = B.area_weights(M, N, 0.8, lost_d, own)
            img_d = torch.from_numpy(img[None].copy()).cuda()
            sel, coef, g = B.extrapolate_ondemand(phi_d, M, N, w, img_d, own, 0.5, 100,
                                                  parts=parts, invariant=True)
            torch.cuda.synchronize()
            sel, coef, g, o = (x.cpu().numpy() for x in (sel, coef, g, img_d))
            for b in own:
                y, x = b.y0 + b.ly, b.x0 + b.lx
                np.testing.assert_array_equal(out[y:y + b.lh, x:x + b.lw],
                                              o[0, y:y + b.lh, x:x + b.lw])
            n = min(len(own), 16 - checked)
            sample = sorted(rng.choice(len(own), n, replace=False))
            st = oracle_check(img[None], own, phi, M, N, 0.8, 0.5, 100, sel, g, o, sample=sample,
                              tol=1e-3, lost=lost[None])
            print(f"dictionary {k} ({M}x{N}), own weights: {len(own)} blocks, {describe(st)}")
            checked += n
        assert checked >= 16
