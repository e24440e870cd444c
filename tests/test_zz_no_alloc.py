"""The allocation-free batched call (se_extrapolate_batch_static) against
se_extrapolate_batch: the same kernels on the same inputs, so every output
(selections, coefficients, model over the loss, pasted image) must be equal
bit for bit.  Two calls in a row on each route, the second with fewer blocks
and other images, so the second call runs on the static scratch the first
one left behind; a batch too large for the scratch is refused on the host."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth

from test_gpu_parity import dev, say, shared_tables, upload_phi

pytestmark = pytest.mark.gpu


def _run(fn, t, images, blocks, iters):
    img = torch.from_numpy(images).to(dev())
    sel, coef, g = fn(t, img, blocks, 0.5, iters)
    torch.cuda.synchronize()
    return [x.cpu() for x in (sel, coef, g, img)]


def _assert_same(a, b, what):
    for name, x, y in zip(("sel", "coef", "g_loss", "image"), a, b):
        assert torch.equal(x, y), f"{what}: {name} differs from se_extrapolate_batch"


@pytest.mark.parametrize("route", ["one_launch", "two_launch"])
def test_static_scratch_equals_batch(route):
    parts = route == "one_launch"
    say(f"se_extrapolate_batch_static vs se_extrapolate_batch: 32x32 areas, K=2048, I=100, "
        f"{route} route, 128 then 48 blocks")
    d1 = synth.area32_inputs(8)
    d2 = synth.area32_inputs(3, seed0=40)
    phi = upload_phi(synth.round_to_f32(d1["phi"]))
    t, _, _ = shared_tables(d1["images"], d1["blocks"], phi, 32, 32, 0.8,
                            parts=d1["tx_parts"] if parts else ())
    assert (t.n_classes == 4) == parts
    for d in (d1, d2):
        ref = _run(B.extrapolate_batch, t, d["images"], d["blocks"], 100)
        got = _run(B.extrapolate_batch_static, t, d["images"], d["blocks"], 100)
        _assert_same(ref, got, f"{route}, {len(d['blocks'])} blocks")
    print(f"static scratch {route}: 128 and 48 blocks bit-identical to the workspace call")


def test_static_scratch_refuses_oversized_batch():
    # two-launch route, K = 2048: each block needs a row of R (8 KiB) and its
    # gathered area (4 KiB), so 2048 blocks exceed 16 MiB
    say("se_extrapolate_batch_static: 2048 blocks on the two-launch route are refused")
    d = synth.area32_inputs(1)
    phi = upload_phi(synth.round_to_f32(d["phi"]))
    t, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8)
    img = torch.from_numpy(np.zeros((128, 128, 128), np.uint8)).to(dev())
    blocks = [synth.Block(i // 16, 32 * ((i // 4) % 4), 32 * (i % 4), 12, 12, 8, 8)
              for i in range(2048)]
    L = B.lib()
    st = t.struct()
    r = L.se_extrapolate_batch_static(C.byref(st), B._ptr(img), 128, 128, 128,
                                      B.blocks_array(blocks), len(blocks),
                                      B.se_params(0.5, 100, 0), None, None, None, 0,
                                      B._stream())
    assert r == B.SE_ENOMEM
    assert b"static scratch" in L.se_last_error()
