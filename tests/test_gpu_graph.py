"""A whole step (initial projections + iteration loop + paste) captured into
a HIP graph and replayed: every replay must reproduce the eager step bit for
bit.  Between replays the program runs eager work of its own and
synchronises, and the outputs are cleared by torch fill kernels (no memset
nodes are recorded)."""
import numpy as np
import pytest
import torch

from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth

from test_gpu_parity import dev, say, shared_tables, upload_phi

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("with_parts", [True, False])
def test_graph_step_replays_match_eager(with_parts):
    d = synth.area32_inputs(8)
    say(f"graph capture of one step: 128 blocks, K=2048, I=100, parts={with_parts}")
    phi = upload_phi(synth.round_to_f32(d["phi"]))
    t, _, _ = shared_tables(d["images"], d["blocks"], phi, 32, 32, 0.8,
                            parts=d["tx_parts"] if with_parts else ())
    blocks = d["blocks"]
    n = len(blocks)
    img0 = torch.from_numpy(d["images"]).to(dev())
    img = img0.clone()
    db = B.DeviceBlocks(t, img, blocks)
    R = torch.empty((n, t.ldG), dtype=torch.float32, device=dev())
    ws = torch.empty(max(1, B.project_ws_bytes(t, n)), dtype=torch.uint8, device=dev())
    sel = torch.zeros((n, 100), dtype=torch.int32, device=dev())
    coef = torch.zeros((n, 100), dtype=torch.float32, device=dev())
    g = torch.zeros((n, 64), dtype=torch.float32, device=dev())

    def step(stream=None):
        B.project(t, img, db, R, ws, stream=stream)
        B.iterate(t, R, img, db, 0.5, 100, sel, coef, g, stream=stream)

    # eager reference
    step()
    torch.cuda.synchronize()
    ref = [x.clone() for x in (sel, coef, g, img)]

    # capture on a side stream (torch's capture protocol), then replay
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(side)                                    # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=side):
        step(side)
    torch.cuda.synchronize()

    other = torch.empty_like(R)
    for rep in range(3):
        for x in (sel, coef, g):
            x.zero_()
        img.copy_(img0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for name, x, r in zip(("sel", "coef", "g", "image"), (sel, coef, g, img), ref):
            assert torch.equal(x, r), f"replay {rep}: {name} differs from the eager step"
        # eager work of the program between replays
        B.project(t, img, db, other, ws)
        torch.cuda.synchronize()
    assert np.isfinite(coef.cpu().numpy()).all()
