"""Rows on demand through a prepared dictionary and a plan: the same results
as se_extrapolate_ondemand, whatever the number of cached table rows per
block, in eager runs and in replays of a captured HIP graph; the row-product
tuner's choice held to the oracle.

Workload: blocks of the clustered/burst frames (other losses and the frame
border inside the areas, so every block has its own weights), per-block
iteration counts I ~ U{100..200}, the dictionaries of those frames (DCT u
Gaussian for 24x24 and 48x48, DCT u WHT for 32x32)."""
import sys

import numpy as np
import pytest
import torch

from helpers import describe, oracle_check
from paper_2204_14194_amd import binding as B
from paper_2204_14194_amd import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-3   # max |g - g_oracle| on the 0..255 scale, as for the other FP32 paths


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev():
    return torch.device("cuda:0")


_DATA = {}


def clustered(area, n_max=None):
    """Blocks of one area size from one clustered frame, their iteration
    counts, the frame, its loss mask, the weights and the dictionary."""
    key = (area, n_max)
    if key not in _DATA:
        d = synth.clustered_inputs(n_img=1, blocks_per_img=500)
        idx = [i for i, b in enumerate(d["blocks"]) if b.ly * 2 + b.lh == area]
        if n_max is not None:
            idx = idx[:n_max]
        blocks = [d["blocks"][i] for i in idx]
        iters = [int(d["iters"][i]) for i in idx]
        lost = synth.lost_mask(1024, 1024, d["blocks"])[None]
        phi = synth.round_to_f32(d["dicts"][area])
        _DATA[key] = dict(blocks=blocks, iters=iters, img=d["images"][:1], lost=lost, phi=phi,
                          parts=d["tx_parts"][area])
    c = _DATA[key]
    w = B.area_weights(area, area, 0.8, torch.from_numpy(c["lost"]).to(dev()), c["blocks"])
    phi_d = torch.from_numpy(c["phi"].astype(np.float32)).to(dev())
    return c, w, phi_d


def run_plan(plan, w, img0):
    img = img0.clone()
    sel, coef, g = plan.outputs(dev())
    try:
        plan.run(w, img, sel, coef, g)
    except B.SENumericError:
        pass
    torch.cuda.synchronize()
    return sel.cpu().numpy(), coef.cpu().numpy(), g.cpu().numpy(), img.cpu().numpy()


def assert_same(a, b, what, iters=None):
    """Bitwise equality of (sel, coef, g_loss, images); with ``iters`` only the
    entries of sel and coef below each block's own iteration count (the rest
    is left unwritten)."""
    for x, y, name in zip(a, b, ("sel", "coef", "g_loss", "images")):
        if iters is not None and name in ("sel", "coef"):
            for i, it in enumerate(iters):
                assert np.array_equal(x[i, :it], y[i, :it]), f"{what}: {name} differs (block {i})"
        else:
            assert np.array_equal(x, y), f"{what}: {name} differs"


@pytest.mark.parametrize("area,with_parts", [(24, True), (32, False), (48, True)])
def test_plan_equals_call_for_any_row_cache(area, with_parts):
    """A plan's run equals se_extrapolate_ondemand bit for bit (the same
    kernels and product shapes) with no cached rows, with a few cached rows
    per block (new atoms past them formed on every use) and with every row
    cached: a cached row holds the values the product forms again."""
    c, w, phi_d = clustered(area, 96)
    parts = c["parts"] if with_parts else ()
    say(f"plan vs call: area {area}, parts {with_parts}, {len(c['blocks'])} blocks")
    img0 = torch.from_numpy(c["img"]).to(dev())
    img = img0.clone()
    ref = B.extrapolate_ondemand(phi_d, area, area, w, img, c["blocks"], 0.5, c["iters"],
                                 parts=parts)
    torch.cuda.synchronize()
    ref = tuple(x.cpu().numpy() for x in ref) + (img.cpu().numpy(),)
    d = B.OnDemandDict(phi_d, area, area, parts=parts)
    # the one-call form on the prepared dictionary, without and with cached rows
    for slots in (0, 200):
        img = img0.clone()
        got = B.OnDemandDict.extrapolate(d, w, img, c["blocks"], 0.5, c["iters"],
                                         row_slots=slots)
        torch.cuda.synchronize()
        assert_same(tuple(x.cpu().numpy() for x in got) + (img.cpu().numpy(),), ref,
                    f"se_ondemand_extrapolate, row_slots={slots}", c["iters"])
    for slots in (0, 3, None):
        plan = B.OnDemandPlan(d, img0, c["blocks"], 0.5, c["iters"], row_slots=slots)
        got = run_plan(plan, w, img0)
        assert_same(got, ref, f"row_slots={slots}", c["iters"])
        plan.close()
    d.close()


def test_plan_bf16x3_rows_equal_call():
    """The same with split-BF16 row products (SE_ROWS_BF16X3): the
    dictionary's split copy is formed once by the preparation."""
    area = 48
    c, w, phi_d = clustered(area, 64)
    say(f"plan vs call, split-BF16 rows: area {area}, {len(c['blocks'])} blocks")
    img0 = torch.from_numpy(c["img"]).to(dev())
    img = img0.clone()
    ref = B.extrapolate_ondemand(phi_d, area, area, w, img, c["blocks"], 0.5, c["iters"],
                                 parts=c["parts"], rows_bf16=True)
    torch.cuda.synchronize()
    ref = tuple(x.cpu().numpy() for x in ref) + (img.cpu().numpy(),)
    d = B.OnDemandDict(phi_d, area, area, parts=c["parts"], rows_bf16=True)
    plan = B.OnDemandPlan(d, img0, c["blocks"], 0.5, c["iters"], rows_bf16=True)
    assert_same(run_plan(plan, w, img0), ref, "split-BF16 rows, every row cached", c["iters"])
    with pytest.raises(B.SEError):   # a plan with split rows needs a dictionary prepared for them
        B.OnDemandPlan(B.OnDemandDict(phi_d, area, area, parts=c["parts"]), img0, c["blocks"],
                       0.5, c["iters"], rows_bf16=True)


def test_row_cache_against_oracle():
    """Every row cached, area 48 with parts: a sample of blocks against the
    FP64 oracle (derived FP32 window, as for the call)."""
    area = 48
    c, w, phi_d = clustered(area)
    say(f"row cache vs oracle: area {area}, {len(c['blocks'])} blocks")
    img0 = torch.from_numpy(c["img"]).to(dev())
    d = B.OnDemandDict(phi_d, area, area, parts=c["parts"])
    plan = B.OnDemandPlan(d, img0, c["blocks"], 0.5, c["iters"])
    sel, coef, g, out = run_plan(plan, w, img0)
    rng = np.random.default_rng(7)
    sample = sorted(rng.choice(len(c["blocks"]), 16, replace=False))
    st = oracle_check(c["img"], c["blocks"], c["phi"], area, area, 0.8, 0.5, c["iters"], sel, g,
                      out, sample=sample, tol=TOL_FP32, lost=c["lost"])
    print(f"row cache area {area}: {describe(st)}")


def _graph_of(fn, stream):
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        fn()
    return g


def test_graph_replay_equals_eager():
    """A run captured in a HIP graph: every replay (with other eager work and
    synchronisations between them, the images restored before each) equals
    the eager run bit for bit."""
    area = 32
    c, w, phi_d = clustered(area, 128)
    say(f"graph replay of a run: area {area}, {len(c['blocks'])} blocks, every row cached")
    img0 = torch.from_numpy(c["img"]).to(dev())
    d = B.OnDemandDict(phi_d, area, area, parts=c["parts"])
    plan = B.OnDemandPlan(d, img0, c["blocks"], 0.5, c["iters"])
    eager = run_plan(plan, w, img0)
    img = img0.clone()
    sel, coef, g = plan.outputs(dev())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = _graph_of(lambda: _run_quiet(plan, w, img, sel, coef, g, s), s)
    for rep in range(3):
        img.copy_(img0)
        sel.fill_(-7)
        coef.fill_(1e9)
        g.zero_()    # entries past a block's loss are not written (zero, as in the eager run)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = (sel.cpu().numpy(), coef.cpu().numpy(), g.cpu().numpy(), img.cpu().numpy())
        assert_same(got, eager, f"replay {rep}", c["iters"])
        _ = (torch.ones(1000, device=dev()) * 2).sum().item()   # eager work between replays


def _run_quiet(plan, w, img, sel, coef, g, stream):
    try:
        plan.run(w, img, sel, coef, g, stream=stream)
    except B.SENumericError:
        pass


def test_graph_of_three_area_groups():
    """The three area groups of the clustered frames on three streams,
    forked and joined inside one capture: each replay equals the eager runs
    bit for bit."""
    say("graph of three area groups (24, 32, 48) on three streams")
    groups = []
    for area in (24, 32, 48):
        c, w, phi_d = clustered(area, 64)
        d = B.OnDemandDict(phi_d, area, area, parts=c["parts"])
        img0 = torch.from_numpy(c["img"]).to(dev())
        plan = B.OnDemandPlan(d, img0, c["blocks"], 0.5, c["iters"])
        groups.append((area, d, plan, w, img0, run_plan(plan, w, img0), c["iters"]))
    # one image per group (their losses overlap between groups of a frame)
    imgs = [gr[4].clone() for gr in groups]
    outs = [gr[2].outputs(dev()) for gr in groups]
    streams = [torch.cuda.Stream() for _ in groups]
    main = torch.cuda.Stream()
    main.wait_stream(torch.cuda.current_stream())

    def body():
        for (area, d, plan, w, img0, _, _), img, (sel, coef, g), st in zip(groups, imgs, outs,
                                                                            streams):
            st.wait_stream(main)
            _run_quiet(plan, w, img, sel, coef, g, st)
        for st in streams:
            main.wait_stream(st)

    graph = _graph_of(body, main)
    for rep in range(2):
        for img, gr in zip(imgs, groups):
            img.copy_(gr[4])
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for gr, img, (sel, coef, g) in zip(groups, imgs, outs):
            got = (sel.cpu().numpy(), coef.cpu().numpy(), g.cpu().numpy(), img.cpu().numpy())
            assert_same(got, gr[5], f"replay {rep}, area {gr[0]}", gr[6])


def test_autotuned_row_products_against_oracle():
    """The tuner times the row products' tile and split on a plan, records
    the fastest (exported as a "rows" line) and sets it; the tuned plan's
    results stay within the FP32 window of the oracle (a split changes the
    order of the sums)."""
    area = 24
    c, w, phi_d = clustered(area)
    say(f"row-product tuner: area {area}, {len(c['blocks'])} blocks")
    B.tune_clear()
    img0 = torch.from_numpy(c["img"]).to(dev())
    d = B.OnDemandDict(phi_d, area, area, parts=c["parts"])
    plan = B.OnDemandPlan(d, img0, c["blocks"], 0.5, c["iters"])
    img = img0.clone()
    tile, split, ms = plan.autotune(w, img, reps=1)
    print(f"tuned: tile {tile}, split {split}, {ms:.3f} ms per run")
    assert tile in (0, 64, 128, 12864) and split in (-1, 1, 2, 4, 8)
    buf = B.tune_export()
    assert any(line.startswith("rows ") for line in buf.splitlines())
    sel, coef, g, out = run_plan(plan, w, img0)
    rng = np.random.default_rng(11)
    sample = sorted(rng.choice(len(c["blocks"]), 16, replace=False))
    st = oracle_check(c["img"], c["blocks"], c["phi"], area, area, 0.8, 0.5, c["iters"], sel, g,
                      out, sample=sample, tol=TOL_FP32, lost=c["lost"])
    print(f"tuned rows area {area}: {describe(st)}")
    # a later plan of the same shape picks the record up: same results
    plan2 = B.OnDemandPlan(d, img0, c["blocks"], 0.5, c["iters"])
    assert_same(run_plan(plan2, w, img0), (sel, coef, g, out), "second plan", c["iters"])
    B.tune_clear()
