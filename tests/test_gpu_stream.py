"""The asynchronous, streamed form of omniseg_segment_slide.

The kept-tile count stays on the device: backbone batches are launched for
every grid tile and skip list positions past the count, each batch is
followed by the stitch of the tile rows it completed, and the tile logits
may live in a ring.  These tests pin that form against the plain one:

* several uneven slides through a minimal ring, with small batches so the
  ring wraps many times, equal one resident-store call per slide bit for bit
  (ramp and vote merges, per-scale strides, tissue-gated masks);
* one HIP graph of the whole call, replayed after the slides' pixels change
  (a different tile list and kept count), equals the eager call on the new
  pixels;
* the call returns while the stream is still busy (no host wait);
* profiled calls make the same launches and their records count exactly the
  kept tiles.
"""

import time

import numpy as np
import pytest
import torch

import synth
from oracle import omniseg_oracle as O
from paper_2305_14566_amd import omniseg as om

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _slides():
    a, _ = synth.strip_slide(31, 300, 517, fg_frac=0.25)
    b, _ = synth.strip_slide(32, 129, 64, fg_frac=0.5)
    c, _ = synth.strip_slide(33, 640, 200, fg_frac=0.15)
    d, _ = synth.strip_slide(34, 96, 700, fg_frac=0.6)
    return [a, b, c, d]


def _plan(precision, merge, batch_tiles, ring, graph=False, emit=True):
    kw = {}
    if merge == om.MERGE_VOTE:
        kw = dict(scale_strides=(32, 16, 8, 16), vote_thresholds=(1, 2, 4, 3))
    return om.Plan(base=8, levels=3, head_out=2, n_classes=3, scales=(0, 1, 2, 3), tile=64, stride=32,
                   fg_filter=True, mask_and_fg=True, precision=precision, emit_logits=emit,
                   batch_tiles=batch_tiles, logit_ring_tiles=ring, graph=graph, merge=merge, **kw)


PAIRS = [(0, 0), (2, 1), (1, 2), (0, 3), (1, 0), (2, 3)]


def _flat():
    return synth.he_normal_weights(41, 8, 3, 3, 4, 2, bias_std=0.05)


@pytest.mark.parametrize("merge", [om.MERGE_RAMP, om.MERGE_VOTE])
@pytest.mark.parametrize("precision", [om.FP32, om.BF16])
def test_ring_store_equals_resident_per_slide(precision, merge):
    slides = _slides()
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    flat = torch.from_numpy(_flat()).to(DEV)
    ring_plan = _plan(precision, merge, batch_tiles=5, ring=1)
    packed = ring_plan.pack(flat)
    masks, logits, ws = ring_plan.segment(ds, PAIRS, packed)
    torch.cuda.synchronize()
    off, nb = ring_plan.region(ds, PAIRS, om.REGION_TILE_LOGITS)
    slots = nb // (2 * 64 * 64 * 4)  # at most two pairs share a scale slot
    off, _ = ring_plan.region(ds, PAIRS, om.REGION_TILE_COUNT)
    kept = int(ws[off:off + 4].view(torch.int32).item())
    assert slots < kept, (slots, kept)  # the ring really wraps
    for i, s in enumerate(ds):
        res_plan = _plan(precision, merge, batch_tiles=64, ring=0)
        m1, l1, _ = res_plan.segment([s], PAIRS, res_plan.pack(flat))
        torch.cuda.synchronize()
        for p in range(len(PAIRS)):
            assert torch.equal(masks[i][p], m1[0][p]), (i, p)
            assert torch.equal(logits[i][p], l1[0][p]), (i, p)


def test_ring_store_matches_oracle_stitch():
    """The ring-store call against the FP64 oracle's stitch of the same
    call's tile logits, read from a resident-store call (the tile logits
    are the same: the backbone does not depend on the store)."""
    slides = _slides()[:2]
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    flat = torch.from_numpy(_flat()).to(DEV)
    ring_plan = _plan(om.FP32, om.MERGE_RAMP, batch_tiles=3, ring=1)
    masks, logits, _ = ring_plan.segment(ds, PAIRS, ring_plan.pack(flat))
    res_plan = _plan(om.FP32, om.MERGE_RAMP, batch_tiles=3, ring=0)
    _, _, ws = res_plan.segment(ds, PAIRS, res_plan.pack(flat))
    torch.cuda.synchronize()
    off, nb = res_plan.region(ds, PAIRS, om.REGION_TILE_LOGITS)
    tl = ws[off:off + nb].view(torch.float32).reshape(-1, 2, 64, 64).cpu().numpy().astype(np.float64)
    off, _ = res_plan.region(ds, PAIRS, om.REGION_TILE_COUNT)
    kept = int(ws[off:off + 4].view(torch.int32).item())
    off, nb = res_plan.region(ds, PAIRS, om.REGION_TILE_LIST)
    lst = ws[off:off + nb].view(torch.int32).reshape(-1, 4)[:kept].cpu().numpy()
    for i, rgb in enumerate(slides):
        for p, (c, si) in enumerate(PAIRS):
            slot = [q for q in PAIRS if q[1] == si].index((c, si))
            k = (0, 1, 2, 3)[si]
            Hk, Wk = O.level_size(rgb.shape[0], k), O.level_size(rgb.shape[1], k)
            sel = [t for t in range(kept) if lst[t, 0] == i and lst[t, 1] == si]
            yx = [(int(lst[t, 2]), int(lst[t, 3])) for t in sel]
            lam, _, _ = O.stitch(yx, [tl[t, slot] for t in sel], Hk, Wk, 64, 32)
            got = logits[i][p].cpu().numpy().astype(np.float64)
            scale = max(1.0, np.abs(lam).max())
            assert np.abs(got - lam).max() <= 1e-5 * scale, (i, p)


def test_whole_call_graph_follows_new_pixels():
    """The graph holds the tile list too: after the slides' pixels change in
    place (another tissue layout, another kept count), a replay equals an
    eager call on the new pixels."""
    a = _slides()
    b = [synth.strip_slide(40 + i, s.shape[0], s.shape[1], fg_frac=0.6)[0] for i, s in enumerate(a)]
    flat = torch.from_numpy(_flat()).to(DEV)
    gplan = _plan(om.BF16, om.MERGE_RAMP, batch_tiles=8, ring=1, graph=True)
    packed = gplan.pack(flat)
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in a]
    ws = torch.empty(gplan.workspace_bytes(ds, PAIRS), dtype=torch.uint8, device=DEV)
    outs = gplan.alloc_outputs(ds, PAIRS)
    side = torch.cuda.Stream()
    counts = []
    for rep, content in enumerate([a, b, a, b]):
        for t, s in zip(ds, content):
            t.copy_(torch.from_numpy(np.ascontiguousarray(s)))
        for row in outs[0] + outs[1]:
            for t in row:
                t.fill_(7)
        torch.cuda.synchronize()
        masks, logits, _ = gplan.segment(ds, PAIRS, packed, workspace=ws, outputs=outs, stream=side)
        side.synchronize()
        off, _ = gplan.region(ds, PAIRS, om.REGION_TILE_COUNT)
        counts.append(int(ws[off:off + 4].view(torch.int32).item()))
        eplan = _plan(om.BF16, om.MERGE_RAMP, batch_tiles=8, ring=0)
        me, le, _ = eplan.segment([t.clone() for t in ds], PAIRS, eplan.pack(flat))
        torch.cuda.synchronize()
        for i in range(len(ds)):
            for p in range(len(PAIRS)):
                assert torch.equal(masks[i][p], me[i][p]), (rep, i, p)
                assert torch.equal(logits[i][p], le[i][p]), (rep, i, p)
    assert counts[0] == counts[2] and counts[1] == counts[3] and counts[0] != counts[1], counts


def test_call_returns_before_the_stream_completes():
    slides = _slides()
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    plan = _plan(om.BF16, om.MERGE_RAMP, batch_tiles=8, ring=1)
    packed = plan.pack(torch.from_numpy(_flat()).to(DEV))
    ws = torch.empty(plan.workspace_bytes(ds, PAIRS), dtype=torch.uint8, device=DEV)
    outs = plan.alloc_outputs(ds, PAIRS)
    plan.segment(ds, PAIRS, packed, workspace=ws, outputs=outs)  # loads the code objects
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    torch.cuda._sleep(int(2.0e9))  # roughly a second of spinning ahead of the call on the same stream
    t0 = time.perf_counter()
    plan.segment(ds, PAIRS, packed, workspace=ws, outputs=outs)
    host_s = time.perf_counter() - t0
    busy = not stream.query()
    torch.cuda.synchronize()
    assert busy and host_s < 0.25, (busy, host_s)


def test_profiled_records_count_kept_tiles():
    slides = _slides()
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    plan = _plan(om.FP32, om.MERGE_RAMP, batch_tiles=6, ring=1)
    packed = plan.pack(torch.from_numpy(_flat()).to(DEV))
    ws = torch.empty(plan.workspace_bytes(ds, PAIRS), dtype=torch.uint8, device=DEV)
    outs = plan.alloc_outputs(ds, PAIRS)
    plain = plan.segment(ds, PAIRS, packed, workspace=ws, outputs=outs)
    ref_m = [[m.clone() for m in row] for row in plain[0]]
    plan.set_profiling(True)
    plan.segment(ds, PAIRS, packed, workspace=ws, outputs=outs)
    recs = plan.read_profile()
    plan.set_profiling(False)
    off, _ = plan.region(ds, PAIRS, om.REGION_TILE_COUNT)
    kept = int(ws[off:off + 4].view(torch.int32).item())
    first = [r for r in recs if r["stage"] == "first_conv"]
    stitch = [r for r in recs if r["stage"] == "stitch"]
    total_grid = sum(
        O.grid_count(O.level_size(s.shape[0], k), 64, 32) * O.grid_count(O.level_size(s.shape[1], k), 64, 32)
        for s in slides for k in (0, 1, 2, 3))
    assert len(first) == len(stitch) == -(-total_grid // 6)
    assert sum(r["tiles"] for r in first) == kept
    assert all(r["bytes"] > 0 for r in stitch[:1])
    for i in range(len(ds)):
        for p in range(len(PAIRS)):
            assert torch.equal(outs[0][i][p], ref_m[i][p])
