"""omniseg_stitch_tiles_noalloc: the stand-alone stitch for callers that
cannot allocate device memory, against omniseg_stitch_tiles (the same
arithmetic with a caller workspace).  Outputs must be bit-identical, on
consecutive calls where the second grid is smaller than the first (the
library array keeps the first call's grid, which the second must not read).
"""

import ctypes

import numpy as np
import pytest
import torch

from oracle import omniseg_oracle as O
from paper_2305_14566_amd import omniseg as om


def _case(H, W, T, s, keep, seed):
    rng = np.random.default_rng(seed)
    ny, nx = O.grid_count(H, T, s), O.grid_count(W, T, s)
    tiles = [(jy, jx) for jy in range(ny) for jx in range(nx) if rng.uniform() < keep]
    logits = rng.standard_normal((len(tiles), T, T)).astype(np.float32)
    return tiles, logits


@pytest.mark.gpu
@pytest.mark.parametrize("vote", [0, 2])
def test_noalloc_stitch_matches_workspace_stitch(vote):
    dev = torch.device("cuda:0")
    # the second call has a smaller grid and fewer tiles than the first
    for (H, W, T, s, keep, seed) in [(900, 1300, 64, 32, 0.6, 1), (300, 257, 64, 32, 0.8, 2),
                                     (97, 250, 32, 8, 0.9, 3)]:
        print(f"noalloc stitch H={H} W={W} T={T} s={s} vote={vote}", flush=True)
        tiles, logits = _case(H, W, T, s, keep, seed)
        lg = torch.from_numpy(logits).to(dev)
        yx = torch.tensor(np.array(tiles, np.int32).reshape(-1, 2), device=dev)
        ref_m, ref_l = om.stitch_tiles(T, s, H, W, lg, yx, vote_threshold=vote)
        mask = torch.full((H, W), 7, dtype=torch.uint8, device=dev)
        logit = torch.full((H, W), 7.0, dtype=torch.float32, device=dev)
        om.stitch_tiles_noalloc(T, s, H, W, lg, yx, mask, logit, vote_threshold=vote)
        torch.cuda.synchronize()
        assert torch.equal(mask, ref_m)
        assert torch.equal(logit, ref_l)
        # against the FP64 oracle's definition too (ramp mean)
        if vote == 0:
            lam, _, _ = O.stitch(tiles, [x.astype(np.float64) for x in logits], H, W, T, s)
            got = logit.cpu().numpy().astype(np.float64)
            assert np.abs(got - lam).max() <= 1e-5 * max(1.0, np.abs(lam).max())


def test_noalloc_stitch_refuses_grids_above_its_array():
    """2^20 grid positions at most; checked before any HIP call."""
    lib = om.lib()
    # tile 16 at stride 1 over 2000 x 2000: 1985^2 positions
    st = lib.omniseg_stitch_tiles_noalloc(16, 1, 2000, 2000, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), 1,
                                          ctypes.c_void_p(16), 2000, None, 0, None)
    assert st == 2, st
    assert b"above" in lib.omniseg_last_error()
    st = lib.omniseg_stitch_tiles_noalloc(16, 32, 100, 100, 0, None, None, 0, ctypes.c_void_p(16), 100, None, 0,
                                          None)
    assert st == 1  # stride above the tile
