"""Shared helpers for the GPU parity tests (marshalling and error metrics only)."""
from __future__ import annotations

import numpy as np

GROUPS = {"mean2d": slice(0, 2), "conic": slice(2, 5), "opacity": slice(5, 6), "rgb": slice(6, 9)}


def dev():
    import torch
    return torch.device("cuda:0")


def t(a, device=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device or dev())


def grads9(g) -> np.ndarray:
    """GPU gradient dict -> [N, 9] in the oracle's column order."""
    return np.concatenate([g["means2d"].cpu().numpy(), g["conics"].cpu().numpy(),
                           g["opacities"].cpu().numpy()[:, None], g["rgb"].cpu().numpy()], 1)


def rel_l2(a, b) -> float:
    d = np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64))
    n = np.linalg.norm(np.asarray(b, np.float64))
    return float(d / n) if n > 0 else float(d)


def group_errors(g, ref) -> dict:
    out = {k: rel_l2(g[:, s], ref[:, s]) for k, s in GROUPS.items()}
    out["all"] = rel_l2(g, ref)
    return out


def splat_arrays(s):
    return dict(means2d=s.means2d, conics=s.conics, opacities=s.opacities, rgb=s.rgb)


def check_schedule(R, p, cfg, ws, items=False):
    """The raster's schedules copied back from the workspace after a backward: the forward's and
    the backward's tile orders are permutations of the tiles; with items, the depth split's work
    items in dispatch order are a permutation of the item count followed by -1, and each tile's
    items cut its 2048-position columns into consecutive ranges that cover them all (so every
    (pixel, splat) pair is composited exactly once). Returns the schedule."""
    sch = R.raster_schedule(p, cfg, ws, items=items)
    T = ((p.width + 31) // 32) * ((p.height + 31) // 32)
    for k in ("fwd_order", "bwd_order"):
        o = sch[k].cpu().numpy().reshape(-1, T)
        for v in range(o.shape[0]):
            np.testing.assert_array_equal(np.sort(o[v]), np.arange(T), err_msg=k)
    if items:
        ncol = (p.n + 2047) // 2048
        for v in range(p.n_views):
            ni = int(sch["n_items"].cpu().numpy().reshape(-1)[v])
            io = sch["item_order"].cpu().numpy().reshape(-1, 4 * T)[v]
            it = sch["items"].cpu().numpy().reshape(-1, 4 * T, 4)[v][:ni]
            assert T <= ni <= 4 * T
            np.testing.assert_array_equal(np.sort(io[:ni]), np.arange(ni))
            assert (io[ni:] == -1).all()
            for t in range(T):
                rows = it[it[:, 0] == t]
                rows = rows[np.argsort(rows[:, 1], kind="stable")]
                assert len(rows) >= 1 and rows[0, 1] == 0 and rows[-1, 2] == ncol, (t, rows)
                assert (rows[1:, 1] == rows[:-1, 2]).all() and (rows[:, 2] >= rows[:, 1]).all()
                assert (rows[:, 3] == -1).all() if len(rows) == 1 else (rows[:, 3] >= 0).all()
    return sch


def certain_grad(G, amb):
    """dL/dC with the pixels that hold a borderline decision of the oracle (R19) set to zero.
    A decision there may go either way in FP32 (a fragment at alpha = 1/255 kept or dropped, a T
    test at 1e-4), which changes T behind it by up to 0.4 %; when a splat's gradient is a sum over
    many pixels with cancelling dL/dC, those few pixels can carry a few per cent of it. Comparing
    gradients with dL/dC zeroed there on both sides measures the arithmetic, as the image check
    does by skipping the flagged pixels."""
    G = np.asarray(G)
    return (G * (np.asarray(amb) == 0)[..., None, :, :]).astype(np.float32)
