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
