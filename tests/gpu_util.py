"""Helpers shared by the GPU tests (not collected by pytest)."""
import numpy as np


def sample_rows(H, width, W, n_random=16, seed=0):
    """Border rows, rows around the window edge, the middle row and a seeded
    random set -- all distinct and in range."""
    rng = np.random.default_rng(seed)
    rows = {0, 1, 2, H // 2, H - 3, H - 2, H - 1}
    for r in (W - 1, W, W + 1, H - W - 2, H - W - 1, H - W):
        rows.add(r)
    rows |= set(int(r) for r in rng.integers(0, H, n_random))
    return np.array(sorted(r for r in rows if 0 <= r < H), dtype=np.int64)


def pixels_of_rows(rows, width):
    return (rows[:, None] * width + np.arange(width)[None, :]).ravel()


def gpu_filter(img, precision="fp32", **kw):
    """Run bf_filter on a numpy image; returns (output ndarray, status)."""
    import torch

    import paper_1603_08081_amd as bfm
    x = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).cuda()
    out, st = bfm.filter(x, precision=precision, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st
