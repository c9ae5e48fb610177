"""MI355X (gfx950) Fourier-kernel shiftable bilateral filter.

The C ABI (include/bf.h, libbf.so) holds the whole path: the host-side
coefficient fit and the HIP kernels.  ``native`` is a thin ctypes binding
with the ABI's names; ``filter`` below is a convenience wrapper that
allocates the output tensor with torch and calls ``bf_filter``.
"""
from __future__ import annotations


def filter(img, *, spatial="gaussian", sigma_s=3.0, W=-1, range_kind="gaussian", sigma_r=30.0,
           T=255, eps=1e-2, K_max=None, d=None, phi_table=None, precision="fp32", integer_input=False,
           f_max=0, out=None, stream=None):
    """Filter one 2-D float32 CUDA tensor with eq. (9); returns (out, status)."""
    import torch

    from . import native
    if img.dtype != torch.float32 or img.dim() != 2 or not img.is_cuda:
        raise ValueError("expected a 2-D float32 tensor on the GPU")
    if img.stride(-1) != 1:
        raise ValueError("rows must be contiguous")
    if out is None:
        out = torch.empty_like(img, memory_format=torch.contiguous_format)
    job = native.Job(img, out, spatial=spatial, sigma_s=sigma_s, W=W, range_kind=range_kind,
                     sigma_r=sigma_r, T=T, eps=eps, K_max=K_max, d=d, phi_table=phi_table,
                     integer_input=integer_input, f_max=f_max)
    st = native.bf_filter(job, precision, stream=stream)
    return out, st


def filter_recursive(img, *, sigma_s=3.0, range_kind="gaussian", sigma_r=30.0, T=255, eps=1e-2,
                     K_max=None, d=None, phi_table=None, integer_input=False, f_max=0, out=None,
                     stream=None):
    """Eq. (9) with Deriche's recursive Gaussian as the spatial smoothing
    (bf_filter_recursive) on one 2-D float32 CUDA tensor; returns (out, status)."""
    import torch

    from . import native
    if img.dtype != torch.float32 or img.dim() != 2 or not img.is_cuda:
        raise ValueError("expected a 2-D float32 tensor on the GPU")
    if img.stride(-1) != 1:
        raise ValueError("rows must be contiguous")
    if out is None:
        out = torch.empty_like(img, memory_format=torch.contiguous_format)
    job = native.Job(img, out, spatial="gaussian", sigma_s=sigma_s, W=0, range_kind=range_kind,
                     sigma_r=sigma_r, T=T, eps=eps, K_max=K_max, d=d, phi_table=phi_table,
                     integer_input=integer_input, f_max=f_max)
    n = native.bf_recursive_workspace_bytes(job)
    ws = torch.empty(n, dtype=torch.uint8, device=img.device)
    st = native.bf_filter_recursive(job, ws, n, stream=stream)
    out._bf_workspace = ws   # keeps the workspace alive until the caller drops the output
    return out, st


def dynamic_range(img, W, stream=None) -> int:
    """Local dynamic range of a 2-D float32 CUDA tensor over [-W, W]^2 windows
    (bf_dynamic_range); synchronises to return the integer."""
    import torch

    from . import native
    if img.dtype != torch.float32 or img.dim() != 2 or not img.is_cuda or img.stride(-1) != 1:
        raise ValueError("expected a 2-D float32 tensor on the GPU with contiguous rows")
    n = native.bf_dynamic_range_workspace_bytes(img.shape[0], img.shape[1])
    ws = torch.empty(n, dtype=torch.uint8, device=img.device)
    t = torch.zeros(1, dtype=torch.int32, device=img.device)
    native.bf_dynamic_range(img, W, t, ws, n, stream=stream)
    return int(t.item())
