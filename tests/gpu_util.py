"""Helpers shared by the GPU tests (device transfer, ulp comparisons)."""
import numpy as np


def dev(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a if dtype is None else np.asarray(a).astype(dtype))
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16)).cuda().view(torch.uint16)
    return torch.from_numpy(a).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def empty(shape, dtype):
    import torch
    return torch.empty(shape, dtype=dtype, device="cuda")


def ulp_diff(gpu_f32, oracle_f64):
    """|gpu - oracle| in units of the FP32 spacing at the oracle value."""
    o32 = np.asarray(oracle_f64, np.float64).astype(np.float32)
    sp = np.spacing(np.abs(o32)).astype(np.float64)
    sp[sp == 0] = np.spacing(np.float32(0))
    return np.abs(np.asarray(gpu_f32, np.float64) - np.asarray(oracle_f64, np.float64)) / sp


def padded(t, pad):
    """A view of t with a row pitch of width + pad elements."""
    import torch
    H, W = t.shape
    if t.dtype == torch.uint16:
        big = torch.zeros((H, W + pad), dtype=torch.int16, device=t.device)
        big[:, :W] = t.view(torch.int16)
        return big.view(torch.uint16)[:, :W]
    big = torch.zeros((H, W + pad), dtype=t.dtype, device=t.device)
    big[:, :W] = t
    return big[:, :W]
