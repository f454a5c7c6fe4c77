"""Shared helpers of the GPU tests (device buffers through torch, contexts)."""
import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch


def dev(a, dtype):
    torch = torch_cuda()
    t = torch.as_tensor(np.ascontiguousarray(a), dtype=dtype)
    return t.to("cuda:0")


def ctx_for(ph, dtype=None, **opts):
    import paper_1003_5402_amd as dao
    torch = torch_cuda()
    stream = torch.cuda.current_stream().cuda_stream
    return dao.DaoContext.from_phantom(ph, dtype=dtype, stream=stream, **opts)


def tdtype(ctx):
    torch = torch_cuda()
    return torch.float64 if ctx.dtype == "f64" else torch.float32


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))
