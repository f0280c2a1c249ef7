"""Helpers for the GPU parity tests: host <-> device copies in the layouts the
C ABI expects (RFP arrays 1-D, full matrices column-major)."""
import numpy as np
import torch


def dev(x):
    """1-D numpy -> device tensor."""
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def dev_colmajor(a):
    """2-D numpy -> device tensor with stride(0) == 1 (column-major)."""
    a = np.asarray(a)
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def host_colmajor(t):
    torch.cuda.synchronize()
    return np.asfortranarray(t.t().contiguous().cpu().numpy().T)


def info_tensor():
    return torch.full((1,), -7, dtype=torch.int32, device="cuda")


def read_info(t):
    torch.cuda.synchronize()
    return int(t.item())
