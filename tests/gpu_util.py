"""Helpers for the GPU tests: device transfer and tolerance checks.
Inputs come from `workloads` (seeded), expected values from `oracle`."""
import numpy as np
import torch


def dev(a, dtype=torch.complex128):
    """numpy -> column-major device tensor."""
    a = np.asarray(a)
    if a.ndim == 2:
        a = np.asfortranarray(a)
        t = torch.from_numpy(a)
        out = torch.empty_strided(a.shape, (1, max(1, a.shape[0])), dtype=dtype, device="cuda")
        out.copy_(t)
        return out
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def colerr(X, R):
    """per-column ||X - R||_inf / ||R||_inf (absolute where R = 0)."""
    d = np.max(np.abs(X - R), axis=0)
    n = np.max(np.abs(R), axis=0)
    return np.where(n > 0, d / np.where(n > 0, n, 1), d)


def announce(msg):
    print("[gpu-test]", msg, flush=True)
