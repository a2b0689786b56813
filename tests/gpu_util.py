"""Helpers shared by the GPU tests (marshalling only)."""
import numpy as np


def device():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to(device())


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def empty(n):
    import torch
    return torch.empty(n, dtype=torch.complex128, device=device())


def rand_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return v / np.linalg.norm(v)


def max_rel(x, ref):
    """max_i |x_i - ref_i| / max_i |ref_i| (element by element)."""
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def say(msg):
    print(msg, flush=True)
