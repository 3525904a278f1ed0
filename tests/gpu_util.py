"""Shared helpers of the GPU tests: a context on cuda:0 and comparisons."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise_rel(y, ref) -> float:
    """max_i ||y_i - ref_i||_inf / max_i ||ref_i||_inf."""
    y = np.asarray(y, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.abs(y - ref).max() / max(np.abs(ref).max(), 1e-30))


_ctx = None


def ctx():
    global _ctx
    if _ctx is None:
        import torch
        from paper_2008_07799_amd import drgraph
        assert torch.cuda.is_available(), "GPU tests need a GPU"
        torch.cuda.set_device(0)
        _ctx = drgraph.Context(0)
    return _ctx


def dev_graph(csr):
    from paper_2008_07799_amd import drgraph
    return drgraph.to_device(csr)


def zeros_y(n, dtype=None):
    import torch
    return torch.zeros((n, 2), dtype=dtype or torch.float32, device="cuda")


def to_y(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()
