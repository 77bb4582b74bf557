"""Shared helpers of the GPU tests: problem upload and handle management."""
import numpy as np

from paper_2206_03410_amd import amm


def gpu_problem(pair, dtype):
    """amm_problem over cuda tensors of the pair's arrays in `dtype`."""
    import torch
    dev = "cuda:0"

    def t(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)

    return amm.make_problem(t(pair.src, dtype), t(pair.tgt, dtype), t(pair.node_idx, torch.int32),
                            t(pair.infl_idx, torch.int32), t(pair.infl_w, dtype),
                            t(pair.edges, torch.int32), pair.mean_edge_len)


def rounded(pair, np_dtype):
    """Copy of the pair whose float arrays are rounded to np_dtype (and kept
    as float64), so that a float32 library run and the float64 oracle see
    identical inputs."""
    import dataclasses
    r = lambda a: np.asarray(a, np_dtype).astype(np.float64)
    return dataclasses.replace(pair, src=r(pair.src), tgt=r(pair.tgt), infl_w=r(pair.infl_w))


class Session:
    def __init__(self, pairs, dtype):
        import torch
        self.torch = torch
        self.stream = torch.cuda.current_stream()
        self.h = amm.amm_create(0, self.stream.cuda_stream)
        pairs = pairs if isinstance(pairs, (list, tuple)) else [pairs]
        self.problems = [gpu_problem(p, dtype) for p in pairs]
        amm.amm_set_problems(self.h, self.problems)

    def close(self):
        if self.h is not None:
            amm.amm_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def margin_ok(d1, d2s, rel=1e-6):
    """Queries whose best and second-best distances (inputs are squared)
    differ by more than `rel` relative: there the closest index must match
    exactly."""
    a, b = np.sqrt(d1), np.sqrt(d2s)
    return (b - a) > rel * b
