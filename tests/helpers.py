"""Shared test helpers: key conversion and oracle-side reference computation."""
import numpy as np
import torch

import oracle


def keys_u32(keys) -> np.ndarray:
    """int64 tensor / array of uint32 values -> uint32 numpy [n, a]."""
    a = keys.numpy() if isinstance(keys, torch.Tensor) else np.asarray(keys)
    a = a.astype(np.uint32)
    return a.reshape(a.shape[0], -1) if a.ndim == 1 else a


def to_device_keys(keys_np: np.ndarray) -> torch.Tensor:
    """uint32 numpy [n, a] -> contiguous int32 device tensor holding the same bits."""
    return torch.from_numpy(np.ascontiguousarray(keys_np).view(np.int32)).cuda()


def oracle_sketches(graph, rels, weights, m, d, seed):
    info = oracle.analyze(graph)
    co = oracle.draw_coefficients(seed, d, len(info.edges), info.n_comp)
    sk = [oracle.create_sketch(info, k, rels[k], None if weights is None else weights[k], m, co)
          for k in range(info.n_rel)]
    return info, co, sk
