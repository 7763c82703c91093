"""Shared helpers for the GPU tests: a session context and cached workload graphs."""

import functools
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def config_graph(cfg: int, scale_down: int = 0):
    from paper_2502_06715_amd import inputs
    return inputs.config_graph(cfg, scale_down)


def sort_rows(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.int64)
    if a.shape[0] == 0:
        return a
    return a[np.lexsort(a.T[::-1])]
