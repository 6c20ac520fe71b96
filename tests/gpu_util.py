"""Shared helpers of the GPU tests (inputs only; no arithmetic of the method)."""
import sys

import numpy as np


def need_gpu():
    import pytest
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def blocks(rng, n, s, p):
    return rng.integers(0, p, size=(n, s), dtype=np.int64), rng.integers(0, p, size=(n, s), dtype=np.int64)
