"""Helpers shared by the GPU parity tests (inputs only; no method arithmetic here)."""
import numpy as np
import pytest
import torch

import rwsynth

HAVE_GPU = torch.cuda.is_available()


def need_gpu():
    if not HAVE_GPU:
        pytest.skip("no GPU")


def dev():
    return torch.device("cuda", 0)


def setup_case(w, seed=0):
    J, rid = rwsynth.phantom(w, seed)
    node, lab = rwsynth.seeds(w, rid, seed)
    return J, rid, node, lab


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
