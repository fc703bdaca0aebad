"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import numpy as np
import pytest
import torch

gpu = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def announce(msg):
    # names the case before the GPU step, so a fault report is attributable
    print(f"[gpu-case] {msg}", flush=True)


def to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()
