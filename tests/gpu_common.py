"""Shared helpers of the GPU parity tests (no oracle arithmetic here)."""
import json
import os
import sys

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def golden(name):
    p = os.path.join(GOLD, name)
    if not os.path.exists(p):
        pytest.skip(f"golden file {name} not generated")
    with open(p) as f:
        return json.load(f)


def build(ctx, g, flags=0):
    return ctx.build_csr(g.n_u, g.n_v, g.eu, g.ev, g.sign, flags)
