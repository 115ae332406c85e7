"""Shared helpers of the test suite (comparison metrics, case logging)."""
import sys

import numpy as np


def rel_err_points(x, ref):
    """Per-point normwise relative error ||x - ref||_F / ||ref||_F (first axis = point)."""
    x = np.asarray(x).reshape(len(x), -1)
    ref = np.asarray(ref).reshape(len(ref), -1)
    num = np.linalg.norm(x - ref, axis=1)
    den = np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    return num / den


def log_case(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()
