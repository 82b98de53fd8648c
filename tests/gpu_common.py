"""Shared helpers of the GPU tests: the handle and oracle-side references."""
import functools
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@functools.lru_cache(maxsize=None)
def handle():
    import paper_1905_13076_amd as P
    return P.Handle(0)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def load_golden(name):
    path = os.path.join(GOLDEN, f"{name}_oracle.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def free_rows(U_nodal, free):
    return np.asarray(U_nodal)[:, free]


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
