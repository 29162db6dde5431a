"""Helpers shared by the GPU parity tests (relative-error definitions)."""
import numpy as np


def rel_scalar(a, b):
    """|a - b| / |b| for scalars."""
    return abs(a - b) / max(abs(b), 1e-300)


def rel_vec(a, b):
    """max_i |a_i - b_i| / |b_i| over elements (per-walker vectors)."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def rel_fro(a, b):
    """||a - b||_F / ||b||_F for tensors."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))


def to_np(t):
    return t.detach().cpu().numpy()
