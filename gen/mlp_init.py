"""Seeded initial weights of the learned-setup network (inputs, not arithmetic).

Layout shared by the library and the CPU oracle: W1 (64 x 128), b1 (128),
W2 (128 x 128), b2 (128), W3 (128 x 64), b3 (64), row-major, concatenated.
"""
import numpy as np

F_IN, HID, F_OUT = 64, 128, 64
SHAPES = [(F_IN, HID), (HID,), (HID, HID), (HID,), (HID, F_OUT), (F_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)


def init_params(seed):
    """He-style normal initialisation from numpy's PCG64; zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((F_IN, HID)) * np.sqrt(2.0 / F_IN)
    W2 = rng.standard_normal((HID, HID)) * np.sqrt(2.0 / HID)
    W3 = rng.standard_normal((HID, F_OUT)) * np.sqrt(1.0 / HID)
    return [W1, np.zeros(HID), W2, np.zeros(HID), W3, np.zeros(F_OUT)]


def flatten(params):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params]).astype(np.float32)


def unflatten(flat):
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(np.asarray(flat[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out
