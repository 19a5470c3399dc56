"""Small helpers for the tests (dense matrices by probing, norms)."""
import numpy as np


def dense_from_apply(fn, in_shape):
    """Dense matrix of a linear map given as a function on arrays of in_shape."""
    n = int(np.prod(in_shape))
    cols = []
    for i in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[i] = 1.0
        cols.append(np.asarray(fn(e.reshape(in_shape))).reshape(-1))
    return np.array(cols).T


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.reshape(-1))
    return np.linalg.norm((a - b).reshape(-1)) / (nb if nb > 0 else 1.0)
