"""Helpers for GPU tests: move seeded inputs to the device and back."""
import numpy as np


def to_dev(x: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def empty_dev(shape, dtype):
    import torch
    tdt = torch.complex64 if np.dtype(dtype) == np.complex64 else torch.complex128
    return torch.empty(tuple(shape), dtype=tdt, device="cuda")


def to_host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def layout_shape(dims, perm):
    return tuple(dims[a] for a in perm)


def bits_equal(a: np.ndarray, b: np.ndarray) -> bool:
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return a.shape == b.shape and a.dtype == b.dtype and a.tobytes() == b.tobytes()


def sampled_dft(x: np.ndarray, points, sign: int = -1) -> np.ndarray:
    """Eq. (2) at chosen output points, each summed over every input point.

    The sum is taken axis by axis (the nested form of Eq. (2)), contracting
    the last axis first, in FP64."""
    xd = np.asarray(x, dtype=np.complex128)
    dims = xd.shape
    out = []
    for k in points:
        v = xd
        for r in range(len(dims) - 1, -1, -1):
            n = dims[r]
            j = np.arange(n)
            w = np.exp(sign * 2j * np.pi * ((j * k[r]) % n) / n)
            v = v @ w
        out.append(complex(v))
    return np.array(out)
