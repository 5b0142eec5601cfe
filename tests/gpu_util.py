"""Helpers for the GPU parity tests (error bounds written from the arithmetic)."""
import numpy as np

U32 = 2.0 ** -24


def sqdist(X, Y):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    q = np.zeros((X.shape[0], Y.shape[0]))
    for k in range(X.shape[1]):
        diff = X[:, k][:, None] - Y[:, k][None, :]
        q += diff * diff
    return q


def fp32_product_bound(X, Y, W, h, tile=64, safety=4.0, mask=None):
    """Elementwise bound for an FP32 kernel product K(X, Y) W whose entries come
    from exact coordinate differences (relative error <= (d + 3) u t on an
    entry with exponent t = q / (2 h^2)), exp2 within 2 ulp, and FP32 sums over
    a tile of `tile` columns followed by FP64 sums:
        |err_i| <= safety * u * [ (tile + 2) (|K| |W|)_i + (d + 3) (|K o T| |W|)_i ]."""
    q = sqdist(X, Y)
    t = q / (2 * h * h)
    K = np.exp(-t)
    if mask is not None:
        K = np.where(mask, 0.0, K)
    aW = np.abs(np.asarray(W, dtype=np.float64)).reshape(W.shape[0], -1)
    d = X.shape[1]
    return safety * U32 * ((tile + 2) * (K @ aW) + (d + 3) * ((K * t) @ aW))


def leaf_ranges(nodes, n):
    lb = np.empty(n, dtype=np.int32)
    le = np.empty(n, dtype=np.int32)
    for b, e, l, r in nodes[:, :4]:
        if l < 0:
            lb[b:e] = b
            le[b:e] = e
    return lb, le
