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


def fp32_wide_product_bound(X, Y, W, h, panel=128, safety=4.0, anchor=None):
    """Elementwise bound for the FP32-entry product of wide points: exponents
    from the norm expansion on coordinates centred on the mean of Y, each FP32
    coordinate split exactly into three BF16 terms with six cross products
    kept, so a dot product sums 6 (d + 2) exact products in FP32, and the three
    dropped products (ml, lm, ll) are below 2 u of each product's magnitude:
    |dt| <= (6 (d + 2) + 2) u (|x'| + |y'|)^2 / (2 h^2) in natural-log units;
    exp2 within 2 ulp, FP32 sums over a panel of `panel` points and FP64 sums
    across panels.  `anchor` replaces the mean of Y as the centre (a batch
    centres every problem on the mean of all its points)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    a = Y.mean(axis=0) if anchor is None else np.asarray(anchor, dtype=np.float64)
    nx = np.linalg.norm(X - a, axis=1)
    ny = np.linalg.norm(Y - a, axis=1)
    q = sqdist(X, Y)
    K = np.exp(-q / (2 * h * h))
    T = (6 * (X.shape[1] + 2) + 2) * (nx[:, None] + ny[None, :]) ** 2 / (2 * h * h)
    aW = np.abs(np.asarray(W, dtype=np.float64)).reshape(W.shape[0], -1)
    return safety * U32 * ((panel + 2) * (K @ aW) + (K * T) @ aW)


U64 = 2.0 ** -53


def fp64_wide_product_bound(X, Y, W, h, safety=4.0, anchor=None):
    """Bound for the FP64-entry product of wide points: exponents from the FP64
    norm expansion on coordinates centred on the mean of Y (matrix-core dot
    products of d + 2 terms and two FP64 norms: |dt| <= (d + 6) u (|x'| +
    |y'|)^2 / (2 h^2)), exp within 1 ulp, FP64 sums over the columns.
    anchor: the centring point when it is not the mean of Y (a batch centres
    on the mean of all its points)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    a = Y.mean(axis=0) if anchor is None else np.asarray(anchor, dtype=np.float64)
    nx = np.linalg.norm(X - a, axis=1)
    ny = np.linalg.norm(Y - a, axis=1)
    K = np.exp(-sqdist(X, Y) / (2 * h * h))
    T = (X.shape[1] + 6) * (nx[:, None] + ny[None, :]) ** 2 / (2 * h * h)
    aW = np.abs(np.asarray(W, dtype=np.float64)).reshape(W.shape[0], -1)
    return safety * U64 * ((Y.shape[0] + 4) * (K @ aW) + (K * T) @ aW)


def sym_rows_per_block(d, form=3):
    """Row block of the matrix-core symmetric product: form 3 (FP32
    exponents) 1024 rows for padded widths up to 8, else 512; form 4 (BF16
    three-term exponents, d <= 31) 512 rows while the packed K (6 d + 6
    rounded up to 32) is at most 64, 256 up to 128, else 128 (the same with
    and without a negligible-tile map)."""
    if form == 4 and d <= 31:
        kt = (6 * d + 6 + 31) // 32 * 32
        return 512 if kt <= 64 else (256 if kt <= 128 else 128)
    D = (d + 3) // 4 * 4 if d <= 24 else 32
    return 1024 if D <= 8 else 512


def fp32_sym_anchored_bound(X, W, h, rows_per_block, tile=64, safety=4.0, form=3):
    """Bound for the symmetric FP32 kernel product with FP32 exponents
    re-centred per row block: an entry between rows of different blocks is
    evaluated once, by the earlier block, on x' = x - a, y' = y - a with a that
    block's mean point; its FP32 norm expansion (d FMAs per norm, d + 2 terms
    in the matrix-core sum, two constants) is off by at most
    (2 d + 6) u (|x'| + |y'|)^2 / (2 h^2) in natural-log units.  The BF16
    three-term form (4) uses the error model of the wide-point product: the
    split of a normal FP32 operand is exact, the products of BF16 terms are
    exact in FP32, the matrix-core sum adds 6 d + 6 of them (six cross
    products per coordinate, three terms of each constant against ones) and
    the dropped cross terms add at most 2 u of each product, so its sum counts
    6 d + 8 units where the FP32 form's counts d + 2: 7 d + 12 in all.
    Entries inside a diagonal block use the FP64 exponent
    (fp32_product_bound's terms)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    blk = np.arange(n) // rows_per_block
    nb = blk[-1] + 1 if n else 0
    anchors = np.stack([X[b * rows_per_block:(b + 1) * rows_per_block].mean(axis=0) for b in range(nb)])
    anchors = anchors.astype(np.float32).astype(np.float64)
    r = np.sqrt(((X[:, None, :] - anchors[None, :, :]) ** 2).sum(axis=2))  # |x_i - a_b|
    bmin = np.minimum(blk[:, None], blk[None, :])
    rows = np.arange(n)
    S = (r[rows[:, None], bmin] + r[rows[None, :], bmin]) ** 2 / (2 * h * h)
    S[blk[:, None] == blk[None, :]] = 0.0
    q = sqdist(X, X)
    T = q / (2 * h * h)
    K = np.exp(-T)
    aW = np.abs(np.asarray(W, dtype=np.float64)).reshape(W.shape[0], -1)
    terms = 7 * d + 12 if form == 4 else 2 * d + 6
    return safety * U32 * ((tile + 2) * (K @ aW) + (d + 3) * ((K * T) @ aW) + terms * ((K * S) @ aW))


def negligible_mass(X, W, h, log2_thr=-31.5):
    """Per row, sum_j |K_ij| |W_j| over the entries below 2^log2_thr: what a
    product that skips tiles whose entries are all below 2^-32 can leave out
    (the threshold is raised by half a binade to cover the error of the
    exponents the skip test reads)."""
    q = sqdist(X, X)
    K = np.exp(-q / (2 * h * h))
    K = np.where(K < 2.0 ** log2_thr, K, 0.0)
    aW = np.abs(np.asarray(W, dtype=np.float64)).reshape(W.shape[0], -1)
    return K @ aW


def leaf_ranges(nodes, n):
    lb = np.empty(n, dtype=np.int32)
    le = np.empty(n, dtype=np.int32)
    for b, e, l, r in nodes[:, :4]:
        if l < 0:
            lb[b:e] = b
            le[b:e] = e
    return lb, le


# relative rounding of one kernel entry by the split modes
SPLIT_U = {("f32", 1): 0.0, ("f16", 1): 2.0 ** -11, ("f16", 2): 2.0 ** -22,
           ("bf16", 1): 2.0 ** -8, ("bf16", 2): 2.0 ** -16}


def mfma_sample_bound(Xp, R, h, lb, le, prec, split, rows, rows_per_block=256, safety=4.0, anchor=None):
    """Bound for the matrix-core sampler on the given rows.

    Entry e_ij = exp2(t) with t formed in FP32 from coordinates re-centred on
    the workgroup's first point a (x' = x - a, y' = y - a): the FMA chain of
    d + 2 terms gives |dt| <= (d + 2) u c (|x'| + |y'|)^2 in log2 units.  The
    split modes at d <= 16 form t from three-term BF16 splits of the same
    operands; the error model is the one of the wide-point product: the split
    of a normal FP32 value is exact, the 6 (d + 2) kept cross products are
    exact in FP32 and summed in FP32, and the dropped ones add at most 2 u of
    each product, so 6 (d + 2) + 2 units take the place of d + 2.  Then
    |de| <= e u [2 + k c (|x'| + |y'|)^2 / (2 h^2)] with k the unit count,
    plus the split's own rounding SPLIT_U * e.  The FP32 accumulation over n
    terms is charged with the probabilistic model sqrt(n_adds) u ||e o r||_2
    (Higham and Mary 2019), FP16 entries (scaled by 2^14) add 2^-38 absolute
    where they fall below FP16's normal range,
    n_adds = n / 16 + 16 for the 16-deep FP16 / BF16 products and n / 2 + 2
    for the 2-deep FP32 ones.  The narrow kernel skips 32 x 32 tiles whose
    entries are all below 2^-32; every dropped entry is below 2^-32 (2^-31
    with the exponent's rounding), so the entries below 2^-31 are charged in
    full.  anchor: the centring point when it is one for all rows (the
    wide-point kernel centres on the mean point)."""
    Xp = np.asarray(Xp, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    n, d = Xp.shape
    out = np.zeros((len(rows), R.shape[1]))
    us = SPLIT_U[(prec, split)]
    nadd = n / 2 + 2 if prec == "f32" else n / 16 + 16
    for t, i in enumerate(rows):
        a = Xp[(i // rows_per_block) * rows_per_block] if anchor is None else anchor
        xr = np.linalg.norm(Xp[i] - a)
        yr = np.linalg.norm(Xp - a, axis=1)
        q = ((Xp - Xp[i]) ** 2).sum(axis=1)
        e = np.exp(-q / (2 * h * h))
        e[lb[i]:le[i]] = 0.0
        units = 6 * (d + 2) + 2 if (prec != "f32" and d <= 16) else d + 2
        de = e * (U32 * (2 + units * (xr + yr) ** 2 / (2 * h * h)) + us)
        if prec == "f16":
            # entries carry a 2^14 scale; below FP16's normal range the hi and
            # lo terms keep an absolute precision of 2^-25 in scaled units
            de = de + np.where(e > 0, 2.0 ** -38, 0.0)
        acc = np.sqrt(nadd) * U32 * np.sqrt((e[:, None] ** 2 * R ** 2).sum(axis=0))
        skipped = np.where(e < 2.0 ** -31, e, 0.0) @ np.abs(R)
        out[t] = safety * (de @ np.abs(R) + acc) + skipped
    return out
