"""Hypothesis strategies shared by the property-based tests (inputs only)."""
import numpy as np
from hypothesis import strategies as st

import graphgen as gg


@st.composite
def graphs(draw):
    """n in [2, 40] split into 1-3 parts of at least 2 vertices, a random tree on
    each part (so some graphs are disconnected, none has an isolated vertex),
    plus up to 3n random extra edges (which may join the parts)."""
    n = draw(st.integers(2, 40))
    k = draw(st.integers(1, max(1, min(3, n // 2))))
    rng = np.random.default_rng(draw(st.integers(0, 2**31 - 1)))
    perm = rng.permutation(n)
    cuts = [0] + sorted(rng.choice(np.arange(1, n // 2), size=k - 1, replace=False) * 2) + [n] \
        if k > 1 else [0, n]
    u, v = [], []
    for s0, s1 in zip(cuts[:-1], cuts[1:]):
        for i in range(s0 + 1, s1):
            u.append(perm[i])
            v.append(perm[s0 + rng.integers(0, i - s0)])
    extra = draw(st.integers(0, 3 * n))
    u = np.concatenate([np.asarray(u, dtype=np.int64), rng.integers(0, n, extra)])
    v = np.concatenate([np.asarray(v, dtype=np.int64), rng.integers(0, n, extra)])
    return gg.csr_from_edges(n, u, v)


@st.composite
def directed_graphs(draw):
    """n in [1, 40]; every vertex gets 0-4 random out-edges (so some are dangling,
    some rows empty); returned by targets (row u lists the sources of v -> u)."""
    n = draw(st.integers(1, 40))
    rng = np.random.default_rng(draw(st.integers(0, 2**31 - 1)))
    deg = rng.integers(0, 5, n)
    src = np.repeat(np.arange(n), deg)
    dst = rng.integers(0, n, src.size)
    keep = src != dst
    key = np.unique(dst[keep].astype(np.int64) * n + src[keep])
    u, v = key // n, key % n
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(u, minlength=n), out=rp[1:])
    return gg.CSR(n=n, row_ptr=rp.astype(np.int32), col_idx=v.astype(np.int32))
