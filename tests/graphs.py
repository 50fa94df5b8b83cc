"""Seeded graphs with a given structure for the GPU tests (inputs only: no
survey arithmetic here)."""
import numpy as np


def huge_targets(seed, na=40, nb=3400, np_=3000, leaf_edges_per_b=3700, density=0.99):
    """Targets of d+ above 3276 with in-edges whose candidates straddle the
    pieces of their out-lists, at few triangles.  Each of `na` vertices A
    is adjacent to most of `nb` vertices B; B vertices get a higher degree
    from leaves of degree 4, so all of B ranks above A and d+(a) > 3276;
    `np_` vertices P (lower degree) each touch 3 of A and 150 of B, so the
    records p -> a carry suffixes of B ranks that the piece bounds cut.
    Returns n, src, dst, times, labels (5 labels)."""
    rng = np.random.default_rng(seed)
    A = np.arange(na)
    B = np.arange(na, na + nb)
    P = np.arange(na + nb, na + nb + np_)
    n_leaves = nb * leaf_edges_per_b // 4
    L0 = na + nb + np_
    n = L0 + n_leaves
    parts = []
    ab = np.array(np.meshgrid(A, B, indexing="ij")).reshape(2, -1)
    ab = ab[:, rng.random(ab.shape[1]) < density]
    parts.append(ab)
    parts.append(np.stack([rng.choice(B, 60000), rng.choice(B, 60000)]))  # sparse B-B
    parts.append(np.stack([np.repeat(P, 3), rng.choice(A, 3 * np_)]))
    parts.append(np.stack([np.repeat(P, 150), rng.choice(B, 150 * np_)]))
    parts.append(np.stack([np.repeat(np.arange(L0, n), 4), rng.choice(B, 4 * n_leaves)]))
    e = np.concatenate(parts, axis=1)
    src, dst = e[0].astype(np.uint32), e[1].astype(np.uint32)
    ts = rng.integers(0, 1 << 22, len(src)).astype(np.uint32)
    vlab = rng.integers(0, 5, n).astype(np.uint8)
    return n, src, dst, ts, vlab
