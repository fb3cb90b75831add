"""The BF16 error bound of the matrix-core BaseCase tiles, on every pair.

The tiles come from the library's own tile code (knn_debug_bf16_tiles runs
the operand construction, MFMA product, row norms and margin that the
search kernels use).  For each pair the estimate acc + ||q - c||^2 of
||q - r||^2 must lie within the margin M of the FP64 value: that is the
property the search's exactness rests on (a pair is discarded only when its
estimate minus M exceeds the threshold).  Every pair of every tile is
checked; the largest error as a fraction of M is printed."""
import numpy as np
import pytest

from oracle import kdtree as okd
from paper_1304_4327_amd import datagen

pytestmark = pytest.mark.gpu


def _tiles_from_leaves(pts, qpts, leaf, n_tiles, seed):
    """(query leaf, reference leaf) tiles as the search sees them: the centre
    is the query leaf's box centre, half the reference leaves are near ones
    (the leaf that holds the query centre's nearest reference point)."""
    rng = np.random.default_rng(seed)
    rt, qt = okd.build(pts, leaf), okd.build(qpts, leaf)
    fr, fq = rt["first_leaf"], qt["first_leaf"]
    nlr, nlq = 1 << rt["depth"], 1 << qt["depth"]
    Q, R, C = [], [], []
    rleaf_of = okd.leaf_of_rows(rt)

    def rows(t, src, node):
        s, c = t["start"][node], t["count"][node]
        idx = t["perm"][s:s + c]
        idx = np.concatenate([idx, np.repeat(idx[:1], 32 - c)])   # pad with a repeat
        return src[idx]

    for i in range(n_tiles):
        ql = int(rng.integers(nlq))
        qn = fq + ql
        cen = (np.float32(0.5) * (qt["lo"][qn] + qt["hi"][qn]).astype(np.float32)).astype(np.float32)
        if i % 2:
            rl = int(rng.integers(nlr))
        else:
            near = int(np.argmin(((pts.astype(np.float64) - cen) ** 2).sum(1)))
            rl = int(rleaf_of[near])
        Q.append(rows(qt, qpts, qn))
        R.append(rows(rt, pts, fr + rl))
        C.append(cen)
    return np.array(Q, np.float32), np.array(R, np.float32), np.array(C, np.float32)


def _synthetic(d, n_tiles, seed):
    """Gaussian tiles with offsets far from the origin, scales from 1e-3 to
    1e2, the centre near (not at) the query rows, one far row in some
    reference tiles, and exact coincidences (q = r = c) in others."""
    rng = np.random.default_rng(seed)
    Q = np.empty((n_tiles, 32, d), np.float32)
    R = np.empty_like(Q)
    C = np.empty((n_tiles, d), np.float32)
    for t in range(n_tiles):
        off = rng.uniform(-1e3, 1e3, d)
        sq = 10.0 ** rng.uniform(-3, 2)
        sr = sq * 10.0 ** rng.uniform(-1, 1)
        q = off + sq * rng.standard_normal((32, d))
        r = off + rng.uniform(-3, 3, d) * sq + sr * rng.standard_normal((32, d))
        c = q.mean(0) + 0.1 * sq * rng.standard_normal(d)
        if t % 5 == 1:
            r[7] = off + 100 * sr * rng.standard_normal(d)
        if t % 5 == 2:
            c = q[3].copy()
            r[3] = q[3]
        Q[t], R[t], C[t] = q, r, c
    return Q, R, C


def _check(Q, R, C, label):
    import torch
    from paper_1304_4327_amd import knn
    acc, qn, mg = knn.knn_debug_bf16_tiles(torch.from_numpy(Q).cuda(), torch.from_numpy(R).cuda(),
                                           torch.from_numpy(C).cuda())
    acc = acc.cpu().numpy().astype(np.float64)
    qn = qn.cpu().numpy().astype(np.float64)
    mg = mg.cpu().numpy().astype(np.float64)
    q64, r64 = Q.astype(np.float64), R.astype(np.float64)
    exact = np.empty(acc.shape)                                        # [t, i, j]
    for t0 in range(0, len(Q), 64):
        diff = r64[t0:t0 + 64, :, None, :] - q64[t0:t0 + 64, None, :, :]
        exact[t0:t0 + 64] = (diff * diff).sum(-1)
    est = acc + qn[:, None, :]
    err = np.abs(est - exact)
    lim = np.broadcast_to(mg[:, None, :], err.shape)
    ratio = float((err / np.maximum(lim, 1e-300)).max())
    print(f"{label}: {err.size} pairs, largest error / margin = {ratio:.3f}", flush=True)
    assert np.all(err <= lim), f"{label}: {(err > lim).sum()} pairs exceed the margin"
    return ratio


@pytest.mark.parametrize("name,scale", [("manifold4m_d16_k10", 0.01),
                                        ("manifold1m_d64_k50", 0.02)])
def test_margin_holds_on_workload_tiles(name, scale):
    ref, q, k, leaf = datagen.make(name, scale=scale)
    Q, R, C = _tiles_from_leaves(ref, q, leaf, 1024, seed=11)
    _check(Q, R, C, name)


@pytest.mark.parametrize("d", [9, 16, 17, 32, 33, 64])
def test_margin_holds_on_synthetic_tiles(d):
    Q, R, C = _synthetic(d, 400, seed=d)
    _check(Q, R, C, f"synthetic d={d}")


def test_margin_is_not_vacuous():
    """The margin is a bound of the right size: on leaf tiles the largest
    observed error uses a sizeable part of it (a margin many orders too
    large would prune nothing and still pass the test above)."""
    ref, q, k, leaf = datagen.make("manifold1m_d64_k50", scale=0.02)
    Q, R, C = _tiles_from_leaves(ref, q, leaf, 1024, seed=12)
    assert _check(Q, R, C, "d=64 leaf tiles") > 0.02
