"""Parity at the full workload sizes, in the launch configuration that the
bench times: one knn_all_knn call (both trees built on two streams, then the
search), or for the learned seed the pair build, the seed features and radii
and the seeded search.  The FP64 oracle computes a seeded sample of query
rows one by one against every reference point; every row is checked for the
properties that hold at any size (indices in range and distinct, distances
ascending and finite)."""
import numpy as np
import pytest

from oracle import knn as ok
from oracle import parity
from paper_1304_4327_amd import datagen

pytestmark = pytest.mark.gpu


def _rows(n, count, salt):
    rng = np.random.default_rng(1000 + salt)
    return np.sort(rng.choice(n, size=min(count, n), replace=False))


def _every_row(gi, gd, m):
    assert ((gi >= 0) & (gi < m)).all()
    s = np.sort(gi, axis=1)
    assert not (s[:, 1:] == s[:, :-1]).any()
    assert np.isfinite(gd).all() and (gd >= 0).all()
    assert (np.diff(gd, axis=1) >= 0).all()


@pytest.mark.parametrize("name,precision,count", [
    ("gmm1m_d3_k10", "fp32", 256),
    ("zipfgmm2m_d8_k10", "fp32", 256),
    ("manifold4m_d16_k10", "fp32", 128),
    ("manifold4m_d16_k10", "bf16", 128),
    ("manifold1m_d64_k50", "bf16", 128),
])
def test_full_size_sampled_rows(name, precision, count):
    import torch
    from paper_1304_4327_amd import knn
    ref, q, k, leaf = datagen.make(name)
    print(f"full size: {name} {precision} n_ref={len(ref)} n_q={len(q)} k={k}", flush=True)
    R = torch.from_numpy(ref).cuda()
    Q = torch.from_numpy(q).cuda()
    idx, dist, _ = knn.knn_all_knn(R, Q, k, leaf, precision=precision)
    torch.cuda.synchronize()
    gi, gd = idx.cpu().numpy(), dist.cpu().numpy()
    del R, Q, idx, dist
    _every_row(gi, gd, len(ref))
    rows = _rows(len(q), count, len(name) + k)
    oi, od = ok.knn_rows(q, rows, ref, k)
    parity.assert_ok(q, ref, k, gi, gd, oi, od, rows=rows)


def test_full_size_learned_bf16_sampled_rows():
    """The combined variant at d = 64 (learned seed radius and BF16 tiles),
    the network trained on small draws of the training seeds: any seed keeps
    the answer exact, so the sampled rows must match the oracle."""
    import torch
    from paper_1304_4327_amd import knn
    from paper_1304_4327_amd import seed as S
    name = "manifold1m_d64_k50"
    base = datagen.DEFAULT_SEEDS[name]
    model = S.train_for_workload(name, [base + 100 + i for i in range(4)], scale=0.05, epochs=5,
                                 precision="bf16")
    ref, q, k, leaf = datagen.make(name)
    print(f"full size learned: {name} n_ref={len(ref)} n_q={len(q)} k={k}", flush=True)
    R = torch.from_numpy(ref).cuda()
    Q = torch.from_numpy(q).cuda()
    rt, qt = knn.knn_build_tree_pair(R, Q, leaf)
    rad = S.radii(model, knn.knn_seed_features(rt, qt))
    idx, dist, st = knn.knn_search(rt, qt, k, precision="bf16", seed_radius=rad, stats=True)
    torch.cuda.synchronize()
    qt.close()
    rt.close()
    gi, gd = idx.cpu().numpy(), dist.cpu().numpy()
    _every_row(gi, gd, len(ref))
    rows = _rows(len(q), 128, 77)
    oi, od = ok.knn_rows(q, rows, ref, k)
    parity.assert_ok(q, ref, k, gi, gd, oi, od, rows=rows)
