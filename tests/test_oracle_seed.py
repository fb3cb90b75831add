"""Properties of the oracle seed features (CPU)."""
import numpy as np

from oracle import kdtree as kd
from oracle import seed_features as sf
from paper_1304_4327_amd import datagen


def test_feature_layout_and_uniform_density():
    """Uniform points in the unit cube: every leaf's log density is close to
    log(count / tight-box volume), which for this input is near log(N)
    (tight boxes are a little smaller than the cells)."""
    pts = datagen.uniform(4096, 3, 9)
    t = kd.build(pts, 8)
    f = sf.features(t, t)
    assert f.shape == (512, 6)
    fl = t["first_leaf"]
    np.testing.assert_array_equal(f[:, 4], t["count"][fl:])
    np.testing.assert_array_equal(f[:, 3], t["lam"][fl:])
    med = np.median(f[:, 5])
    assert np.log(4096) - 0.5 < med < np.log(4096) + 3.0


def test_self_descent_reaches_own_leaf():
    """With query tree = reference tree the centre of a leaf lies in that
    leaf's box, so the nearer-child descent ends in it whenever no other
    leaf box also contains the centre (almost always for continuous data)."""
    pts = datagen.uniform(2048, 2, 4)
    t = kd.build(pts, 4)
    fl = t["first_leaf"]
    own = 0
    for leaf in range(1 << t["depth"]):
        node = fl + leaf
        c = (np.float32(0.5) * (t["lo"][node] + t["hi"][node]).astype(np.float32)).astype(np.float32)
        r = 0
        while r < fl:
            a, b = 2 * r + 1, 2 * r + 2
            r = b if sf._box_d2(t["lo"][b], t["hi"][b], c) < sf._box_d2(t["lo"][a], t["hi"][a], c) else a
        own += r == node
    assert own >= 0.95 * (1 << t["depth"])


def _read_fixture(path):
    ref, qry, feats, leaf = [], [], [], None
    for line in open(path):
        t = line.split("#", 1)[0].split()
        if not t:
            continue
        if t[0] == "ref":
            ref.append([float(v) for v in t[1:]])
        elif t[0] == "query":
            qry.append([float(v) for v in t[1:]])
        elif t[0] == "feature":
            feats.append([float(v) for v in t[1:]])
        elif t[0] == "leaf_size":
            leaf = int(t[1])
    return (np.array(ref, np.float32), np.array(qry, np.float32), np.array(feats), leaf)


def test_features_of_hand_built_tree(golden_dir):
    """Hand-derived features of a tiny tree pair: leaf centres, lambda,
    counts and the density of the reference leaf that the nearer-child
    descent reaches (distinct densities on both sides of each descent
    choice, so a wrong centre or a wrong child choice changes the value)."""
    import os
    ref, qry, want, leaf = _read_fixture(os.path.join(golden_dir, "seed_features_tiny.txt"))
    got = sf.features(kd.build(ref, leaf), kd.build(qry, leaf))
    assert got.shape == want.shape
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
