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
