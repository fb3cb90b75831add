"""Learned seed radius on the GPU: network kernels vs the FP64 reference,
features vs the oracle, exactness under any seed, and the gain of a
trained network over the plain search."""
import numpy as np
import pytest

from oracle import kdtree as okd
from oracle import knn as ok
from oracle import mlp as omlp
from oracle import parity
from oracle import seed_features as osf
from paper_1304_4327_amd import datagen

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _net(n_in, seed):
    from paper_1304_4327_amd import knn
    rng = np.random.default_rng(seed)
    p = datagen.mlp_init(n_in, 64, seed)
    p[64 * n_in:64 * n_in + 64] = rng.normal(0, 0.1, 64)     # non-zero biases
    mu = rng.normal(size=n_in).astype(np.float32)
    isd = rng.uniform(0.5, 2.0, n_in).astype(np.float32)
    net = knn.Mlp(n_in)
    net.set_params(p)
    net.set_norm(mu, isd)
    return net, p.astype(np.float64), mu.astype(np.float64), isd.astype(np.float64)


@pytest.mark.parametrize("n_in,n", [(11, 1), (11, 1000), (19, 333), (67, 257)])
def test_forward_and_gradient_match_fp64(n_in, n):
    torch = _torch()
    net, p, mu, isd = _net(n_in, n_in + n)
    rng = np.random.default_rng(n)
    x = rng.normal(size=(n, n_in)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    X, T = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    y = net.forward(X).cpu().numpy()
    y64 = omlp.forward(p, x, mu, isd, n_in, 64)
    np.testing.assert_allclose(y, y64, rtol=1e-4, atol=1e-5 * np.abs(y64).max())
    loss = net.loss_grad(X, T)
    L64, g64 = omlp.loss_and_grad(p, x, t, mu, isd, n_in, 64)
    assert abs(loss - L64) <= 1e-4 * L64
    g = net.get_grads()
    scale = np.abs(g64).max()
    assert np.all(np.abs(g - g64) <= 1e-4 * (np.abs(g64) + 1e-3 * scale))


def test_adam_steps_match_fp64():
    torch = _torch()
    n_in, n = 11, 500
    net, p, mu, isd = _net(n_in, 5)
    rng = np.random.default_rng(6)
    x = rng.normal(size=(n, n_in)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    X, T = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(1, 4):
        net.loss_grad(X, T)
        net.adam_step(1e-3)
        _, g = omlp.loss_and_grad(p, x, t, mu, isd, n_in, 64)
        p, m, v = omlp.adam_step(p, g, m, v, step, 1e-3)
    got = net.get_params()
    assert np.all(np.abs(got - p) <= 2e-6 + 1e-5 * np.abs(p))


def test_save_load_roundtrip(tmp_path):
    from paper_1304_4327_amd import knn
    net, p, mu, isd = _net(11, 2)
    f = str(tmp_path / "net.knnseed")
    net.save(f)
    back = knn.Mlp.load_file(f)
    np.testing.assert_array_equal(back.get_params(), net.get_params())
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a model")
    with pytest.raises(knn.KnnError) as e:
        knn.Mlp.load_file(str(bad))
    assert e.value.status == knn.KNN_E_MODEL


def test_seed_features_match_oracle():
    torch = _torch()
    from paper_1304_4327_amd import knn
    ref, q, k, leaf = datagen.make("zipfgmm2m_d8_k10", scale=0.004)
    rt = knn.knn_build_tree(torch.from_numpy(ref).cuda(), leaf)
    qt = knn.knn_build_tree(torch.from_numpy(q).cuda(), leaf)
    f = knn.knn_seed_features(rt, qt).cpu().numpy().astype(np.float64)
    o = osf.features(okd.build(ref, leaf), okd.build(q, leaf))
    d = ref.shape[1]
    np.testing.assert_array_equal(f[:, :d], o[:, :d])            # centres
    np.testing.assert_array_equal(f[:, d + 1], o[:, d + 1])      # counts
    assert np.all(f[:, d] >= o[:, d]) and np.all(f[:, d] <= o[:, d] * (1 + 3e-7))
    np.testing.assert_allclose(f[:, d + 2], o[:, d + 2], rtol=1e-5, atol=1e-4)


def _seeded(ref, q, k, leaf, seed_fn, precision="fp32"):
    torch = _torch()
    from paper_1304_4327_amd import knn
    rt = knn.knn_build_tree(torch.from_numpy(ref).cuda(), leaf)
    qt = knn.knn_build_tree(torch.from_numpy(q).cuda(), leaf)
    nl = qt.info()["n_leaves"]
    seed = seed_fn(nl)
    s = None if seed is None else torch.from_numpy(seed.astype(np.float32)).cuda()
    idx, dist, st = knn.knn_search(rt, qt, k, precision=precision, seed_radius=s, stats=True)
    return idx.cpu().numpy(), dist.cpu().numpy(), st


# seeds that send every leaf, some leaves or no leaf to the second pass;
# "half" and "quarter" flag some of the leaves that share a wavefront (FP32
# kernel) or a workgroup of four (d = 64 leaf sweep)
def _seed_fn(kind, plain_dist):
    rng = np.random.default_rng(1)
    mean_kth = float(plain_dist[:, -1].mean())
    return {"zero": lambda n: np.zeros(n), "inf": lambda n: np.full(n, np.inf),
            "random": lambda n: rng.exponential(mean_kth, n),
            "half": lambda n: np.where(np.arange(n) % 2 == 0, np.inf, 0.0),
            "quarter": lambda n: np.where(np.arange(n) % 4 == 3, 0.0, np.inf),
            "nan": lambda n: np.full(n, np.nan), "negative": lambda n: -np.ones(n)}[kind]


@pytest.mark.parametrize("kind", ["zero", "inf", "random", "half", "quarter", "nan", "negative"])
@pytest.mark.parametrize("name,precision,scale", [("zipfgmm2m_d8_k10", "fp32", 0.003),
                                                  ("manifold4m_d16_k10", "bf16", 0.003),
                                                  ("manifold1m_d64_k50", "bf16", 0.01)])
def test_any_seed_gives_the_oracle_answer(kind, name, precision, scale):
    """Any seed keeps the answer exact: leaves whose queries end beyond
    their seed are searched again (the FP32 kernel's in-wave second pass,
    the BF16 kernels' second launch) and must still match the oracle, and
    equal the plain search bit for bit."""
    ref, q, k, leaf = datagen.make(name, scale=scale)
    print(f"seed {kind}: {name} {precision} n_ref={len(ref)} n_q={len(q)}", flush=True)
    plain = _seeded(ref, q, k, leaf, lambda n: None, precision)
    got = _seeded(ref, q, k, leaf, _seed_fn(kind, plain[1]), precision)
    oi, od = ok.knn(q, ref, k)
    parity.assert_ok(q, ref, k, got[0], got[1], oi, od)
    assert np.array_equal(got[0], plain[0]) and np.array_equal(got[1], plain[1])
    st, nl = got[2], got[2]["n_query_leaves"]
    if kind in ("zero", "nan", "negative"):
        assert st["fallback_leaves"] == nl
    elif kind == "inf":
        assert st["fallback_leaves"] == 0
    elif kind == "half":
        assert st["fallback_leaves"] == nl // 2
    elif kind == "quarter":
        assert st["fallback_leaves"] == nl // 4
    else:
        assert 0 < st["fallback_leaves"] < nl


@pytest.mark.parametrize("kind", ["zero", "half", "random"])
def test_any_seed_per_leaf_bf16_kernel(kind):
    """Stride 32 with lists of 32: the per-leaf BF16 kernel and its second
    launch over the flagged leaves give the oracle's answer for any seed."""
    rng = np.random.default_rng(24)
    basis = rng.standard_normal((6, 24))
    ref = (rng.random((12000, 6)) @ basis + 0.05 * rng.standard_normal((12000, 24))).astype(np.float32)
    q = (rng.random((1500, 6)) @ basis + 0.05 * rng.standard_normal((1500, 24))).astype(np.float32)
    k, leaf = 20, 32
    plain = _seeded(ref, q, k, leaf, lambda n: None, "bf16")
    got = _seeded(ref, q, k, leaf, _seed_fn(kind, plain[1]), "bf16")
    oi, od = ok.knn(q, ref, k)
    parity.assert_ok(q, ref, k, got[0], got[1], oi, od)
    assert np.array_equal(got[0], plain[0]) and np.array_equal(got[1], plain[1])
    st, nl = got[2], got[2]["n_query_leaves"]
    if kind == "zero":
        assert st["fallback_leaves"] == nl
    elif kind == "half":
        assert st["fallback_leaves"] == nl // 2


@pytest.mark.parametrize("kind", ["zero", "half", "quarter", "random"])
def test_any_seed_matrix_core_traversal_stride32(kind):
    """Stride 32 with lists of 10: the matrix-core traversal's second pass in
    the same wave, for any seed, against the oracle and the plain search."""
    rng = np.random.default_rng(28)
    basis = rng.standard_normal((6, 28))
    ref = (rng.random((12000, 6)) @ basis + 0.05 * rng.standard_normal((12000, 28))).astype(np.float32)
    q = (rng.random((1500, 6)) @ basis + 0.05 * rng.standard_normal((1500, 28))).astype(np.float32)
    k, leaf = 10, 32
    plain = _seeded(ref, q, k, leaf, lambda n: None, "bf16")
    got = _seeded(ref, q, k, leaf, _seed_fn(kind, plain[1]), "bf16")
    oi, od = ok.knn(q, ref, k)
    parity.assert_ok(q, ref, k, got[0], got[1], oi, od)
    assert np.array_equal(got[0], plain[0]) and np.array_equal(got[1], plain[1])
    st, nl = got[2], got[2]["n_query_leaves"]
    if kind == "zero":
        assert st["fallback_leaves"] == nl
    elif kind == "half":
        assert st["fallback_leaves"] == nl // 2
    elif kind == "quarter":
        assert st["fallback_leaves"] == nl // 4


def test_trained_seed_prunes_more_and_stays_exact():
    """Train on 8 seeded draws of the Zipf-GMM workload (scaled down), then
    on a held-out draw: the seeded search returns the oracle's answer with
    fewer pair evaluations than the plain search."""
    torch = _torch()
    from paper_1304_4327_amd import knn, seed as S
    scale = 0.01
    model = S.train_for_workload("zipfgmm2m_d8_k10", range(40, 48), scale=scale, epochs=15)
    assert model.history[-1] < model.history[0]
    ref, q, k, leaf = datagen.make("zipfgmm2m_d8_k10", seed=48, scale=scale)
    rt = knn.knn_build_tree(torch.from_numpy(ref).cuda(), leaf)
    qt = knn.knn_build_tree(torch.from_numpy(q).cuda(), leaf)
    _, _, plain = knn.knn_search(rt, qt, k, stats=True)
    feats = knn.knn_seed_features(rt, qt)
    rad = S.radii(model, feats)
    idx, dist, st = knn.knn_search(rt, qt, k, seed_radius=rad, stats=True)
    rows = np.arange(0, len(q), 7)
    oi, od = ok.knn_rows(q, rows, ref, k)
    parity.assert_ok(q, ref, k, idx.cpu().numpy(), dist.cpu().numpy(), oi, od, rows=rows)
    assert st["fallback_leaves"] < 0.5 * st["n_query_leaves"]
    # the seeded pass itself prunes more than the plain search; the total
    # (with the fallback pass) is reported by the benchmark
    assert st["pairs"] - st["fallback_pairs"] < plain["pairs"]


def _train_data(n, n_in, seed):
    """Feature rows of seed-feature scale (centres, lambda, counts, log
    densities) and k-th distances log-linear in them, with noise."""
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, n_in)) * rng.uniform(0.1, 30.0, n_in) + rng.uniform(-50, 50, n_in)
    w = rng.normal(size=n_in) / (1.0 + np.abs(x).mean(axis=0))
    kth = np.exp(x @ w + 0.1 * rng.normal(size=n))
    return x.astype(np.float32), kth.astype(np.float32)


@pytest.mark.parametrize("n,n_in,epochs,batch", [(300, 6, 2, 64), (1000, 11, 1, 1000),
                                                 (257, 67, 3, 50), (4096, 11, 4, 512)])
def test_seed_train_follows_the_fp64_procedure(n, n_in, epochs, batch):
    """knn_seed_train against the FP64 training procedure with the same
    random streams: per-epoch losses, predictions on every row (these carry
    the standardisation), and the calibrated margin.  The FP32 and FP64 runs
    drift apart by rounding only; the bounds are a few times the drift the
    FP32 gradient (about 1e-6 relative) can build up over these step
    counts."""
    torch = _torch()
    from paper_1304_4327_amd import knn
    x, kth = _train_data(n, n_in, n + n_in)
    lr, vf, tf, seed = 1e-3, 0.2, 0.1, 17 + n
    net, margin, losses = knn.knn_seed_train(torch.from_numpy(x).cuda(), torch.from_numpy(kth).cuda(),
                                            epochs=epochs, batch=batch, lr=lr, val_frac=vf,
                                            target_fallback=tf, seed=seed)
    p, mu, isd, y_mu, y_sd, om, hist = omlp.train(x, kth, epochs, batch, lr, vf, tf, seed)
    np.testing.assert_allclose(losses, hist, rtol=2e-3)
    gy = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    oy = omlp.forward(p, x, mu, isd, n_in, 64)
    assert np.max(np.abs(gy - oy)) < 2e-3 * max(1.0, np.max(np.abs(oy)))
    assert abs(margin - om) < 5e-3 * y_sd
    gp = net.get_params().astype(np.float64)
    assert np.mean(np.abs(gp - p) < 1e-4) > 0.99


def test_seed_train_is_deterministic_and_checks_targets():
    torch = _torch()
    from paper_1304_4327_amd import knn
    x, kth = _train_data(500, 11, 3)
    X, K_ = torch.from_numpy(x).cuda(), torch.from_numpy(kth).cuda()
    a, ma, la = knn.knn_seed_train(X, K_, epochs=2, batch=100, seed=5)
    b, mb, lb = knn.knn_seed_train(X, K_, epochs=2, batch=100, seed=5)
    assert np.array_equal(a.get_params(), b.get_params()) and ma == mb and la == lb
    c, *_ = knn.knn_seed_train(X, K_, epochs=2, batch=100, seed=6)
    assert not np.array_equal(a.get_params(), c.get_params())
    for badv in (-1.0, float("nan"), float("inf")):
        kb = kth.copy()
        kb[77] = badv
        with pytest.raises(knn.KnnError) as e:
            knn.knn_seed_train(X, torch.from_numpy(kb).cuda(), epochs=1)
        assert e.value.status == knn.KNN_E_INVALID_ARG
    with pytest.raises(knn.KnnError):
        knn.knn_seed_train(X[:1].contiguous(), K_[:1].contiguous(), epochs=1)
    with pytest.raises(knn.KnnError):
        knn.knn_seed_train(X, K_, epochs=1, val_frac=1.0)
    # a zero distance (duplicate points) is a valid target
    kz = kth.copy()
    kz[:5] = 0.0
    knn.knn_seed_train(X, torch.from_numpy(kz).cuda(), epochs=1)
