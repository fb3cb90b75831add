"""knn_search_noalloc (the entry point that allocates nothing) against
knn_search, through the C ABI: the same answers and counters, bit for bit,
on two calls in a row (the second with a smaller input, so stale scratch
from the first call would show), for every kernel family and with a seed
that sends leaves to the fallback pass; and the size limit.  At d = 64 with
BF16 tiles the no-alloc form runs the staged sweep (the wave-independent one
needs 4 KB of operands per reference leaf): the answers and fallback counts
are still identical, the traversal counters are not compared."""
import numpy as np
import pytest

from oracle import knn as ok
from oracle import parity
from paper_1304_4327_amd import datagen

pytestmark = pytest.mark.gpu

CASES = [
    # name, scale (large, small), precision, self mode, seeded
    ("gmm1m_d3_k10", (0.02, 0.005), "fp32", False, False),
    ("uniform10k_d3_k5", (1.0, 0.3), "fp32", True, False),
    ("zipfgmm2m_d8_k10", (0.004, 0.001), "fp32", False, True),
    ("manifold4m_d16_k10", (0.004, 0.001), "bf16", False, True),
    ("manifold1m_d64_k50", (0.01, 0.004), "bf16", False, True),
]


def _trees(ref, q, leaf):
    import torch
    from paper_1304_4327_amd import knn
    rt = knn.knn_build_tree(torch.from_numpy(ref).cuda(), leaf)
    qt = None if q is None else knn.knn_build_tree(torch.from_numpy(q).cuda(), leaf)
    return rt, qt


@pytest.mark.parametrize("name,scales,precision,self_mode,seeded", CASES)
def test_noalloc_matches_knn_search_twice(name, scales, precision, self_mode, seeded):
    import torch
    from paper_1304_4327_amd import knn
    for call, scale in enumerate(scales):
        ref, q, k, leaf = datagen.make(name, scale=scale)
        print(f"no-alloc call {call}: {name} scale {scale} {precision} seeded={seeded}",
              flush=True)
        rt, qt = _trees(ref, q, leaf)
        nq = len(ref) if q is None else len(q)
        seed = None
        if seeded:
            nl = (qt or rt).info()["n_leaves"]
            rng = np.random.default_rng(call)
            seed = torch.from_numpy(np.where(rng.random(nl) < 0.3, 0.0, np.inf)
                                    .astype(np.float32)).cuda()
        want = knn.knn_search(rt, qt, k, precision=precision, exclude_self=self_mode,
                              seed_radius=seed, stats=True)
        out = (torch.full((nq, k), -7, dtype=torch.int64, device="cuda"),
               torch.full((nq, k), -7.0, dtype=torch.float32, device="cuda"))
        got = knn.knn_search_noalloc(rt, qt, k, out, precision=precision,
                                     exclude_self=self_mode, seed_radius=seed, stats=True)
        torch.cuda.synchronize()
        assert torch.equal(got[0], want[0]) and torch.equal(got[1], want[1])
        same_kernel = not (precision == "bf16" and ref.shape[1] > 32)
        keys = ("score_calls", "pairs", "inserts") if same_kernel else ()
        for key in keys + ("fallback_leaves", "fallback_queries"):
            assert got[2][key] == want[2][key], key
        if seeded:
            assert got[2]["fallback_leaves"] > 0
        if call == 1:
            qq = ref if q is None else q
            oi, od = ok.knn(qq, ref, k, exclude_self=self_mode)
            parity.assert_ok(qq, ref, k, got[0].cpu().numpy(), got[1].cpu().numpy(), oi, od,
                             exclude_self=self_mode)


def test_noalloc_rejects_a_query_tree_beyond_its_scratch():
    import torch
    from paper_1304_4327_amd import knn
    ref = datagen.uniform(4096, 3, 1)
    q = datagen.uniform(1 << 19, 3, 2)
    rt, qt = _trees(ref, q, 1)
    assert qt.info()["n_leaves"] == 1 << 19
    out = (torch.empty((1 << 19, 4), dtype=torch.int64, device="cuda"),
           torch.empty((1 << 19, 4), dtype=torch.float32, device="cuda"))
    seed = torch.zeros(1 << 19, dtype=torch.float32, device="cuda")
    with pytest.raises(knn.KnnError) as e:
        knn.knn_search_noalloc(rt, qt, 4, out, seed_radius=seed)
    assert e.value.status == knn.KNN_E_INVALID_ARG
    # without a seed the same tree fits (4 bytes per wavefront of 8 leaves)
    knn.knn_search_noalloc(rt, qt, 4, out)
    want = knn.knn_search(rt, qt, 4)
    assert torch.equal(out[0], want[0]) and torch.equal(out[1], want[1])
