"""The learned CDF bucket path on the GPU.

Network: forward, loss and gradient of the device kernels against the fp64
oracle (norm-wise relative error per parameter tensor), one Adam step against
the oracle's Adam on the oracle's gradient, and training lowering the loss.
Sort: bit-exact parity with the oracle on the learned workloads and on ties,
signed zeros and NaNs; heavy values (buckets of their own for the sample's
long runs of equal keys, next to neighbouring doubles, signed zeros and
infinities); the fallback paths (non-monotone table via the test hook, a
bucket above the limit, a degenerate sample); and a gain test: the trained
network balances buckets better than the untrained linear CDF.
"""
import math

import numpy as np
import pytest

import workloads as W
from gpu_util import multiset_hash_dev, announce, bits, need_gpu, to_dev

pytestmark = pytest.mark.gpu

TENSORS = ("W1", "b1", "W2", "b2", "w3", "b3")


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2402_01816_amd as g
    return g


def _he_params(orc, seed):
    rng = np.random.default_rng(seed)
    sl = orc.mlp_slices()
    p = np.zeros(orc.MLP_NUM_PARAMS)
    p[sl["W1"]] = rng.normal(0, math.sqrt(2.0), 64)
    p[sl["b1"]] = rng.normal(0, 0.2, 64)
    p[sl["W2"]] = rng.normal(0, math.sqrt(2.0 / 64), 64 * 64)
    p[sl["b2"]] = rng.normal(0, 0.2, 64)
    p[sl["w3"]] = rng.normal(0, math.sqrt(2.0 / 64), 64)
    p[sl["b3"]] = rng.normal(0, 0.2, 1)
    return p.astype(np.float32)


def _batch(seed, n):
    rng = np.random.default_rng(seed)
    u = rng.random(n).astype(np.float32)
    t = np.sqrt(u).astype(np.float32)          # a CDF-like target
    return u, t


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("batch", [32, 256, 2048])
def test_gradient_matches_oracle(gs, orc, batch):
    announce("mlp grad", batch)
    p = _he_params(orc, batch)
    u, t = _batch(batch + 1, batch)
    loss, grad = gs.gs_mlp_loss_grad(to_dev(p), to_dev(u), to_dev(t))
    ref_loss, ref_grad = orc.mlp_loss_grad(p.astype(np.float64), u.astype(np.float64), t.astype(np.float64))
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * max(1.0, abs(ref_loss))
    g = grad.cpu().numpy().astype(np.float64)
    for name, sl in orc.mlp_slices().items():
        assert _relerr(g[sl], ref_grad[sl]) <= 1e-4, name
        # entry by entry too, so that a wrong entry cannot hide in the norm
        # of a large tensor (W2 has 4,096): fp32 sums of at most 2048 terms
        scale = np.max(np.abs(ref_grad[sl]))
        assert np.max(np.abs(g[sl] - ref_grad[sl])) <= 1e-4 * scale, name


def test_forward_matches_oracle(gs, orc):
    announce("mlp forward")
    p = _he_params(orc, 7)
    u = np.linspace(-0.5, 1.5, 4099).astype(np.float32)
    y = gs.gs_mlp_forward(to_dev(p), to_dev(u)).cpu().numpy()
    ref = orc.mlp_forward(p.astype(np.float64), u.astype(np.float64))
    assert np.max(np.abs(y - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))


def test_adam_step_matches_oracle(gs, orc):
    torch = need_gpu()
    announce("mlp adam")
    p = _he_params(orc, 9)
    u, t = _batch(10, 512)
    P, M, V = to_dev(p), torch.zeros(p.size, device="cuda"), torch.zeros(p.size, device="cuda")
    losses = gs.gs_mlp_train(P, M, V, to_dev(u), to_dev(t), steps=1, batch=512, lr=1e-3,
                             full_batch=True)
    _, g = orc.mlp_loss_grad(p.astype(np.float64), u.astype(np.float64), t.astype(np.float64))
    ref = p.astype(np.float64).copy()
    m, v = np.zeros_like(ref), np.zeros_like(ref)
    orc.adam_step(ref, g, m, v, 1, lr=1e-3)
    got = P.cpu().numpy().astype(np.float64)
    upd, ref_upd = got - p, ref - p
    big = np.abs(g) > 1e-5                        # |g| >> eps: update is lr*sign(g)
    assert np.allclose(upd[big], ref_upd[big], rtol=1e-3, atol=1e-7)
    assert np.all(np.abs(upd) <= 1e-3 + 1e-6)
    assert _relerr(M.cpu().numpy().astype(np.float64), 0.1 * g) <= 1e-4
    assert _relerr(V.cpu().numpy().astype(np.float64), 0.001 * g * g) <= 1e-3
    assert float(losses[0].item()) > 0


def test_training_lowers_loss(gs, orc):
    torch = need_gpu()
    announce("mlp train")
    p = _he_params(orc, 11)
    u, t = _batch(12, 65536)
    P, M, V = to_dev(p), torch.zeros(p.size, device="cuda"), torch.zeros(p.size, device="cuda")
    losses = gs.gs_mlp_train(P, M, V, to_dev(u), to_dev(t), steps=200, batch=2048, lr=1e-2, seed=3)
    first, last = (float(x) for x in losses.cpu().numpy())
    assert last < 0.05 * first
    # same seed, same result: the reductions are deterministic
    P2, M2, V2 = to_dev(p), torch.zeros(p.size, device="cuda"), torch.zeros(p.size, device="cuda")
    gs.gs_mlp_train(P2, M2, V2, to_dev(u), to_dev(t), steps=200, batch=2048, lr=1e-2, seed=3)
    assert torch.equal(P, P2)


N_SMALL = 1 << 20


def _learned(gs, x, report=True, **kw):
    t = to_dev(x)
    rep = gs.gs_learned_sort(t, report=report, **kw)
    return t, rep


@pytest.mark.parametrize("pattern", ["lognormal", "gaussmix", "zipf_ints"])
def test_learned_sort_parity(gs, orc, pattern):
    announce("learned", pattern)
    x = W.learned_pattern(pattern, N_SMALL + 12345, seed=1)
    t, rep = _learned(gs, x, sample_size=16384)
    assert rep["fallback"] == 0
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    if pattern == "zipf_ints":
        # the most frequent integers fill long runs of the sorted sample; with
        # the runs left out of the density targets the rest is nearly flat
        # (the untrained network's zero output already fits it: no spikes)
        assert rep["heavy_values"] == 31
        assert rep["train_loss_last"] < 1.0
    else:
        assert rep["train_loss_last"] < rep["train_loss_first"]
    if pattern == "lognormal":
        assert rep["heavy_values"] == 0


def _heavy_input(case, n, seed):
    """Uniform keys in [-2, 2) with runs of equal keys laid over them (by the
    fraction of keys each value holds)."""
    rng = np.random.default_rng(seed)
    x = rng.random(n) * 4.0 - 2.0
    u = rng.random(n)
    v = 0.25
    if case == "edges":
        zeros = np.where(rng.random(n) < 0.5, -0.0, 0.0)
        runs = [(zeros, 0.12), (v, 0.08), (np.nextafter(v, 1.0), 0.05), (np.nextafter(v, 0.0), 0.04),
                (np.inf, 0.03), (-1.5, 0.02)] + [(1.0 + j / 16.0, 0.01) for j in range(12)]
    else:                                        # ten values holding 7% each
        runs = [(-1.0 + j / 8.0, 0.07) for j in range(10)]
    lo = 0.0
    for val, frac in runs:
        x = np.where((u >= lo) & (u < lo + frac), val, x)
        lo += frac
    x[rng.integers(0, n, 200)] = np.nan
    return x


@pytest.mark.parametrize("case,buckets,heavy", [("edges", 4096, 18), ("edges", 64, 2), ("cap", 64, 8)])
def test_learned_heavy_values_edges(gs, orc, case, buckets, heavy):
    """Heavy values (sample runs of at least 4 average buckets' share) beside
    their nearest doubles, the heavy value 0 held by both -0.0 and +0.0
    (equal keys: their input order is kept), +inf as the largest heavy value,
    NaNs: each heavy value's bucket holds that value alone and is not sorted,
    so stability and the neighbours' buckets are what this checks, bit for
    bit.  With 64 buckets a run must hold 1/16 of the sample and at most 8
    heavy values are taken (the longest runs); the rest are sorted in
    ordinary buckets."""
    announce("learned heavy", case, buckets)
    x = _heavy_input(case, N_SMALL + 777, 21)
    t, rep = _learned(gs, x, sample_size=16384, num_buckets=buckets)
    assert rep["fallback"] == 0
    assert rep["heavy_values"] == heavy
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


@pytest.mark.parametrize("pattern", ["uniform", "tied", "presorted", "reversed", "zeros_signed"])
def test_learned_sort_other_patterns(gs, orc, pattern):
    announce("learned other", pattern)
    x = W.f64_pattern(pattern, N_SMALL - 3, seed=2)
    t, rep = _learned(gs, x, sample_size=16384)
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_learned_sort_special_values(gs, orc):
    announce("learned special")
    x = W.learned_pattern("gaussmix", N_SMALL, seed=3)
    rng = np.random.default_rng(4)
    idx = rng.integers(0, x.size, 5000)
    x[idx[:1000]] = np.nan
    x[idx[1000:2000]] = np.inf
    x[idx[2000:3000]] = -np.inf
    x[idx[3000:4000]] = -0.0
    x[idx[4000:]] = 0.0
    t, rep = _learned(gs, x, sample_size=16384)
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_learned_many_long_runs(gs, orc):
    """300 values holding 0.25 % of the keys each: more long runs of equal keys
    than the sample pass records (256).  With the screening on, the runs it
    could not see send the call to the plain path (fallback 2); with it off,
    31 of the recorded runs become heavy values and the rest are sorted in
    ordinary buckets.  Bit for bit the definition's result either way."""
    announce("learned many runs")
    n = N_SMALL + 99
    rng = np.random.default_rng(23)
    x = rng.random(n)
    vals = rng.random(300)
    pick = rng.random(n) < 0.75
    x[pick] = vals[rng.integers(0, 300, int(pick.sum()))]
    t, rep = _learned(gs, x, sample_size=16384)
    assert rep["fallback"] == 2
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    t, rep = _learned(gs, x, sample_size=16384, screen=1)
    assert rep["fallback"] == 0 and rep["heavy_values"] == 31
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


@pytest.mark.parametrize("pattern", ["lognormal", "gaussmix", "zipf_ints"])
def test_learned_sample_table_parity(gs, orc, pattern):
    """Mode 2: the knot table is the sorted sample's CDF at the knots (no
    network); bit for bit the definition's result."""
    announce("learned mode2", pattern)
    x = W.learned_pattern(pattern, N_SMALL + 4321, seed=15)
    t, rep = _learned(gs, x, sample_size=16384, mode=2)
    assert rep["fallback"] == 0 and rep["feature"] & 2
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_learned_rescue_by_sample_table(gs, orc):
    """A network whose log density is -200 u puts nearly every key into the
    last bucket.  The screening on the sample sees it and replaces the table
    by the sample's CDF at the knots, which spreads the keys: the learned path
    still sorts (fallback 0, feature bit 1), bit for bit.  Without the
    screening the full bucket totals reject the network's table instead."""
    announce("learned rescue")
    n = 1 << 22
    x = W.learned_pattern("gaussmix", n, seed=14)
    sl = orc.mlp_slices()
    p = np.zeros(orc.MLP_NUM_PARAMS, np.float32)
    p[sl["W1"].start] = 1.0                     # h1[0] = relu(u)
    p[sl["W2"].start] = 1.0                     # h2[0] = h1[0]
    p[sl["w3"].start] = -200.0                  # log density -200 u
    P = to_dev(p)
    t, rep = _learned(gs, x, weights_override=P.data_ptr())
    assert rep["fallback"] == 0 and rep["feature"] & 2
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    t, rep = _learned(gs, x, weights_override=P.data_ptr(), screen=1)
    assert rep["fallback"] == 1 and rep["overflow_buckets"] > 0 and not rep["feature"] & 2
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_learned_untrained_mode(gs, orc):
    announce("learned mode1")
    x = W.learned_pattern("lognormal", N_SMALL, seed=5)
    t, rep = _learned(gs, x, sample_size=16384, mode=1)
    assert rep["fallback"] == 0
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_learned_weights_override(gs, orc):
    announce("learned override")
    p = _he_params(orc, 13)
    x = W.learned_pattern("zipf_ints", N_SMALL, seed=6)
    P = to_dev(p)
    t, rep = _learned(gs, x, sample_size=16384, weights_override=P.data_ptr())
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_learned_fallback_on_order_violation(gs, orc):
    """A non-monotone raw bucket table (test hook) must be rejected before any
    key moves; the plain path then sorts the untouched input."""
    announce("learned fallback order")
    params = gs.gs_learned_default_params()
    G = params.knots
    table = np.linspace(1.0, 0.0, G + 1).astype(np.float32)        # decreasing
    T = to_dev(table)
    x = W.learned_pattern("gaussmix", N_SMALL, seed=7)
    t, rep = _learned(gs, x, sample_size=16384, test_bucket_table=T.data_ptr())
    assert rep["fallback"] == 1
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_learned_fallback_on_overflow(gs, orc):
    """60% of a 2^22-key input in an interval of width 1e-9 (distinct keys, so
    no heavy value; far narrower than a knot) puts more than the bucket limit
    (2^20) into one bucket of each half.  The sample predicts it, so the
    plain path takes the call before any key moves (fallback 2); with that
    early screening off, the check on the full bucket totals catches it
    (fallback 1).  Either way the result is the plain sort's."""
    announce("learned fallback overflow")
    n = 1 << 22
    x = W.f64_pattern("uniform", n, seed=8)
    rng = np.random.default_rng(9)
    spike = rng.random(n) < 0.6
    x[spike] = 0.5 + rng.random(int(spike.sum())) * 1e-9
    t, rep = _learned(gs, x, sample_size=16384)
    assert rep["fallback"] == 2 and rep["max_bucket"] > (1 << 20)
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    t, rep = _learned(gs, x, sample_size=16384, screen=1)
    assert rep["fallback"] == 1 and rep["overflow_buckets"] > 0
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


@pytest.mark.parametrize("pattern", ["gaussmix", "zipf_ints"])
def test_learned_uneven_inputs_at_full_size(gs, orc, pattern):
    """The trained network may leave the narrowest Gaussian component in too
    few buckets: then the screening on the sample replaces its table by the
    sample's CDF at the knots (at 2^28 keys it does).  The Zipf integers' most frequent
    values take buckets of their own (a tenth of the keys are the most
    frequent one) and the rest stay within the limit.  The learned path sorts
    both; sortedness, the multiset and sampled oracle ranks fix the result."""
    torch = need_gpu()
    n = 1 << 26
    announce("learned uneven", pattern, n)
    x = W.learned_pattern(pattern, n, seed=0)
    t, rep = _learned(gs, x)
    assert rep["fallback"] == 0
    if pattern == "zipf_ints":
        assert rep["heavy_values"] == 31
    h = multiset_hash_dev(torch.from_numpy(x).to("cuda"))
    assert multiset_hash_dev(t) == h
    assert bool((t[1:] >= t[:-1]).all().item())
    rng = np.random.default_rng(3)
    idx = np.concatenate([[0, n - 1], rng.integers(0, n, 14)])
    got = t[torch.from_numpy(orc.rank_f64(x, idx)).to("cuda")].cpu().numpy()
    assert np.array_equal(bits(got), bits(x[idx]))


def test_learned_full_size_lognormal(gs, orc):
    """The learned workload at its full size, 2^28 lognormal(0, 2) keys: the
    trained table spreads them (no fallback), and sortedness, the multiset and
    sampled positions from the oracle's counting form fix the result."""
    torch = need_gpu()
    n = 1 << 28
    announce("learned full", "lognormal", n)
    x = W.learned_pattern("lognormal", n, seed=0)
    t, rep = _learned(gs, x)
    assert rep["fallback"] == 0
    h = multiset_hash_dev(torch.from_numpy(x).to("cuda"))
    assert multiset_hash_dev(t) == h
    assert bool((t[1:] >= t[:-1]).all().item())
    rng = np.random.default_rng(4)
    idx = np.concatenate([[0, n - 1], rng.integers(0, n, 14)])
    got = t[torch.from_numpy(orc.rank_f64(x, idx)).to("cuda")].cpu().numpy()
    assert np.array_equal(bits(got), bits(x[idx]))


def test_learned_degenerate_all_equal(gs, orc):
    announce("learned all equal")
    x = np.full(N_SMALL, 3.25)
    x[::7] = -0.0 + 3.25
    t, rep = _learned(gs, x, sample_size=16384)
    assert rep["fallback"] == 1
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_learned_small_input_runs_plain(gs, orc):
    announce("learned small")
    for n in (0, 1, 2, 1000, 65535):
        x = W.f64_pattern("zeros_signed", n, seed=10)
        t, rep = _learned(gs, x)
        assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


@pytest.mark.parametrize("p", [0.25, 1 / 64])
def test_learned_small_buffer_runs_plain(gs, orc, p):
    """Below buffer fraction 0.5 the distribution passes' half buffer does not
    fit: the plain sort at that fraction sorts (fallback 3), within the
    caller's memory bound."""
    announce("learned small buffer", p)
    x = W.learned_pattern("lognormal", (1 << 21) + 77, seed=12)
    x[::301] = -0.0
    x[::307] = 0.0
    t, rep = _learned(gs, x, buffer_fraction=p)
    assert rep["fallback"] == 3
    assert rep["ram_fraction"] < 1 + p + 0.02
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_learned_gain_over_untrained(gs):
    """On lognormal keys the trained network spreads keys over the buckets
    far more evenly than the untrained linear CDF on the same feature."""
    announce("learned gain")
    x = W.learned_pattern("lognormal", 1 << 22, seed=11)
    _, trained = _learned(gs, x)
    _, untrained = _learned(gs, x, mode=1)
    assert trained["fallback"] == 0 and untrained["fallback"] == 0
    avg = (1 << 22) / 2 / 4096
    assert trained["max_bucket"] < 0.5 * untrained["max_bucket"]
    assert trained["max_bucket"] < 4 * avg


@pytest.mark.parametrize("pattern,n", [("lognormal", 1 << 20), ("zipf_ints", 1 << 24)])
def test_learned_graph_capture(gs, orc, pattern, n):
    """Captured into a graph, the call keeps its decision on the device (both
    paths enqueued, gated); every replay on a freshly restored input gives
    the definition's result."""
    torch = need_gpu()
    announce("learned capture", pattern, n)
    x = W.learned_pattern(pattern, n, seed=12)
    src = to_dev(x)
    t = torch.empty_like(src)
    p = gs.gs_learned_default_params()
    p.sample_size = 16384
    need = gs.gs_workspace_bytes_learned(n, p)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    ws = ws[(-ws.data_ptr()) % 256:][:need]
    t.copy_(src)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        g.capture_begin()
        try:
            gs.gs_learned_sort(t, p, workspace=ws, stream=s)
        finally:
            g.capture_end()
    ref = bits(orc.sort_f64(x))
    for _ in range(3):
        t.copy_(src)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(bits(t), ref)
