"""GPU parity of the CDF-model kernels against the fp64 oracle, and of the
learned / linear co-rank modes against the oracle (results must be exact).

Tolerances (fp32 kernels vs fp64 oracle): a forward value is a chain of two
32-term fp32 dot products, so its error is a few hundred units of 2^-24
relative to the sum of |terms|; a gradient entry adds a sum over the batch in
chunks of 128 then over the chunks, so its error is bounded by about
(128 + B/128 + 100) * 2^-24 * sum_b |term_b|.  The tests use the per-entry
bound 1e-4 * (sum_b |term_b|) computed by the oracle side, with room to spare
(B = 4096 gives about 1.6e-5)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_03970_amd as hv
from oracle import mlp
from paper_2409_03970_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _p32(seed, scale=1.0):
    return (inputs.mlp_init(seed) * scale).to(DEV)


def _batch(b, seed):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0, 1, b)).astype(np.float32)
    t = (np.arange(b) / b).astype(np.float32)
    return x, t


def _abs_terms(p, x, t):
    """sum_b |per-sample term| of every gradient entry, in fp64."""
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    y, (x, z1, h1, z2, h2) = mlp.forward(p, x)
    B = x.shape[0]
    dy = 2.0 * (y - t) / B
    dz2 = np.outer(dy, W3) * (z2 > 0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    a = np.abs
    return np.concatenate([a(dz1).T @ a(x), a(dz1).sum(0), (a(dz2).T @ a(h1)).reshape(-1),
                           a(dz2).sum(0), a(h2).T @ a(dy), [a(dy).sum()]])


def test_forward_matches_oracle():
    p = _p32(1)
    x = torch.linspace(0, 1, 10000, device=DEV, dtype=torch.float32)
    y = hv.cdf_forward(p, x).cpu().numpy()
    want, _ = mlp.forward(p.cpu().double().numpy(), x.cpu().double().numpy())
    assert np.max(np.abs(y - want)) <= 1e-5 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("b", [1, 127, 128, 129, 4096, 65536])
def test_backward_matches_oracle(b):
    p = _p32(2)
    x, t = _batch(b, b)
    loss, g = hv.cdf_backward(p, torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV))
    pd = p.cpu().double().numpy()
    L, g64 = mlp.backward(pd, x.astype(np.float64), t.astype(np.float64))
    bound = 1e-4 * _abs_terms(pd, x.astype(np.float64), t.astype(np.float64)) + 1e-12
    err = np.abs(g.cpu().double().numpy() - g64)
    assert np.all(err <= bound), (np.argmax(err / bound), err.max())
    assert abs(loss - L) <= 1e-4 * max(L, 1e-12)


def test_backward_is_deterministic():
    p = _p32(3)
    x, t = _batch(70000, 3)
    xd, td = torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)
    l1, g1 = hv.cdf_backward(p, xd, td)
    l2, g2 = hv.cdf_backward(p, xd, td)
    assert l1 == l2 and torch.equal(g1, g2)


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(4)
    p = torch.from_numpy(rng.normal(0, 0.3, mlp.N_PARAMS).astype(np.float32)).to(DEV)
    m = torch.from_numpy(rng.normal(0, 0.01, mlp.N_PARAMS).astype(np.float32)).to(DEV)
    v = torch.from_numpy(rng.uniform(0, 1e-3, mlp.N_PARAMS).astype(np.float32)).to(DEV)
    g = torch.from_numpy(rng.normal(0, 0.1, mlp.N_PARAMS).astype(np.float32)).to(DEV)
    p0, m0, v0 = (a.cpu().double().numpy() for a in (p, m, v))
    hv.cdf_adam_step(p, m, v, g, step=7, lr=1e-3)
    gd = g.cpu().double().numpy()
    pw, mw, vw = mlp.adam_step(p0, m0, v0, gd, step=7, lr=1e-3)
    # the kernel holds beta1, beta2, 1 - beta1 and 1 - beta2 in fp32 (0.9f is
    # 2.7e-8 off, 1 - 0.9f 2.4e-7 off relative) and rounds each of its few
    # operations once, so each moment is within ~5e-7 of its terms' sizes
    assert np.all(np.abs(m.cpu().double().numpy() - mw) <= 5e-7 * (np.abs(m0) + np.abs(gd)))
    assert np.all(np.abs(v.cpu().double().numpy() - vw) <= 5e-7 * (np.abs(v0) + gd * gd))
    # the step lr * mhat / (sqrt(vhat) + eps) inherits ~1e-6 relative error,
    # plus one rounding of the parameter itself
    step = np.abs(pw - p0)
    assert np.all(np.abs(p.cpu().double().numpy() - pw) <= 1e-5 * step + 1.2e-7 * np.abs(p0))


def _splitmix64(seed, counter):
    # output `counter` (from 0) of SplitMix64 seeded with `seed`
    M = (1 << 64) - 1
    z = (seed + (counter + 1) * 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_sample_kernel_positions():
    keys = torch.arange(1000003, device=DEV, dtype=torch.int32) * 3 - 7
    s = hv.cdf_sample(keys, 5000, seed=12345).cpu().numpy()
    want = np.array([(_splitmix64(12345, k) % 1000003) * 3 - 7 for k in range(5000)], np.int64)
    assert np.array_equal(s.astype(np.int64), want)


def test_one_training_step_matches_oracle():
    m_keys = 20000
    sorted_keys = oracle.sort(inputs.keys(m_keys, "mixture", seed=5).numpy())
    p = _p32(5)
    p0 = p.cpu().double().numpy()
    batch, seed = 2048, 77
    hv.cdf_train(p, torch.from_numpy(sorted_keys).to(DEV), batch=batch, steps=1, lr=1e-3, seed=seed)
    idx = np.array([_splitmix64(seed, k) % m_keys for k in range(batch)])
    x = ((sorted_keys[idx].astype(np.float64) + 2**31) / 2**32).astype(np.float32).astype(np.float64)
    t = (idx / m_keys).astype(np.float32).astype(np.float64)
    _, g = mlp.backward(p0, x, t)
    want, _, _ = mlp.adam_step(p0, np.zeros_like(p0), np.zeros_like(p0), g, step=1, lr=1e-3)
    # each parameter moves by almost exactly lr against the sign of its
    # gradient; entries whose gradient is tiny may differ in sign by rounding
    got = p.cpu().double().numpy()
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.allclose(got[big], want[big], rtol=0, atol=1e-6)
    assert np.all(np.abs(got - p0) <= 1e-3 * (1 + 1e-5))


def test_training_reduces_loss():
    keys = inputs.keys(1 << 20, "mixture", seed=6, device=DEV)
    sample = hv.sort(hv.cdf_sample(keys, 1 << 16, seed=6))
    p = _p32(6)
    x = ((sample.double() + 2**31) / 2**32).float()
    t = torch.arange(sample.numel(), device=DEV, dtype=torch.float32) / sample.numel()
    l0, _ = hv.cdf_backward(p, x, t)
    hv.cdf_train(p, sample, batch=8192, steps=300, lr=3e-3, seed=6)
    l1, _ = hv.cdf_backward(p, x, t)
    assert l1 < 0.05 * l0, (l0, l1)


# ---------------------------------------------------- learned co-rank modes

@pytest.mark.parametrize("dist", ["uniform", "sorted", "reverse", "mixture", "zipf"])
def test_learned_sort_is_exact(dist):
    n = 3_000_001
    x = inputs.keys(n, dist, seed=8, device=DEV)
    params = hv.fit_cdf_model(x, frac=0.01, steps=200, batch=8192, lr=3e-3, seed=8)
    want = oracle.sort(x.cpu().numpy())
    for mode in (hv.CORANK_LEARNED, hv.CORANK_LINEAR):
        st = torch.zeros(hv.STATS_WORDS, dtype=torch.int64, device=DEV)
        y = hv.sort(x, opts={"corank_mode": mode, "cdf_params": params, "radius_log2": 10,
                             "stats": st})
        assert np.array_equal(y.cpu().numpy(), want), mode
        assert int(st[0]) > 0


def test_full_size_2pow30_learned():
    # the learned co-rank's own configuration: 2^30 mixture keys, the CDF
    # model trained on the GPU from a 1 % sample, learned co-ranks with the
    # bounded search (radius 2^13) in the best two-way launch shape (every
    # co-rank predicted), element by element against the oracle (run in
    # parts on the host); the linear and binary modes, and the tuned
    # four-way shape in every mode, must give the identical array
    import oracle_parts
    from paper_2409_03970_amd import tune
    n = 1 << 30
    print("full size 2^30 learned", flush=True)
    x = inputs.keys(n, "mixture", seed=0, device=DEV)
    params = hv.fit_cdf_model(x, frac=0.01, steps=400, batch=65536, lr=3e-3, seed=2)
    two = dict(tune.tuned_options("sort", n, two_way=True) or {}, merge_ways=2)
    st = torch.zeros(hv.STATS_WORDS, dtype=torch.int64, device=DEV)
    y = hv.sort(x, opts=dict(two, corank_mode=hv.CORANK_LEARNED, cdf_params=params,
                             radius_log2=13, stats=st))
    torch.cuda.synchronize()
    s = hv.corank_stats(st.cpu())
    assert s["coranks"] > 0 and s.get("predicted", 0) > 0
    want = oracle_parts.sort_in_parts(x.cpu().numpy(), parts=16, threads=16)
    assert np.array_equal(y.cpu().numpy(), want)
    del want
    four = dict(tune.tuned_options("sort", n) or {})
    for opts, mode in ((two, hv.CORANK_LINEAR), (two, hv.CORANK_BINARY),
                       (four, hv.CORANK_LEARNED), (four, hv.CORANK_BINARY)):
        y2 = hv.sort(x, opts=dict(opts, corank_mode=mode, cdf_params=params, radius_log2=13))
        assert torch.equal(y2, y), (opts.get("merge_ways"), mode)
        del y2


def test_learned_prediction_exact_on_disjoint_runs():
    # already sorted input: every pair of runs has disjoint key ranges, so the
    # model's breakpoints give every co-rank exactly (no fallback), while the
    # linear prediction is off by half a diagonal
    n = 1 << 22
    x = inputs.keys(n, "sorted", seed=9, device=DEV)
    params = hv.fit_cdf_model(x, frac=0.01, steps=300, batch=8192, lr=3e-3, seed=9)
    res = {}
    for mode in (hv.CORANK_LEARNED, hv.CORANK_LINEAR, hv.CORANK_BINARY):
        st = torch.zeros(hv.STATS_WORDS, dtype=torch.int64, device=DEV)
        y = hv.sort(x, opts={"corank_mode": mode, "cdf_params": params, "radius_log2": 8,
                             "stats": st})
        assert torch.equal(y, x)
        res[mode] = st.cpu().tolist()
    learned, linear, binary = res[hv.CORANK_LEARNED], res[hv.CORANK_LINEAR], res[hv.CORANK_BINARY]
    assert learned[2] < linear[2]                   # fewer fallbacks
    assert learned[1] < binary[1]                   # fewer probes than binary search
    # the error statistics cover the predicted co-ranks only: on disjoint
    # runs every prediction is exact
    assert learned[5] > 0 and learned[4] == 0 and learned[3] == 0
    assert sum(learned[72:136]) == learned[5] == learned[72]


def _check_histograms(w, mode, predicts=True):
    # predicts: the sort has two-way co-ranks (four-way ones use no prediction)
    n = w[0]
    ph, eh = w[8:72], w[72:136]
    assert sum(ph) == n                                         # every co-rank in one bin
    if ph[63] == 0:
        assert sum(p * h for p, h in enumerate(ph)) == w[1]      # exact probe total
    if mode == hv.CORANK_BINARY or (not predicts and w[5] == 0):
        assert w[5] == 0 and sum(eh) == 0 and w[2] == w[3] == w[4] == 0
        return
    assert 0 < w[5] <= n and sum(eh) == w[5] and w[2] <= w[5]
    top = max(b for b, h in enumerate(eh) if h)                 # highest error bin
    assert top == int(w[4]).bit_length()
    lo = sum(h << (b - 1) for b, h in enumerate(eh) if b)        # error sum bounds
    hi = sum(h * ((1 << b) - 1) for b, h in enumerate(eh))
    assert lo <= w[3] <= hi


@pytest.mark.parametrize("dist", ["uniform", "mixture", "distinct16"])
@pytest.mark.parametrize("ways", [2, 4])
def test_corank_histograms_are_consistent(dist, ways):
    n = 2_000_003
    x = inputs.keys(n, dist, seed=12, device=DEV)
    params = hv.fit_cdf_model(x, frac=0.01, steps=150, batch=8192, lr=3e-3, seed=12)
    want = oracle.sort(x.cpu().numpy())
    for mode in (hv.CORANK_BINARY, hv.CORANK_LEARNED, hv.CORANK_LINEAR):
        st = torch.zeros(hv.STATS_WORDS, dtype=torch.int64, device=DEV)
        y = hv.sort(x, opts={"corank_mode": mode, "cdf_params": params, "radius_log2": 9,
                             "stats": st, "merge_ways": ways})
        assert np.array_equal(y.cpu().numpy(), want)
        w = st.cpu().tolist()
        assert w[0] > 0
        _check_histograms(w, mode, predicts=ways == 2)
        s = hv.corank_stats(w)
        assert s["probes_p99"] is not None and s["probes_p99"] * 1.0 >= 0


def test_corank_list_learned_matches_oracle():
    rng = np.random.default_rng(10)
    A = np.sort(rng.integers(0, 1000, 5000)).astype(np.int32)
    B = np.sort(rng.integers(500, 3000, 7000)).astype(np.int32)
    keys = torch.from_numpy(np.concatenate([A, B])).to(DEV)
    params = hv.fit_cdf_model(keys, frac=0.5, steps=200, batch=4096, lr=3e-3, seed=10)
    diag = np.arange(0, A.size + B.size + 1, dtype=np.int64)
    got = hv.corank(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV),
                    torch.from_numpy(diag).to(DEV),
                    opts={"corank_mode": hv.CORANK_LEARNED, "cdf_params": params,
                          "radius_log2": 5}).cpu().numpy()
    want = [oracle.corank(A, B, int(d)) for d in diag[::7]]
    assert got[::7].tolist() == want
