"""Seeded synthetic workloads for the sort, shared by tests, benchmark and smoke.

This module holds none of the sort's arithmetic: it only draws keys, payloads,
segment sizes and initial model parameters.  Every generator is deterministic
for a given (seed, device); data drawn on different devices differ, so a test
draws once and hands the same array to both sides.

Workloads (the paper times random integers: 64K keys for its in-register and
merge tables, 2^9..2^27 keys for its overall sort rate, Sec. 3):
  uniform      keys uniform in [0, 2^31)
  gaussian     rint(N(2^30, 2^28)), clipped to [0, 2^31 - 1]
  sorted       the order statistics of a uniform draw (ascending)
  reverse      the same, descending
  distinct16   16 values drawn uniformly from [0, 2^31); each key uniform among them
  zipf         ranks r in 1..2^20 with P(r) proportional to r^-1.1; key = r - 1
  mixture      9 equal-weight components: 8 Gaussians (means uniform in
               [2^28, 2^31 - 2^28), sd = 2^U[18, 24]) and exp(N(20, 1.5));
               rint, clipped to [0, 2^31 - 1]
"""
import math

import torch

DISTRIBUTIONS = ("uniform", "gaussian", "sorted", "reverse", "distinct16", "zipf")
INT32_MAX = 2**31 - 1


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    return g


def _seed(*parts):
    """Fold a tuple of small integers into one 63-bit seed."""
    h = 0x243F6A8885A308D3
    for p in parts:
        h = (h * 6364136223846793005 + int(p) + 1442695040888963407) & 0xFFFFFFFFFFFFFFFF
    return h & 0x7FFFFFFFFFFFFFFF


def _clip_round(x):
    return torch.clamp(torch.round(x), 0, INT32_MAX).to(torch.int32)


def keys(n, dist="uniform", seed=0, device="cpu"):
    """n int32 keys of the named distribution."""
    n = int(n)
    dev = torch.device(device)
    g = _gen(_seed(2, DISTRIBUTIONS.index(dist) if dist in DISTRIBUTIONS else 99, seed), dev)
    if n == 0:
        return torch.empty(0, dtype=torch.int32, device=dev)
    if dist == "uniform":
        return torch.randint(0, 2**31, (n,), generator=g, device=dev, dtype=torch.int64).to(torch.int32)
    if dist == "gaussian":
        x = torch.randn(n, generator=g, device=dev, dtype=torch.float64) * 2.0**28 + 2.0**30
        return _clip_round(x)
    if dist in ("sorted", "reverse"):
        # Order statistics of n uniforms: normalised partial sums of n + 1
        # exponential gaps (nondecreasing by construction, no sort needed).
        e = torch.empty(n + 1, device=dev, dtype=torch.float64).exponential_(1.0, generator=g)
        s = torch.cumsum(e, 0)
        u = s[:n] / s[n]
        k = torch.clamp(torch.floor(u * 2.0**31), 0, INT32_MAX).to(torch.int32)
        return torch.flip(k, (0,)) if dist == "reverse" else k
    if dist == "distinct16":
        vals = torch.randint(0, 2**31, (16,), generator=g, device=dev, dtype=torch.int64)
        idx = torch.randint(0, 16, (n,), generator=g, device=dev, dtype=torch.int64)
        return vals[idx].to(torch.int32)
    if dist == "zipf":
        r = torch.arange(1, 2**20 + 1, device=dev, dtype=torch.float64)
        cdf = torch.cumsum(r ** -1.1, 0)
        cdf = cdf / cdf[-1]
        u = torch.rand(n, generator=g, device=dev, dtype=torch.float64)
        rank0 = torch.searchsorted(cdf, u, right=True)
        return torch.clamp(rank0, 0, 2**20 - 1).to(torch.int32)
    if dist == "mixture":
        gp = _gen(_seed(4, 1, seed), torch.device("cpu"))
        means = 2.0**28 + torch.rand(8, generator=gp, dtype=torch.float64) * (2.0**31 - 2.0**29)
        sds = 2.0 ** (18.0 + 6.0 * torch.rand(8, generator=gp, dtype=torch.float64))
        comp = torch.randint(0, 9, (n,), generator=g, device=dev, dtype=torch.int64)
        z = torch.randn(n, generator=g, device=dev, dtype=torch.float64)
        mu = torch.cat([means, torch.tensor([20.0], dtype=torch.float64)]).to(dev)[comp]
        sd = torch.cat([sds, torch.tensor([1.5], dtype=torch.float64)]).to(dev)[comp]
        x = mu + sd * z
        lognormal = comp == 8
        x = torch.where(lognormal, torch.exp(torch.clamp(x, max=700.0)), x)
        return _clip_round(x)
    raise ValueError(f"unknown distribution {dist!r}")


def pairs(n, dist="uniform", seed=0, device="cpu"):
    """(keys, vals) with vals = 0..n-1, the original index of each key."""
    k = keys(n, dist, seed, device)
    v = torch.arange(int(n), device=k.device, dtype=torch.int32)
    return k, v


def segment_distributions(nseg, seed=0):
    """A distribution index in 0..5 (into DISTRIBUTIONS) for each segment."""
    g = _gen(_seed(6, seed, nseg), torch.device("cpu"))
    return torch.randint(0, len(DISTRIBUTIONS), (int(nseg),), generator=g)


def segment_pairs(sizes, dists, first_segment=0, seed=0, device="cpu"):
    """Keys and payloads of consecutive segments: segment s (numbered from
    first_segment) draws sizes[i] keys of DISTRIBUTIONS[dists[i]] from its own
    seed; its payload is the index within the segment."""
    ks, vs = [], []
    for i, (m, d) in enumerate(zip(sizes.tolist(), dists.tolist())):
        ks.append(keys(m, DISTRIBUTIONS[d], seed=_seed(5, seed, first_segment + i), device=device))
        vs.append(torch.arange(m, dtype=torch.int32, device=device))
    if not ks:
        e = torch.empty(0, dtype=torch.int32, device=device)
        return e, e.clone()
    return torch.cat(ks), torch.cat(vs)


def adversarial_keys(n, pattern, seed=0, device="cpu"):
    """Edge-case patterns: equal, two_values, extremes, organ_pipe, sawtooth, negatives."""
    n = int(n)
    dev = torch.device(device)
    g = _gen(_seed(7, seed, n), dev)
    i = torch.arange(n, device=dev, dtype=torch.int64)
    if pattern == "equal":
        return torch.full((n,), 12345, dtype=torch.int32, device=dev)
    if pattern == "two_values":
        return (torch.randint(0, 2, (n,), generator=g, device=dev) * 7 - 3).to(torch.int32)
    if pattern == "extremes":
        c = torch.tensor([-2**31, 2**31 - 1, 0, -1], dtype=torch.int64, device=dev)
        return c[torch.randint(0, 4, (n,), generator=g, device=dev)].to(torch.int32)
    if pattern == "organ_pipe":
        return torch.minimum(i, n - 1 - i).to(torch.int32)
    if pattern == "sawtooth":
        return (i % 97).to(torch.int32)
    if pattern == "negatives":
        return torch.randint(-2**31, 2**31, (n,), generator=g, device=dev, dtype=torch.int64).to(torch.int32)
    raise ValueError(f"unknown pattern {pattern!r}")


def log_uniform_sizes(nseg, lo, hi, seed=0):
    """nseg integer sizes floor(exp(U[ln lo, ln(hi + 1)))), clamped to [lo, hi]."""
    g = _gen(_seed(3, seed, nseg, lo, hi), torch.device("cpu"))
    u = torch.rand(int(nseg), generator=g, dtype=torch.float64)
    s = torch.floor(torch.exp(math.log(lo) + u * (math.log(hi + 1) - math.log(lo))))
    return torch.clamp(s, lo, hi).to(torch.int64)


def offsets_from_sizes(sizes):
    o = torch.zeros(sizes.numel() + 1, dtype=torch.int64)
    o[1:] = torch.cumsum(sizes.to(torch.int64), 0)
    return o


def mlp_init(seed=0):
    """Initial CDF-model parameters (1153 fp32), uniform(-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    g = _gen(_seed(5, seed), torch.device("cpu"))
    H = 32

    def u(size, fan_in):
        b = 1.0 / math.sqrt(fan_in)
        return (torch.rand(size, generator=g, dtype=torch.float64) * 2 - 1) * b

    parts = [u(H, 1), u(H, 1), u(H * H, H), u(H, H), u(H, H), u(1, H)]
    return torch.cat(parts).to(torch.float32)
