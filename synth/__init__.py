"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and shapes them into workloads; it holds
none of the set's arithmetic (no sorting network, codec, search or reduction of
the method).  Every stream is the counter-based splitmix64 generator
(Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014): value i of stream `seed` is mix64(seed + (i + 1) * golden_gamma).

Workload recipes follow the paper's experiments:
  * uniform 40-bit keys (Section "Evaluation on microbenchmarks", setup);
  * Zipf-distributed range lengths (skewed batch of queries);
  * R-MAT edges with a=0.5, b=c=0.1, d=0.3 (graph batch-insert setup);
  * Erdos-Renyi edges, uniform vertex pairs (the synthetic graph of the graph
    evaluation's datasets).
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
SEED_BASE = 0x230505055

MASK40 = (1 << 40) - 1


def splitmix64(seed, n, offset=0):
    """n consecutive outputs of the splitmix64 stream `seed`, starting at index offset."""
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_keys(n, seed, bits=40, offset=0):
    """n uniform keys of `bits` bits (duplicates possible)."""
    z = splitmix64(seed, n, offset)
    if bits < 64:
        z &= np.uint64((1 << bits) - 1)
    return z


def uniform_keys_at(idx, seed, bits=40):
    """The keys at positions idx of the uniform_keys stream `seed` (the stream
    is counter-based, so any position is drawn directly)."""
    with np.errstate(over="ignore"):
        i = np.asarray(idx, dtype=np.uint64) + np.uint64(1)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    if bits < 64:
        z &= np.uint64((1 << bits) - 1)
    return z


def unique_uniform_keys(n, seed, bits=40):
    """Exactly n distinct uniform keys of `bits` bits, returned in generation order.

    Draws n keys, drops repeats (keeping first occurrences) and tops up from the
    continuation of the same stream until n distinct keys exist.
    """
    keys = uniform_keys(n, seed, bits)
    _, first = np.unique(keys, return_index=True)
    if len(first) == n:
        return keys
    keep = keys[np.sort(first)]
    offset = n
    while len(keep) < n:
        need = n - len(keep)
        extra = uniform_keys(2 * need + 16, seed, bits, offset)
        offset += len(extra)
        cand = np.concatenate([keep, extra])
        _, first = np.unique(cand, return_index=True)
        keep = cand[np.sort(first)][:n]
    return keep


def sample_indices(n, k, seed):
    """k distinct indices in [0, n), uniformly at random (k <= n)."""
    if k > n:
        raise ValueError("k > n")
    if k == 0:
        return np.empty(0, dtype=np.int64)
    if 2 * k >= n:
        r = splitmix64(seed, n)
        return np.argsort(r, kind="stable")[:k].astype(np.int64)
    idx = np.empty(0, dtype=np.int64)
    offset = 0
    while len(idx) < k:
        r = splitmix64(seed, 2 * (k - len(idx)) + 16, offset)
        offset += len(r)
        cand = (r % np.uint64(n)).astype(np.int64)
        cat = np.concatenate([idx, cand])
        _, first = np.unique(cat, return_index=True)
        idx = cat[np.sort(first)]
    return idx[:k]


def uniform_float(n, seed, offset=0):
    """n doubles in [0, 1) from the top 53 bits of the stream."""
    z = splitmix64(seed, n, offset) >> np.uint64(11)
    return z.astype(np.float64) * (1.0 / (1 << 53))


def zipf_lengths(n, seed, alpha=1.2, lmax=10**6):
    """n lengths in {1..lmax} with P(l) proportional to l^-alpha (inverse-CDF table)."""
    ranks = np.arange(1, lmax + 1, dtype=np.float64)
    w = ranks ** (-alpha)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = uniform_float(n, seed)
    return (np.searchsorted(cdf, u, side="right") + 1).clip(1, lmax).astype(np.int64)


def zipf_zeta(N, theta, head=1 << 20):
    """zeta(N, theta) = sum_{i=1..N} i^-theta: the first `head` terms summed,
    the rest by the Euler-Maclaurin formula (the integral, the end terms and
    the first- and third-derivative corrections), which leaves an error far
    below double rounding for the smooth tail of i^-theta."""
    m = min(N, head)
    i = np.arange(1, m + 1, dtype=np.float64)
    s = float(np.sum(i ** (-theta)))
    if N <= head:
        return s
    a, b = float(m), float(N)

    def f(x, d=0):  # d-th derivative of x^-theta, d in {0, 1, 3}
        c = {0: 1.0, 1: -theta, 3: -theta * (theta + 1) * (theta + 2)}[d]
        return c * x ** (-theta - d)

    integral = (b ** (1 - theta) - a ** (1 - theta)) / (1 - theta)
    tail = integral + (f(b) - f(a)) / 2 + (f(b, 1) - f(a, 1)) / 12 - (f(b, 3) - f(a, 3)) / 720
    return s + tail


def zipf_keys(n, seed, bits=34, theta=0.99, offset=0):
    """n keys in [0, 2^bits) with P(key = r - 1) proportional to r^-theta for
    rank r in 1..2^bits, unscrambled, so the popular keys are the small ones.

    The sampler is the one of Gray, Sundaresan, Englert, Baclawski and
    Weinberger ("Quickly generating billion-record synthetic databases",
    SIGMOD 1994), which YCSB uses with its skew constant 0.99: ranks 1 and 2
    exactly, the others from the inverse of a continuous approximation."""
    N = float(1 << bits)
    zetan = zipf_zeta(1 << bits, theta)
    zeta2 = 1.0 + 0.5 ** theta
    alpha = 1.0 / (1.0 - theta)
    eta = (1.0 - (2.0 / N) ** (1.0 - theta)) / (1.0 - zeta2 / zetan)
    u = uniform_float(n, seed, offset)
    uz = u * zetan
    r = 1.0 + np.floor(N * (eta * u - eta + 1.0) ** alpha)
    r = np.where(uz < zeta2, 2.0, r)
    r = np.where(uz < 1.0, 1.0, r)
    r = np.clip(r, 1.0, N)
    return (r - 1.0).astype(np.uint64)


def range_queries_width(n, seed, width, bits=40):
    """Queries [lo, lo + width) with lo uniform over the key space."""
    lo = uniform_keys(n, seed, bits)
    hi = lo + np.uint64(width)
    return lo, hi


def range_queries_by_count(keys_sorted, lengths, seed):
    """Queries that cover exactly lengths[i] keys of the sorted key array.

    lo = keys[s], hi = keys[s + l] (or keys[-1] + 1 at the end), s uniform in
    [0, n - l].  Counting keys here is workload shaping on the harness side.
    """
    n = len(keys_sorted)
    lengths = np.minimum(np.asarray(lengths, dtype=np.int64), n)
    u = uniform_float(len(lengths), seed)
    start = np.floor(u * (n - lengths + 1)).astype(np.int64)
    start = np.minimum(start, n - lengths)
    lo = keys_sorted[start]
    end = start + lengths
    top = np.uint64(keys_sorted[-1]) + np.uint64(1)
    hi = np.where(end < n, keys_sorted[np.minimum(end, n - 1)], top).astype(np.uint64)
    return lo.astype(np.uint64), hi


def rmat_edges(m, seed, scale=24, a=0.5, b=0.1, c=0.1):
    """m directed R-MAT edges (src, dst) on 2^scale vertices, `scale` quadrant draws each.

    No noise and no vertex permutation, so vertex 0 is the hub.
    """
    src = np.zeros(m, dtype=np.uint64)
    dst = np.zeros(m, dtype=np.uint64)
    ab, abc = a + b, a + b + c
    for lvl in range(scale):
        u = uniform_float(m, seed + 7919 * (lvl + 1))
        bit = np.uint64(1 << (scale - 1 - lvl))
        right = ((u >= a) & (u < ab)) | (u >= abc)   # quadrants b and d: dst bit set
        down = u >= ab                                # quadrants c and d: src bit set
        dst |= np.where(right, bit, np.uint64(0))
        src |= np.where(down, bit, np.uint64(0))
    return src, dst


def er_edges(m, seed, nv):
    """m ordered vertex pairs (src, dst) drawn uniformly from [0, nv)^2: an
    Erdos-Renyi graph (each of the nv^2 ordered pairs appears with probability
    about m / nv^2) before self-loops are dropped and edges symmetrised."""
    src = np.floor(uniform_float(m, seed) * nv).astype(np.uint64)
    dst = np.floor(uniform_float(m, seed + 1) * nv).astype(np.uint64)
    return src, dst


def edge_keys(src, dst, symmetric=True, drop_self_loops=True):
    """Edge keys src<<32|dst (unsorted, possibly with repeats)."""
    src = np.asarray(src, dtype=np.uint64)
    dst = np.asarray(dst, dtype=np.uint64)
    if drop_self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    k = (src << np.uint64(32)) | dst
    if symmetric:
        k = np.concatenate([k, (dst << np.uint64(32)) | src])
    return k


# ---- the same streams drawn with torch (on any device), bit-identical to numpy ----
def _t_splitmix64(seed, n, offset, device):
    import torch
    g = -0x61C8864680B583EB            # 0x9E3779B97F4A7C15 as int64
    m1 = -0x40A7B892E31B1A47           # 0xBF58476D1CE4E5B9 as int64
    m2 = -0x6B2FB644ECCEEE15           # 0x94D049BB133111EB as int64
    s = seed & 0xFFFFFFFFFFFFFFFF
    if s >= 1 << 63:
        s -= 1 << 64
    i = torch.arange(offset + 1, offset + n + 1, dtype=torch.int64, device=device)
    z = s + i * g

    def lsr(x, k):
        return (x >> k) & ((1 << (64 - k)) - 1)

    z = (z ^ lsr(z, 30)) * m1
    z = (z ^ lsr(z, 27)) * m2
    return z ^ lsr(z, 31)


def uniform_float_torch(n, seed, device, offset=0):
    import torch
    z = _t_splitmix64(seed, n, offset, device)
    return ((z >> 11) & ((1 << 53) - 1)).to(torch.float64) * (1.0 / (1 << 53))


def rmat_edges_torch(m, seed, scale=24, a=0.5, b=0.1, c=0.1, device="cpu"):
    """rmat_edges drawn with torch: same values, int64 tensors on `device`."""
    import torch
    src = torch.zeros(m, dtype=torch.int64, device=device)
    dst = torch.zeros(m, dtype=torch.int64, device=device)
    ab, abc = a + b, a + b + c
    for lvl in range(scale):
        u = uniform_float_torch(m, seed + 7919 * (lvl + 1), device)
        bit = 1 << (scale - 1 - lvl)
        right = ((u >= a) & (u < ab)) | (u >= abc)
        down = u >= ab
        dst |= right.to(torch.int64) * bit
        src |= down.to(torch.int64) * bit
    return src, dst


def er_edges_torch(m, seed, nv, device="cpu"):
    """er_edges drawn with torch: same values, int64 tensors on `device`."""
    import torch
    src = torch.floor(uniform_float_torch(m, seed, device) * nv).to(torch.int64)
    dst = torch.floor(uniform_float_torch(m, seed + 1, device) * nv).to(torch.int64)
    return src, dst


def edge_keys_torch(src, dst, symmetric=True, drop_self_loops=True):
    import torch
    if drop_self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    k = (src << 32) | dst
    if symmetric:
        k = torch.cat([k, (dst << 32) | src])
    return k


def uniform_keys_torch(n, seed, device, bits=40, offset=0):
    """uniform_keys drawn with torch (int64 tensor on `device`, same values)."""
    z = _t_splitmix64(seed, n, offset, device)
    if bits < 64:
        z = z & ((1 << bits) - 1)
    return z


def log_uniform_sizes(n, seed, lo_exp=1.0, hi_exp=6.0):
    """n sizes floor(10^(lo_exp + (hi_exp - lo_exp) u)), u uniform in [0, 1)."""
    u = uniform_float(n, seed)
    return np.floor(10.0 ** (lo_exp + (hi_exp - lo_exp) * u)).astype(np.int64)
