"""Seeded synthetic inputs shaped like the paper's single-cell workloads.

This module is the only code shared by the CPU oracle and the GPU path.  It
draws random numbers and lays them out; it holds none of the method's
arithmetic (no Gram matrix, no eigendecomposition, no likelihood, no
recomposition, no top-k).

Recipes (all seeded, all reproducible block by block):

* ``nb_log1p`` -- a cells x genes matrix X = log1p(counts) with negative
  binomial counts (dispersion alpha, Var = mu + alpha mu^2) whose means follow
  log mu_ij = beta0 + 0.5 (A B^T)_ij / sqrt(rank) + M[cl(i), j] + g_j with a
  rank-8 factor A (cells x 8), B (genes x 8) ~ N(0, 1), a per-cluster gene
  effect M ~ N(0, 1) and gene offsets g ~ N(0, variance 0.5).  Cluster sizes
  are equal or Zipf(1.2) with largest-remainder rounding; Zipf-sized rows are
  shuffled by a seeded permutation.  The values are rounded to float32, which
  is what both sides consume.
* ``cell_factor_proxy`` -- an n x r matrix with orthonormal columns whose rows
  carry the structure of a cell-axis factor of such data: a cluster part, the
  shared rank-8 factor and per-cell noise directions.
* ``spectrum_proxy`` -- a descending positive spectrum of a p x p Gram matrix
  with a few signal spikes above a Marchenko-Pastur bulk.
* ``nb_log1p_gpu`` -- the ``nb_log1p`` recipe drawn on the GPU with torch's
  seeded Philox generator (normals, gamma, Poisson), for the many mid-sized
  instances of the warm-start training set; not used by any oracle
  comparison.
* ``nb_log1p_csr_gpu`` -- the same recipe at full scale (1M x 20k at 5%):
  row blocks drawn on the GPU, each block's own Philox stream, kept as CSR
  (columns ascending); the rank-8 cell factor A can be passed in so that a
  second modality shares it.
* ``peaks_csr_gpu`` -- binary peaks of a modality sharing the cell axis:
  Bernoulli(sigmoid(c0 + (A Bp^T)_ij / sqrt(8) + N(0, 1) noise)) with the
  cells' rank-8 factor A, Bp ~ N(0, 1) per peak and c0 set for the requested
  density, as CSR on the GPU.
* ``rotating_objects`` -- tensors shaped like the paper's COIL-20 videos:
  objects of (frames x h x w) whose pixels vary with the frame angle through
  the first three circular harmonics (a rank-3 image per harmonic) plus noise.

Each row block of ``nb_log1p`` draws from its own Philox stream keyed by
(seed, block), so any block of rows can be regenerated alone.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "zipf_sizes",
    "cluster_labels",
    "nb_log1p",
    "nb_log1p_rows",
    "dense_to_csr",
    "cell_factor_proxy",
    "csr_proxy",
    "spectrum_proxy",
    "workload",
    "rotating_objects",
    "nb_log1p_gpu",
    "nb_log1p_csr_gpu",
    "peaks_csr_gpu",
    "cell_factor_gpu",
    "ROW_BLOCK",
]

ROW_BLOCK = 4096
FACTOR_RANK = 8
ALPHA = 2.0

# The workloads by shape: sizes and generator parameters.
WORKLOADS = {
    "2000x500": dict(n=2000, p=500, clusters=8, zipf=False, beta0=0.0, r_c=500, r_g=500, k=10, seed=1000),
    "100kx2000": dict(n=100_000, p=2000, clusters=20, zipf=True, beta0=0.0, r_c=50, r_g=2000, k=10, seed=2000),
    "1Mx20k": dict(n=1_000_000, p=20_000, clusters=40, zipf=True, beta0=None, density=0.05,
                   r_c=100, r_g=20_000, k=10, seed=3000),
}


def workload(name: str) -> dict:
    return dict(WORKLOADS[name])


def zipf_sizes(n: int, n_clusters: int, s: float = 1.2) -> np.ndarray:
    """Cluster sizes proportional to c^-s, largest-remainder rounding, min 1."""
    w = np.arange(1, n_clusters + 1, dtype=np.float64) ** (-s)
    raw = n * w / w.sum()
    base = np.maximum(np.floor(raw).astype(np.int64), 1)
    short = n - int(base.sum())
    if short > 0:
        order = np.argsort(-(raw - np.floor(raw)), kind="stable")
        base[order[:short]] += 1
    elif short < 0:
        order = np.argsort(-base, kind="stable")
        i = 0
        while short < 0:
            j = order[i % n_clusters]
            if base[j] > 1:
                base[j] -= 1
                short += 1
            i += 1
    assert int(base.sum()) == n
    return base


def cluster_labels(n: int, n_clusters: int, zipf: bool, seed: int) -> np.ndarray:
    if zipf:
        sizes = zipf_sizes(n, n_clusters)
    else:
        sizes = np.full(n_clusters, n // n_clusters, dtype=np.int64)
        sizes[: n - int(sizes.sum())] += 1
    labels = np.repeat(np.arange(n_clusters, dtype=np.int32), sizes)
    if zipf:
        rng = np.random.Generator(np.random.Philox(key=[seed, 0xC1]))
        labels = labels[rng.permutation(n)]
    return labels


def _gene_params(p: int, n_clusters: int, seed: int):
    rng = np.random.Generator(np.random.Philox(key=[seed, 0x9E]))
    B = rng.standard_normal((p, FACTOR_RANK))
    M = rng.standard_normal((n_clusters, p))
    g = rng.standard_normal(p) * math.sqrt(0.5)
    return B, M, g


def _block_rows(block: int, n: int, p: int, labels, gene, beta0: float, seed: int):
    lo = block * ROW_BLOCK
    hi = min(n, lo + ROW_BLOCK)
    rng = np.random.Generator(np.random.Philox(key=[seed, 0x5EED0000 + block]))
    A = rng.standard_normal((hi - lo, FACTOR_RANK))
    B, M, g = gene
    log_mu = beta0 + 0.5 * (A @ B.T) / math.sqrt(FACTOR_RANK) + M[labels[lo:hi]] + g[None, :]
    mu = np.exp(log_mu)
    # NB(mean mu, dispersion alpha): failures before 1/alpha successes, success prob 1/(1+alpha mu)
    counts = rng.negative_binomial(1.0 / ALPHA, 1.0 / (1.0 + ALPHA * mu))
    return np.log1p(counts).astype(np.float32)


def _calibrate_beta0(density: float, p: int, n_clusters: int, labels, seed: int) -> float:
    """beta0 such that the mean probability of a nonzero count equals ``density``."""
    gene = _gene_params(p, n_clusters, seed)
    B, M, g = gene
    rng = np.random.Generator(np.random.Philox(key=[seed, 0xCA1]))
    m = 1_000_000
    ii = rng.integers(0, labels.shape[0], m)
    jj = rng.integers(0, p, m)
    A = rng.standard_normal((m, FACTOR_RANK))
    base = 0.5 * np.einsum("mk,mk->m", A, B[jj]) / math.sqrt(FACTOR_RANK) + M[labels[ii], jj] + g[jj]

    def frac(b0):
        mu = np.exp(b0 + base)
        return float(np.mean(1.0 - (1.0 + ALPHA * mu) ** (-1.0 / ALPHA)))

    lo, hi = -20.0, 10.0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if frac(mid) < density:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def nb_log1p(n: int, p: int, n_clusters: int, zipf: bool, seed: int,
             beta0: float | None = 0.0, density: float | None = None):
    """Dense float32 X (n x p) and the cluster labels.  See the module docstring."""
    labels = cluster_labels(n, n_clusters, zipf, seed)
    if beta0 is None:
        beta0 = _calibrate_beta0(density, p, n_clusters, labels, seed)
    gene = _gene_params(p, n_clusters, seed)
    X = np.empty((n, p), dtype=np.float32)
    for b in range((n + ROW_BLOCK - 1) // ROW_BLOCK):
        lo = b * ROW_BLOCK
        X[lo:lo + ROW_BLOCK] = _block_rows(b, n, p, labels, gene, beta0, seed)
    return X, labels, beta0


def nb_log1p_rows(rows, n: int, p: int, n_clusters: int, zipf: bool, seed: int, beta0: float):
    """Regenerate selected rows of ``nb_log1p`` without building the whole matrix."""
    rows = np.asarray(rows, dtype=np.int64)
    labels = cluster_labels(n, n_clusters, zipf, seed)
    gene = _gene_params(p, n_clusters, seed)
    out = np.empty((rows.shape[0], p), dtype=np.float32)
    cache = {}
    for t, i in enumerate(rows):
        b = int(i) // ROW_BLOCK
        if b not in cache:
            cache[b] = _block_rows(b, n, p, labels, gene, beta0, seed)
        out[t] = cache[b][int(i) - b * ROW_BLOCK]
    return out


def dense_to_csr(X: np.ndarray):
    """(row_ptr int64, col int32, val float32) of the nonzeros of X, columns ascending."""
    nz = X != 0
    row_ptr = np.zeros(X.shape[0] + 1, dtype=np.int64)
    np.cumsum(nz.sum(axis=1), out=row_ptr[1:])
    rr, cc = np.nonzero(nz)
    return row_ptr, cc.astype(np.int32), X[rr, cc].astype(np.float32)


def cell_factor_proxy(n: int, r: int, n_clusters: int, seed: int, zipf: bool = True,
                      noise: float = 1.0) -> np.ndarray:
    """n x r float32 with orthonormal columns and cell-factor-like rows.

    Columns span [cluster centroids | rank-8 factor | per-cell noise]; rows in
    one cluster share the centroid part, so near-duplicate cells exist as in
    clustered single-cell data.
    """
    labels = cluster_labels(n, n_clusters, zipf, seed)
    rng = np.random.Generator(np.random.Philox(key=[seed, 0xFAC7]))
    n_c = min(n_clusters, max(1, r // 2))
    n_f = min(FACTOR_RANK, max(0, r - n_c))
    n_e = r - n_c - n_f
    parts = []
    cent = rng.standard_normal((n_clusters, n_c)) * 3.0
    parts.append(cent[labels])
    if n_f:
        parts.append(rng.standard_normal((n, n_f)) * 1.5)
    if n_e:
        parts.append(rng.standard_normal((n, n_e)) * noise)
    Y = np.concatenate(parts, axis=1)
    Q, R = np.linalg.qr(Y)
    Q *= np.sign(np.diag(R))[None, :]
    return np.ascontiguousarray(Q.astype(np.float32))


def spectrum_proxy(p: int, n: int, n_spikes: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Descending spectrum of a p x p Gram of n samples: spikes over an MP bulk."""
    rng = np.random.Generator(np.random.Philox(key=[seed, 0x5EC7]))
    q = min(p, n) / max(p, n)
    lo, hi = (1 - math.sqrt(q)) ** 2, (1 + math.sqrt(q)) ** 2
    # Marchenko-Pastur quantiles by inverting the CDF on a fine grid
    x = np.linspace(lo, hi, 200_001)
    dens = np.sqrt(np.maximum((hi - x) * (x - lo), 0.0)) / (2 * math.pi * q * x)
    cdf = np.cumsum(dens)
    cdf /= cdf[-1]
    m = min(p, n)
    u = (np.arange(m) + 0.5) / m
    bulk = np.interp(u, cdf, x) * max(p, n)
    spikes = hi * max(p, n) * (2.0 + 10.0 * rng.random(n_spikes) ** 2) ** 2
    e = np.concatenate([spikes, bulk])
    e = np.sort(e)[::-1][:m] * scale
    return np.ascontiguousarray(e)


def _csr_proxy_block(b: int, n: int, p: int, density: float, seed: int, block: int):
    rows = min(block, n - b * block)
    rng = np.random.Generator(np.random.Philox(key=[seed, 0xC5B0000 + b]))
    s = rng.lognormal(0.0, 0.25, rows)
    s /= math.exp(0.25 ** 2 / 2)
    d = np.clip(density * s, 1e-6, 0.999)
    m_max = int(p * float(d.max()) * 1.5 + 100)
    gaps = rng.geometric(d[:, None], size=(rows, m_max))
    pos = np.cumsum(gaps, axis=1, dtype=np.int64) - 1
    mask = pos < p
    assert not mask[:, -1].any(), "position budget exhausted"
    c = rng.geometric(0.6, size=int(mask.sum()))
    return mask.sum(axis=1), pos[mask].astype(np.int32), np.log1p(c).astype(np.float32)


def csr_proxy(n: int, p: int, density: float, seed: int, block: int = 16384, workers: int = 1):
    """Fast CSR stand-in for ``nb_log1p`` at large sizes (same shape and density,
    log1p-of-small-count values, per-cell depth variation), without the cluster
    and factor structure.  Returns (row_ptr int64, col int32 ascending per row,
    val float32).  Row block b draws from Philox key (seed, 0xC5B0000 + b), so
    the result does not depend on ``workers`` (processes generating blocks).

    Per row i: depth s_i ~ lognormal(0, 0.25) scaled to mean 1, nonzero
    positions from geometric gaps with success probability density * s_i
    (a Bernoulli(density * s_i) pattern), counts ~ Geometric(0.6) >= 1 and
    values log1p(count)."""
    nblk = (n + block - 1) // block
    args = [(b, n, p, density, seed, block) for b in range(nblk)]
    if workers > 1 and nblk > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            parts = list(ex.map(_csr_proxy_block, *zip(*args)))
    else:
        parts = [_csr_proxy_block(*a) for a in args]
    counts = np.concatenate([q[0] for q in parts])
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, np.concatenate([q[1] for q in parts]), np.concatenate([q[2] for q in parts])


def rotating_objects(n_obj=20, frames=72, h=128, w=128, seed=0, noise=0.05):
    """List of n_obj float64 arrays (frames x h x w): sum over harmonics q = 1..3
    and cos / sin of trig(q angle_f) B_q,trig with B a rank-3 h x w image
    (Gaussian factors, weight 1/q), plus Gaussian noise; angle_f = 2 pi f / frames."""
    rng = np.random.default_rng(seed)
    ang = 2 * np.pi * np.arange(frames) / frames
    out = []
    for _ in range(n_obj):
        X = np.zeros((frames, h, w))
        for q in range(1, 4):
            for trig in (np.cos, np.sin):
                B = rng.standard_normal((h, 3)) @ rng.standard_normal((3, w)) / q
                X += trig(q * ang)[:, None, None] * B[None]
        X += noise * rng.standard_normal(X.shape)
        out.append(X)
    return out


def nb_log1p_gpu(n, p, n_clusters, zipf, seed, beta0=0.0, device="cuda"):
    """X = log1p(NB counts) (n x p, float32, on `device`) of the ``nb_log1p``
    recipe: log mu = beta0 + 0.5 (A B^T)_ij / sqrt(8) + M[cl(i), j] + g_j, counts
    Gamma(1/alpha, alpha mu) -> Poisson, drawn from torch's Philox generator
    seeded with `seed` (cluster labels as in ``cluster_labels``)."""
    import torch
    gen = torch.Generator(device=device).manual_seed(int(seed))
    lab = torch.from_numpy(cluster_labels(n, n_clusters, zipf, seed).astype(np.int64)).to(device)
    f64 = torch.float64
    A = torch.randn(n, FACTOR_RANK, generator=gen, device=device, dtype=f64)
    B = torch.randn(p, FACTOR_RANK, generator=gen, device=device, dtype=f64)
    M = torch.randn(n_clusters, p, generator=gen, device=device, dtype=f64)
    g = torch.randn(p, generator=gen, device=device, dtype=f64) * math.sqrt(0.5)
    mu = torch.exp(beta0 + 0.5 * (A @ B.T) / math.sqrt(FACTOR_RANK) + M[lab] + g[None, :])
    del A, M
    shape = torch.full_like(mu, 1.0 / ALPHA)
    lam = torch._standard_gamma(shape, generator=gen) * (ALPHA * mu)
    del shape, mu
    counts = torch.poisson(lam, generator=gen)
    del lam
    return torch.log1p(counts).to(torch.float32)


def cell_factor_gpu(n, seed, device="cuda"):
    """The rank-8 cell factor A (n x 8, FP64, N(0, 1)) of the full-scale
    generators, from its own Philox stream."""
    import torch
    gen = torch.Generator(device=device).manual_seed(int(seed) * 7919 + 1)
    return torch.randn(n, FACTOR_RANK, generator=gen, device=device, dtype=torch.float64)


def nb_log1p_csr_gpu(n, p, n_clusters, zipf, seed, beta0=0.0, A=None, block=32768, device="cuda"):
    """(row_ptr int64, col int32, val float32) device tensors of X = log1p(NB
    counts), the ``nb_log1p`` recipe: gene parameters B, M, g from one Philox
    stream, then row blocks of `block` rows each from its own stream (seed,
    block).  A: the cell factor (n x 8 FP64 on `device`), default
    cell_factor_gpu(n, seed)."""
    import torch
    gen = torch.Generator(device=device).manual_seed(int(seed))
    f64 = torch.float64
    B = torch.randn(p, FACTOR_RANK, generator=gen, device=device, dtype=f64)
    M = torch.randn(n_clusters, p, generator=gen, device=device, dtype=f64)
    g = torch.randn(p, generator=gen, device=device, dtype=f64) * math.sqrt(0.5)
    lab = torch.from_numpy(cluster_labels(n, n_clusters, zipf, seed).astype(np.int64)).to(device)
    if A is None:
        A = cell_factor_gpu(n, seed, device)
    counts, cols, vals = [], [], []
    for b in range((n + block - 1) // block):
        lo, hi = b * block, min(n, (b + 1) * block)
        gb = torch.Generator(device=device).manual_seed(int(seed) * 1_000_003 + 7 + b)
        mu = torch.exp(beta0 + 0.5 * (A[lo:hi] @ B.T) / math.sqrt(FACTOR_RANK) + M[lab[lo:hi]] + g[None, :])
        lam = torch._standard_gamma(torch.full_like(mu, 1.0 / ALPHA), generator=gb)
        lam *= ALPHA * mu
        del mu
        X = torch.log1p(torch.poisson(lam, generator=gb)).to(torch.float32)
        del lam
        nz = X != 0
        counts.append(nz.sum(dim=1))
        cols.append(nz.nonzero()[:, 1].to(torch.int32))
        vals.append(X[nz])
        del X, nz
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(torch.cat(counts), dim=0, out=row_ptr[1:])
    return row_ptr, torch.cat(cols), torch.cat(vals)


def peaks_csr_gpu(A, p, density, seed, block=16384, device="cuda"):
    """(row_ptr int64, col int32) device tensors of a binary cells x peaks
    matrix: entry (i, j) is 1 with probability sigmoid(c0 + (A Bp^T)_ij / sqrt(8)
    + e_ij), e_ij ~ N(0, 1), Bp ~ N(0, 1) per peak; c0 by bisection so that
    the mean probability over a 1M-entry sample equals `density`."""
    import torch
    n = A.shape[0]
    gen = torch.Generator(device=device).manual_seed(int(seed))
    Bp = torch.randn(p, FACTOR_RANK, generator=gen, device=device, dtype=torch.float64)
    ii = torch.randint(0, n, (1_000_000,), generator=gen, device=device)
    jj = torch.randint(0, p, (1_000_000,), generator=gen, device=device)
    base = (A[ii] * Bp[jj]).sum(dim=1) / math.sqrt(FACTOR_RANK) + torch.randn(1_000_000, generator=gen,
                                                                              device=device, dtype=torch.float64)
    lo, hi = -30.0, 10.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if float(torch.sigmoid(mid + base).mean()) < density:
            lo = mid
        else:
            hi = mid
    c0 = 0.5 * (lo + hi)
    Bp32 = (Bp / math.sqrt(FACTOR_RANK)).to(torch.float32)
    counts, cols = [], []
    for b in range((n + block - 1) // block):
        r0, r1 = b * block, min(n, (b + 1) * block)
        gb = torch.Generator(device=device).manual_seed(int(seed) * 1_000_003 + 11 + b)
        z = A[r0:r1].to(torch.float32) @ Bp32.T
        z += c0
        z += torch.randn(z.shape, generator=gb, device=device, dtype=torch.float32)
        hit = torch.rand(z.shape, generator=gb, device=device, dtype=torch.float32) < torch.sigmoid(z)
        del z
        counts.append(hit.sum(dim=1))
        cols.append(hit.nonzero()[:, 1].to(torch.int32))
        del hit
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(torch.cat(counts), dim=0, out=row_ptr[1:])
    return row_ptr, torch.cat(cols)

