"""Seeded point-set generators (NumPy PCG64) for the merge workloads.

Seeds follow one scheme: seed = 1000 * workload + stream, with stream
1 = first set, 2 = second set (or the split), 3 = cluster centres/offsets,
4 = merge random stream, 5 = request stream, 6 = graph perturbation.

Workloads (sizes as named in the benchmark description):
  W1  two sets of 5,000 x 32, i.i.d. N(0,1)                        (l2)
  W2  1,000 isotropic clusters, centres U[0,255]^128, sigma 20, rounded and
      clipped to integers in [0,255], stored fp32; 1M draws split 500k/500k
  W3  |N(0,1)|^960 plus one of 200 offsets U[0,2)^960, rows L2-normalised in
      FP64 then stored fp32; 250k + 250k                           (cosine)
  W4  50-component Gaussian mixture, means U[0,10)^100, sigma U[0.5,2],
      8 blocks of 125,000                                           (l1)
  W5  base of 2M points from the W2 mixture plus log-uniform request sizes
The real datasets of the paper (SIFT, GIST, ...) are not used: these stand
in for their shapes (d=128 byte-valued, d=960, d=100).
"""
import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_sets(n1=5000, n2=5000, d=32, workload=1):
    """W1: two disjoint i.i.d. N(0,1) sets."""
    S1 = rng(1000 * workload + 1).standard_normal((n1, d)).astype(np.float32)
    S2 = rng(1000 * workload + 2).standard_normal((n2, d)).astype(np.float32)
    return S1, S2


def byte_cluster_points(n, d=128, n_centers=1000, sigma=20.0, workload=2, stream=1):
    """Points of the W2 mixture: uniform centre, + N(0, sigma^2), rint, clip."""
    C = rng(1000 * workload + 3).uniform(0.0, 255.0, size=(n_centers, d))
    g = rng(1000 * workload + stream)
    out = np.empty((n, d), np.float32)
    step = 1 << 16
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        c = g.integers(0, n_centers, size=hi - lo)
        x = C[c] + g.normal(0.0, sigma, size=(hi - lo, d))
        out[lo:hi] = np.clip(np.rint(x), 0.0, 255.0)
    return out


def byte_cluster_sets(n1=500_000, n2=500_000, d=128, n_centers=1000, sigma=20.0, workload=2):
    """W2: n1+n2 draws of the byte-valued mixture split at random."""
    X = byte_cluster_points(n1 + n2, d, n_centers, sigma, workload, stream=1)
    perm = rng(1000 * workload + 2).permutation(n1 + n2)
    return X[perm[:n1]].copy(), X[perm[n1:]].copy()


def cosine_sets(n1=250_000, n2=250_000, d=960, n_offsets=200, workload=3):
    """W3: nonnegative rows |N(0,1)| + offset, L2-normalised in FP64."""
    O = rng(1000 * workload + 3).uniform(0.0, 2.0, size=(n_offsets, d))
    out = []
    for stream, n in ((1, n1), (2, n2)):
        g = rng(1000 * workload + stream)
        X = np.empty((n, d), np.float32)
        step = 1 << 14
        for lo in range(0, n, step):
            hi = min(n, lo + step)
            c = g.integers(0, n_offsets, size=hi - lo)
            x = np.abs(g.standard_normal((hi - lo, d))) + O[c]
            x /= np.linalg.norm(x, axis=1, keepdims=True)
            X[lo:hi] = x
        out.append(X)
    return out[0], out[1]


def gmm_blocks(n_blocks=8, block=125_000, d=100, n_comp=50, workload=4):
    """W4: i.i.d. blocks of a Gaussian mixture with per-component sigma."""
    g0 = rng(1000 * workload + 3)
    mu = g0.uniform(0.0, 10.0, size=(n_comp, d))
    sig = g0.uniform(0.5, 2.0, size=n_comp)
    blocks = []
    for b in range(n_blocks):
        g = rng(1000 * workload + 100 + b)
        c = g.integers(0, n_comp, size=block)
        x = mu[c] + sig[c][:, None] * g.standard_normal((block, d))
        blocks.append(x.astype(np.float32))
    return blocks


def request_sizes(count, lo=1, hi=20_000, workload=5):
    """W5 request sizes: floor(exp(U[0, ln(hi+1)))) clipped to [lo, hi]."""
    u = rng(1000 * workload + 5).uniform(0.0, np.log(hi + 1.0), size=count)
    return np.clip(np.floor(np.exp(u)).astype(np.int64), lo, hi)


def degrade_positions(n, m, k, target_recall, workload=2, stream=6):
    """Index-level perturbation of exact neighbour lists into approximate
    ones.  Rows hold m >= 2k exact neighbours in ascending order; the entry at
    rank r (0-based, r < k) is dropped with probability
    2 (1 - target) (r + 0.5) / k, so drops grow with rank and average
    1 - target; a row keeps the first k entries that survive, so recall@k is
    close to `target_recall`.  Returns the kept column positions (n, k), in
    ascending rank order."""
    assert m >= 2 * k
    g = rng(1000 * workload + stream)
    p = 2.0 * (1.0 - target_recall) * (np.arange(m) + 0.5) / k
    p[k:] = 0.0
    keep = g.random((n, m)) >= p[None, :]
    # stable order: survivors first (in rank order), then the dropped ones
    order = np.argsort(~keep, axis=1, kind="stable")[:, :k]
    return np.sort(order, axis=1)


def degrade_lists(ids_ext, k, target_recall, workload=2, stream=6):
    """degrade_positions applied to exact lists `ids_ext` (n, >= 2k)."""
    ids_ext = np.asarray(ids_ext)
    pos = degrade_positions(ids_ext.shape[0], ids_ext.shape[1], k, target_recall, workload,
                            stream)
    return np.take_along_axis(ids_ext, pos, axis=1).astype(np.int32)
