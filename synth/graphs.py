"""Input graphs for the large workloads, built on the GPU with plain PyTorch
(float64 GEMM + top-k).  These are INPUTS of the merge (the paper builds its
sub-graphs beforehand, Section 5), not part of the merge path, and share
nothing with the HIP library or the oracle.

For integer-valued rows (the byte-valued cluster workload) every squared-l2
distance is an integer below 2^24, so the float64 GEMM form is exact and
equals the canonical FP32 value bit for bit; rows are then ordered by
(distance, id), as the merge requires of given distances."""
import numpy as np
import torch

from .gen import degrade_positions


def exact_knn_l2_integer(X, kk, device="cuda", chunk=1024):
    """Exact kk nearest neighbours (self excluded) of every row of X under
    squared l2, for integer-valued rows.  Returns (ids int64, dist float64),
    each row sorted by (distance, id)."""
    n = X.shape[0]
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(device=device, dtype=torch.float64)
    sq = (Xd * Xd).sum(1)
    ids = torch.empty((n, kk), dtype=torch.int64, device=device)
    dist = torch.empty((n, kk), dtype=torch.float64, device=device)
    ar = torch.arange(chunk, device=device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        q = Xd[lo:hi]
        D = sq[lo:hi, None] + sq[None, :] - 2.0 * (q @ Xd.T)
        D[ar[:hi - lo], lo + ar[:hi - lo]] = float("inf")
        v, i = torch.topk(D, kk + 1, dim=1, largest=False, sorted=True)
        # (distance, id) order; the extra column absorbs a tie at the cut
        key = v * float(2 ** 22) + i.to(torch.float64)
        o = torch.argsort(key, dim=1)[:, :kk]
        ids[lo:hi] = torch.gather(i, 1, o)
        dist[lo:hi] = torch.gather(v, 1, o)
        del D
    return ids.cpu().numpy(), dist.cpu().numpy()


def approximate_graph(X, k, target_recall, device="cuda", workload=2, stream=6):
    """An approximate k-NN graph near `target_recall` (recall@k): exact 2k
    lists perturbed by rank-dependent drops (synth.gen.degrade_positions).
    Returns (ids int32, dist float32) with rows sorted by (distance, id)."""
    ids_ext, d_ext = exact_knn_l2_integer(X, 2 * k, device)
    pos = degrade_positions(X.shape[0], 2 * k, k, target_recall, workload, stream)
    ids = np.take_along_axis(ids_ext, pos, axis=1).astype(np.int32)
    dist = np.take_along_axis(d_ext, pos, axis=1).astype(np.float32)
    return ids, dist
