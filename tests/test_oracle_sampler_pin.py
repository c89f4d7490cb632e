"""Pin of the oracle's repeat loop (forward sample, Reverse(G), neighbourhood
G[u] = reverse(u) u forward(u), local join, UpdateNN) against an independent
rebuild written here in plain Python from the definitions (Algorithms 1 and
2 of Zhao et al., "On the Merge of k-NN Graph"; NN-Descent sampling, which
Section 3.1 invokes by citation, as the readings state it):

  - forward sample: the s NEW entries of smallest priority H(seed, FWD, t,
    u, id) become u's NEW sample and are marked OLD; entries that were OLD
    before form its OLD sample;
  - Reverse(G): each sampled edge u -> v offers u to v's reverse list of the
    same kind, which keeps the s offers of smallest priority;
  - the neighbourhood of u is NEW = fwd-new u rev-new and OLD = (fwd-old u
    rev-old) minus NEW; every unordered pair {p, q}, p in NEW, q in NEW u OLD,
    p != q, that the merge predicate admits (S-Merge: different sets;
    J-Merge: not both from the base) is compared and offered to both lists;
  - UpdateNN in set form: the round's list is the top k by (distance, id) of
    the old list and every proposal, self and duplicates excluded; entries
    that were not in the list before the round are NEW;
  - c_t = the entries present after round t that were not there before.

Nothing here calls the oracle except the function under test: the hash is
SplitMix64 written out from its published definition (checked against the
published outputs below), and distances are exact integers (small integer
coordinates), so no rounding question arises.  With s at least the largest
list and reverse in-degree, sampling takes everything, and the test checks
the structure of the round alone; with small s it also checks the
priority selections.  A swapped NEW/OLD mark, a reverse list built from the
wrong side, old x old pairs joined, or a missing direction of UpdateNN each
change the per-round pair counts or lists compared here."""
import numpy as np
import pytest

import oracle

M64 = (1 << 64) - 1
TAG_APPEND, TAG_INIT, TAG_FWD, TAG_RNEW, TAG_ROLD = 0xA1, 0xA2, 0xB1, 0xB2, 0xB3


def sm64(x):
    """SplitMix64 output for state x (Steele, Lea, Flood 2014)."""
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def H(seed, tag, a, b, c):
    return sm64(sm64(sm64(sm64((seed ^ tag) & M64) ^ a) ^ b) ^ c)


def test_local_splitmix_is_the_published_generator():
    gamma = 0x9E3779B97F4A7C15
    assert [sm64((i * gamma) & M64) for i in range(3)] == \
        [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def distinct_draws(seed, tag, row, N, skip, m):
    """m distinct values of [0, N) minus `skip` by rejection from the stream
    H(seed, tag, row, t, 0), scaled by multiply-shift (all of them, ascending,
    when m covers every admissible value)."""
    avail = N - (1 if skip >= 0 else 0)
    if m >= avail:
        return [v for v in range(N) if v != skip][:m]
    out = []
    t = 0
    while len(out) < m:
        h = H(seed, tag, row, t, 0)
        if skip >= 0:
            v = ((h >> 32) * (N - 1)) >> 32
            v += v >= skip
        else:
            v = ((h >> 32) * N) >> 32
        if v not in out:
            out.append(v)
        t += 1
    return out


def int_sets(n1, n2, d, seed, hi=12):
    # distinct integer rows (no zero distance between different ids): cells
    # of the grid [0, hi)^d drawn without replacement
    rng = np.random.default_rng(seed)
    cells = rng.choice(hi ** d, size=n1 + n2, replace=False)
    X = np.stack([(cells // hi ** t) % hi for t in range(d)], axis=1).astype(np.float32)
    return X[:n1], X[n1:]


def D2(X):
    """exact squared l2 distances of integer rows"""
    Xi = X.astype(np.int64)
    return ((Xi[:, None, :] - Xi[None, :, :]) ** 2).sum(-1)


def exact_lists(Dm, k):
    """exact k-NN lists by (distance, id), self excluded (plain definition)"""
    n = Dm.shape[0]
    out = []
    for i in range(n):
        cand = sorted((int(Dm[i, j]), j) for j in range(n) if j != i)
        out.append(cand[:k])
    return out


class Rebuild:
    """Lists as {id: [dist, isnew]} per row; rounds as defined above."""

    def __init__(self, Dfull, n1, k, s, seed, joint):
        self.D, self.n1, self.k, self.s, self.seed, self.joint = Dfull, n1, k, s, seed, joint
        self.n = Dfull.shape[0]
        self.G = [dict() for _ in range(self.n)]
        self.rear = [[] for _ in range(self.n)]
        self.max_in_degree = 0

    def admits(self, p, q):
        p1, q1 = p < self.n1, q < self.n1
        return not (p1 and q1) if self.joint else p1 != q1

    @staticmethod
    def topk(entries, k):
        return sorted(entries, key=lambda e: (e[1], e[0]))[:k]  # (id, dist) by (dist, id)

    def round(self, t):
        n, k, s, seed = self.n, self.k, self.s, self.seed
        new_f, old_f = [], []
        for u in range(n):
            L = self.G[u]
            olds = [i for i, (_, isnew) in L.items() if not isnew]
            news = sorted((H(seed, TAG_FWD, t, u, i) >> 32, i) for i, (_, isnew) in L.items()
                          if isnew)
            take = [i for _, i in news[:s]]
            for i in take:
                L[i][1] = False
            new_f.append(take)
            old_f.append(olds)
        rnew = [[] for _ in range(n)]
        rold = [[] for _ in range(n)]
        for u in range(n):
            for v in new_f[u]:
                rnew[v].append((H(seed, TAG_RNEW, t, v, u) >> 32, u))
            for v in old_f[u]:
                rold[v].append((H(seed, TAG_ROLD, t, v, u) >> 32, u))
        for v in range(n):
            self.max_in_degree = max(self.max_in_degree, len(rnew[v]), len(rold[v]))
            rnew[v] = [u for _, u in sorted(rnew[v])[:s]]
            rold[v] = [u for _, u in sorted(rold[v])[:s]]
        prop = [dict() for _ in range(n)]
        pairs = 0
        for u in range(n):
            NEW = set(new_f[u]) | set(rnew[u])
            OLD = (set(old_f[u]) | set(rold[u])) - NEW
            NEWl, OLDl = sorted(NEW), sorted(OLD)
            cand = [(p, q) for a, p in enumerate(NEWl) for q in NEWl[a + 1:]]
            cand += [(p, q) for p in NEWl for q in OLDl]
            for p, q in cand:
                if p == q or not self.admits(p, q):
                    continue
                pairs += 1
                dd = int(self.D[p, q])
                prop[p][q] = dd
                prop[q][p] = dd
        c = 0
        for p in range(n):
            L = self.G[p]
            merged = [(i, dv) for i, (dv, _) in L.items()]
            merged += [(q, dv) for q, dv in prop[p].items() if q != p and q not in L]
            keep = self.topk(merged, k)
            newG = {}
            for i, dv in keep:
                if i in L:
                    newG[i] = L[i]
                else:
                    newG[i] = [dv, True]
                    c += 1
            self.G[p] = newG
        return pairs, c

    def final(self):
        ids = np.full((self.n, self.k), -1, np.int32)
        dist = np.full((self.n, self.k), np.inf, np.float32)
        for i in range(self.n):
            merged = dict((j, dv) for j, (dv, _) in self.G[i].items())
            for j, dv in self.rear[i]:
                merged.setdefault(j, dv)
            keep = self.topk([(j, dv) for j, dv in merged.items() if j != i], self.k)
            for c, (j, dv) in enumerate(keep):
                ids[i, c], dist[i, c] = j, dv
        return ids, dist


def rebuild_smerge(S1, S2, GL1, GL2, k, s, seed, rounds, keep_ratio=0.5):
    """S-Merge: Divide (k1 kept, OLD), Append (k - k1 other-set draws, NEW)."""
    n1, n2 = len(S1), len(S2)
    Dm = D2(np.concatenate([S1, S2]))
    R = Rebuild(Dm, n1, k, s, seed, joint=False)
    k1 = int(np.floor(np.float32(keep_ratio) * np.float32(k)))
    for i in range(n1 + n2):
        own1 = i < n1
        row = GL1[i] if own1 else [(dv, j + n1) for dv, j in GL2[i - n1]]
        for dv, j in row[:k1]:
            R.G[i][j] = [dv, False]
        R.rear[i] = [(j, dv) for dv, j in row[k1:]]
        N = n2 if own1 else n1
        for v in distinct_draws(seed, TAG_APPEND, i, N, -1, min(k - k1, N)):
            g = n1 + v if own1 else v
            R.G[i][g] = [int(Dm[i, g]), True]
    return R, Dm, k1


def rebuild_jmerge(Sb, GLb, Sr, k, s, seed, keep_ratio=0.5):
    """J-Merge: Divide the base lists, Append raw draws to them, Initialize
    every raw row with k draws of S u raw minus itself (all NEW)."""
    nb, nr = len(Sb), len(Sr)
    n = nb + nr
    Dm = D2(np.concatenate([Sb, Sr]))
    R = Rebuild(Dm, nb, k, s, seed, joint=True)
    k1 = int(np.floor(np.float32(keep_ratio) * np.float32(k)))
    for i in range(nb):
        for dv, j in GLb[i][:k1]:
            R.G[i][j] = [dv, False]
        R.rear[i] = [(j, dv) for dv, j in GLb[i][k1:]]
        for v in distinct_draws(seed, TAG_APPEND, i, nr, -1, min(k - k1, nr)):
            R.G[i][nb + v] = [int(Dm[i, nb + v]), True]
    for g in range(nb, n):
        for v in distinct_draws(seed, TAG_INIT, g, n, g, min(k, n - 1)):
            R.G[g][v] = [int(Dm[g, v]), True]
    return R, Dm


def graph_arrays(GL, k):
    ids = np.array([[j for _, j in row[:k]] for row in GL], np.int32)
    dist = np.array([[dv for dv, _ in row[:k]] for row in GL], np.float32)
    return ids, dist


def run_rounds(R, T):
    pairs, cs = [], []
    for t in range(T):
        p, c = R.round(t)
        pairs.append(p)
        cs.append(c)
        if c == 0:
            break
    return pairs, cs


SMERGE_CASES = [
    # (n1, n2, d, k, s, seed): s = 32 takes every NEW entry and every reverse
    # offer (checked below); s = 2 and 3 make both selections bite
    (40, 36, 3, 6, 32, 11),
    (40, 36, 3, 6, 2, 12),
    (33, 45, 4, 8, 3, 13),
]


@pytest.mark.parametrize("n1,n2,d,k,s,seed", SMERGE_CASES)
def test_smerge_rounds_match_the_rebuild(n1, n2, d, k, s, seed):
    S1, S2 = int_sets(n1, n2, d, seed=100 + seed)
    GL1 = exact_lists(D2(S1), k)
    GL2 = exact_lists(D2(S2), k)
    G1, G2 = graph_arrays(GL1, k), graph_arrays(GL2, k)
    R, _, _ = rebuild_smerge(S1, S2, GL1, GL2, k, s, seed, rounds=None)
    pairs, cs = run_rounds(R, 30)
    if s == 32:
        # the precondition of "sampling takes everything"
        assert R.max_in_degree <= s and k <= s
    assert len(pairs) >= 2 and pairs[0] > 0 and cs[0] > 0
    # round by round: the oracle stopped after T rounds has the rebuild's
    # lists after T rounds (then Merge and Sort with the rear parts)
    for T in range(1, len(pairs) + 1):
        R2, _, _ = rebuild_smerge(S1, S2, GL1, GL2, k, s, seed, rounds=None)
        run_rounds(R2, T)
        eids, edist = R2.final()
        ids, dist, st = oracle.smerge(S1, G1, S2, G2, k, "l2", sample=s, seed=seed,
                                      max_rounds=T)
        assert st["rounds"] == T
        assert st["pairs"] == pairs[:T], f"pairs per round differ after {T} rounds"
        assert st["c"] == cs[:T], f"updates per round differ after {T} rounds"
        np.testing.assert_array_equal(ids, eids, err_msg=f"lists differ after {T} rounds")
        np.testing.assert_array_equal(dist, edist)
    # and the whole run, to convergence
    _, _, st = oracle.smerge(S1, G1, S2, G2, k, "l2", sample=s, seed=seed)
    assert st["pairs"] == pairs and st["c"] == cs


@pytest.mark.parametrize("nb,nr,d,k,s,seed", [(30, 25, 3, 6, 32, 21), (40, 20, 3, 6, 2, 22),
                                              (0, 50, 3, 6, 4, 23)])
def test_jmerge_rounds_match_the_rebuild(nb, nr, d, k, s, seed):
    Sb, Sr = int_sets(nb, nr, d, seed=200 + seed)
    GLb = exact_lists(D2(Sb), k) if nb else []
    Gb = graph_arrays(GLb, k) if nb else (None, None)
    R, _ = rebuild_jmerge(Sb, GLb, Sr, k, s, seed)
    pairs, cs = run_rounds(R, 30)
    if s == 32:
        assert R.max_in_degree <= s and k <= s
    assert len(pairs) >= 2 and pairs[0] > 0
    for T in (1, 2, len(pairs)):
        R2, _ = rebuild_jmerge(Sb, GLb, Sr, k, s, seed)
        run_rounds(R2, T)
        eids, edist = R2.final()
        ids, dist, st = oracle.jmerge(Sb if nb else None, Gb, Sr, k, "l2", sample=s, seed=seed,
                                      max_rounds=T)
        assert st["pairs"] == pairs[:T] and st["c"] == cs[:T]
        np.testing.assert_array_equal(ids, eids)
        np.testing.assert_array_equal(dist, edist)


def test_second_round_joins_no_old_pair():
    # Entries sampled in round 0 are OLD in round 1, so a pair of two rows
    # that were both only OLD members of every neighbourhood is never joined
    # again: round 1's pair count is that of NEW x NEW and NEW x OLD alone,
    # and it is strictly below the count that would also take OLD x OLD.
    n1, n2, d, k, s, seed = 40, 36, 3, 6, 32, 11
    S1, S2 = int_sets(n1, n2, d, seed=100 + seed)
    GL1, GL2 = exact_lists(D2(S1), k), exact_lists(D2(S2), k)
    G1, G2 = graph_arrays(GL1, k), graph_arrays(GL2, k)
    R, _, _ = rebuild_smerge(S1, S2, GL1, GL2, k, s, seed, rounds=None)
    R.round(0)
    # round 1's neighbourhoods, counted with and without OLD x OLD
    snapshot = [{i: list(v) for i, v in L.items()} for L in R.G]
    with_old = 0
    for u in range(R.n):
        fwd = set(snapshot[u])
        rev = {v for v in range(R.n) if u in snapshot[v]}
        members = sorted(fwd | rev)
        for a_, p in enumerate(members):
            for q in members[a_ + 1:]:
                with_old += R.admits(p, q)
    p1, _ = R.round(1)
    _, _, st = oracle.smerge(S1, G1, S2, G2, k, "l2", sample=s, seed=seed, max_rounds=2)
    assert st["pairs"][1] == p1
    assert p1 < with_old
