"""The parallel code-length construction reaches the oracle's lengths exactly.

Algorithm 1 (GenerateCL) of the paper combines, per round, every subtree
lighter than the sum t of the two lightest ones, merging the selected leaves
with the internal-node queue and melding adjacent pairs.  The printed
pseudo-code uses a strict `< t` threshold and leaves the order of equal
weights open.  The reading implemented by the GPU kernel is: per round,
select all unconsumed leaves with weight <= t and every queued internal node
(all are <= t), merge them by the key (weight, leaf-before-internal, rank),
meld consecutive pairs, and carry an odd last node into the next round; code
lengths follow from parent links by pointer jumping.  This file is a plain
Python model of that round structure (not of the kernel's memory layout),
checked against the heap-based oracle on tie-heavy histograms.
"""
import numpy as np

import oracle


def parallel_round_lengths(h):
    h = [int(v) for v in h]
    A = len(h)
    used = [s for s in range(A) if h[s] > 0]
    leaves = sorted(used, key=lambda s: (h[s], s))
    m = len(leaves)
    cl = [0] * A
    if m == 0:
        return cl, 0
    if m == 1:
        cl[leaves[0]] = 1
        return cl, 0
    lw = [h[s] for s in leaves]
    iw = []           # internal node weights, creation order
    parent = {}       # ('L', i) / ('I', k) -> internal k
    lc = ih = 0
    rounds = 0
    while (m - lc) + (len(iw) - ih) > 1:
        rounds += 1
        # t = sum of the two smallest available nodes (leaf first on ties)
        cand = [(lw[i], 0, i) for i in range(lc, min(m, lc + 2))] + \
               [(iw[k], 1, k) for k in range(ih, min(len(iw), ih + 2))]
        cand.sort()
        t = cand[0][0] + cand[1][0]
        a = 0
        while lc + a < m and lw[lc + a] <= t:
            a += 1
        b = len(iw) - ih  # every queued internal node is <= t
        sel = [(lw[i], 0, i) for i in range(lc, lc + a)] + [(iw[k], 1, k) for k in range(ih, len(iw))]
        sel.sort()  # the merge of two sorted runs by key
        pairs = len(sel) // 2
        base = len(iw)
        for p in range(pairs):
            x, y = sel[2 * p], sel[2 * p + 1]
            iw.append(x[0] + y[0])
            for node in (x, y):
                parent[("L" if node[1] == 0 else "I", node[2])] = base + p
        carry = sel[-1] if len(sel) % 2 else None
        lc += a - (1 if carry is not None and carry[1] == 0 else 0)
        ih += b - (1 if carry is not None and carry[1] == 1 else 0)
    # pointer jumping over internal nodes: depth(root) = 0
    nint = len(iw)
    root = nint - 1
    d = [0 if k == root else 1 for k in range(nint)]
    nx = [root if k == root else parent[("I", k)] for k in range(nint)]
    while any(nx[k] != root for k in range(nint)):
        d, nx = [d[k] + d[nx[k]] for k in range(nint)], [nx[nx[k]] for k in range(nint)]
    for i, s in enumerate(leaves):
        cl[s] = d[parent[("L", i)]] + 1
    return cl, rounds


def test_parallel_rounds_equal_heap_on_tie_heavy_histograms():
    rng = np.random.default_rng(21)
    max_rounds = 0
    for trial in range(1500):
        A = int(rng.integers(1, 200))
        choices = np.array([0, 0, 1, 1, 2, 3, 4, 8, 16, 100])
        h = rng.choice(choices, size=A).astype(np.uint32)
        cl_ref, _ = oracle.code_lengths(h)
        cl, rounds = parallel_round_lengths(h)
        max_rounds = max(max_rounds, rounds)
        assert list(cl_ref) == cl, (h.tolist(), list(cl_ref), cl)
    assert max_rounds > 3


def test_parallel_rounds_fibonacci_needs_one_round_per_level():
    fib = [1, 1]
    while len(fib) < 30:
        fib.append(fib[-1] + fib[-2])
    cl, rounds = parallel_round_lengths(fib)
    cl_ref, _ = oracle.code_lengths(np.array(fib, dtype=np.uint32))
    assert cl == list(cl_ref) and max(cl) == 29 and rounds >= 28
