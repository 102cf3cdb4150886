"""Write bench_expected.json: the oracle's cumulants (and central moments) at
sampled block-storage entries of the benchmark workloads.

The benchmark compares the library's outputs with these stored values, so
that it runs nothing under ``oracle/`` outside its CPU-baseline leg.  This
script calls only ``oracle/`` (the dense FP64 definitions: eq. cum_r of
Section 3.2 evaluated entry by entry) and the seeded generators of
``workloads.py``; the entries are chosen here from the block-storage layout
of Section 2.1 (sorted block tuples in lexicographic order, each block's b^d
entries in row-major order), and every chosen offset is checked against the
oracle's own offset-to-index map.

For each workload and order d the file holds the sampled offsets, the oracle
value of c_d there and the central moment M_d there (the mean of the products
of the oracle's centred columns), for:
  - ``count`` random offsets (padding entries of ragged blocks dropped),
  - every pure-diagonal entry (i, ..., i),
  - ``count // 3`` random copies in blocks with a repeated block index.

    python tests/golden/bench_expected.py        # about a minute on 8 cores
"""
from __future__ import annotations

import itertools
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "bench_expected.json")

# (case, data, n, b, orders, random offsets per order, seed of the sample draw)
def cases():
    for name in ["t-wishart-n16-t5000", "t-gamma-mix-n48-t100000", "laplace-mix-n24-t200000",
                 "ar1-garch-n64-t50000"]:
        w = workloads.WORKLOADS[name]
        yield name, (lambda name=name: workloads.generate(name)), w["n"], w["b"], range(2, w["d_max"] + 1), 300, 7
    for n, d_max in [(16, 8), (8, 10)]:
        yield (f"laplace-mix-n{n}-t20000-d{d_max}", (lambda n=n: workloads.laplace_mix(t=20_000, n=n, seed=1701006)),
               n, 2, range(d_max - 1, d_max + 1), 64, d_max)


class Layout:
    """Offsets of block storage (Section 2.1) for n variables, order d, block size b."""

    def __init__(self, n, d, b):
        self.n, self.d, self.b = n, d, b
        self.nbar = -(-n // b)
        self.rank = {tup: r for r, tup in enumerate(itertools.combinations_with_replacement(range(self.nbar), d))}
        self.elems = len(self.rank) * b ** d

    def offset(self, block, digits):
        inb = 0
        for x in digits:
            inb = inb * self.b + int(x)
        return self.rank[tuple(int(j) for j in block)] * self.b ** self.d + inb

    def sorted_offset(self, idx):
        i = sorted(int(x) for x in idx)
        return self.offset([x // self.b for x in i], [x % self.b for x in i])


def sample(lay, count, rng):
    n, d, b = lay.n, lay.d, lay.b
    offs = [int(o) for o in rng.choice(lay.elems, size=min(count, lay.elems), replace=False)]
    offs += [lay.sorted_offset([i] * d) for i in range(n)]
    copies = []
    while len(copies) < count // 3:
        j = np.sort(rng.integers(0, lay.nbar, size=d))
        k = rng.integers(1, d)
        j[k] = j[k - 1]
        i = rng.permutation(j * b + rng.integers(0, b, size=d))
        if i.max() >= n:
            continue
        order = np.argsort(i // b, kind="stable")
        copies.append(lay.offset(np.sort(i // b), [i[q] % b for q in order]))
    offs = np.unique(np.array(offs + copies, dtype=np.int64))
    idx = oracle.block_indices(n, d, b, offs)
    keep = idx[:, 0] >= 0
    offs, idx = offs[keep], idx[keep]
    # the layout used here and the oracle's offset-to-index map agree
    for o, ix in zip(offs, idx):
        assert lay.sorted_offset(ix) // b ** d == o // b ** d
        assert sorted(ix.tolist()) == sorted(oracle.block_indices(n, d, b, [lay.sorted_offset(ix)])[0].tolist())
    return offs, idx


def central_moment_at(Xc, idx):
    out = np.empty(len(idx))
    for s in range(0, len(idx), 32):
        sl = idx[s:s + 32]
        prod = Xc[:, sl[:, 0]].copy()
        for k in range(1, sl.shape[1]):
            prod *= Xc[:, sl[:, k]]
        out[s:s + 32] = prod.mean(axis=0)
    return out


def main():
    oracle.build()
    res = {"source": "oracle/ (dense FP64 definitions; eq. cum_r, Section 3.2, entry by entry) on the seeded "
                     "workloads of workloads.py; written by tests/golden/bench_expected.py",
           "cases": {}}
    for name, gen, n, b, orders, count, seed in cases():
        X = gen()
        _, Xc = oracle.center(X)
        rng = np.random.default_rng(seed)
        rec = {"n": n, "b": b, "t": int(X.shape[0]), "orders": {}}
        for d in orders:
            lay = Layout(n, d, b)
            offs, idx = sample(lay, count, rng)
            kappa = oracle.cumulant_at(Xc, idx.astype(np.int32))
            rec["orders"][str(d)] = {"offsets": offs.tolist(), "kappa": [float(v) for v in kappa],
                                     "moment": [float(v) for v in central_moment_at(Xc, idx)]}
            print(name, d, len(offs), flush=True)
        res["cases"][name] = rec
    with open(OUT, "w") as f:
        json.dump(res, f, separators=(",", ":"))
        f.write("\n")
    print(OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
