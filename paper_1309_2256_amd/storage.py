"""Base-2 accumulation storage of per-source loop results (appendix A.4, binary
storage system, fig. St).

Stochastic estimates are averages over sources, so the individual per-source
contractions need not be kept.  Sources are numbered from 1 and source n goes
into bin k = floor(log2 n): bin k holds the sum of sources 2^k .. 2^(k+1) - 1,
i.e. of 2^k sources when complete ("File.1, File.2, File.4, File.8 ...").  An
estimate over any n sources is rebuilt from the bins selected by the binary
digits of n, so N sources take O(log2 N) stored arrays instead of O(N).  Only
one subset of sources is reachable for a given n (the bins are sums); every
n up to the number of sources in complete bins is reachable.

The arrays are whatever the library returns per source (for example the
[n_est][n_mom][16][Lt] momentum-resolved loops of one noise); this module is
host-side bookkeeping and file I/O, no arithmetic beyond the sums.
"""
import json
import os

import numpy as np


class Base2Store:
    """Accumulates per-source arrays of one shape into base-2 bins."""

    def __init__(self, shape, dtype=np.complex128):
        self.shape = tuple(shape)
        self.dtype = np.dtype(dtype)
        self.sums = []      # sums[k]: sum of the sources 2^k .. 2^(k+1) - 1 added so far
        self.counts = []    # counts[k]: how many of them were added
        self.n = 0

    def add(self, x):
        x = np.asarray(x)
        if x.shape != self.shape:
            raise ValueError("shape %s, store holds %s" % (x.shape, self.shape))
        self.n += 1
        k = self.n.bit_length() - 1
        if k == len(self.sums):
            self.sums.append(np.zeros(self.shape, dtype=self.dtype))
            self.counts.append(0)
        self.sums[k] += x
        self.counts[k] += 1

    def add_many(self, xs):
        for x in xs:
            self.add(x)

    def complete(self, k):
        return k < len(self.counts) and self.counts[k] == 1 << k

    def max_reachable(self):
        """Largest n for which every m <= n can be rebuilt (complete bins only)."""
        m = 0
        while self.complete(m):
            m += 1
        return (1 << m) - 1

    def sources(self, n):
        """1-based source numbers that the estimate over n sources uses."""
        out = []
        for k in self._bins(n):
            out.extend(range(1 << k, (1 << (k + 1))))
        return out

    def total(self, n):
        """Sum over the n sources selected by the binary digits of n."""
        acc = np.zeros(self.shape, dtype=self.dtype)
        for k in self._bins(n):
            acc += self.sums[k]
        return acc

    def mean(self, n):
        return self.total(n) / n

    def _bins(self, n):
        if n < 1:
            raise ValueError("n must be >= 1")
        bins = [k for k in range(n.bit_length()) if (n >> k) & 1]
        for k in bins:
            if not self.complete(k):
                raise ValueError("estimate over %d sources needs bin %d (%d sources) complete; "
                                 "%d added" % (n, k, 1 << k, self.n))
        return bins

    # ------------------------------------------------------------ files
    def save(self, directory, prefix="loops"):
        """One binary file per bin, prefix.<weight>.npy, plus prefix.index.json
        with the shape, dtype and the number of sources in each bin."""
        os.makedirs(directory, exist_ok=True)
        for k, s in enumerate(self.sums):
            np.save(os.path.join(directory, "%s.%d.npy" % (prefix, 1 << k)), s, allow_pickle=False)
        meta = {"shape": list(self.shape), "dtype": self.dtype.str, "counts": self.counts,
                "n_sources": self.n}
        with open(os.path.join(directory, prefix + ".index.json"), "w") as f:
            json.dump(meta, f)

    @classmethod
    def load(cls, directory, prefix="loops"):
        with open(os.path.join(directory, prefix + ".index.json")) as f:
            meta = json.load(f)
        st = cls(meta["shape"], np.dtype(meta["dtype"]))
        st.counts = [int(c) for c in meta["counts"]]
        st.n = int(meta["n_sources"])
        st.sums = [np.load(os.path.join(directory, "%s.%d.npy" % (prefix, 1 << k)), allow_pickle=False)
                   for k in range(len(st.counts))]
        for k, s in enumerate(st.sums):
            if s.shape != st.shape or s.dtype != st.dtype:
                raise ValueError("bin %d: shape %s dtype %s, index says %s %s"
                                 % (k, s.shape, s.dtype, st.shape, st.dtype))
        return st
