"""The oracle's sort of a large array, computed in parts on several host
threads: sort(a ++ b) = merge(sort(a), sort(b)).  The merge is the oracle's
(taking the first run on ties), so for keys the result is the unique sorted
arrangement, the same array oracle.sort returns; tests pin this identity on
the CPU (test_oracle.py).  Only the oracle's own functions run here."""
import concurrent.futures

import numpy as np

import oracle


def sort_in_parts(x, parts=8, threads=8):
    """oracle.sort(x), as `parts` contiguous pieces sorted concurrently and
    then merged pairwise (each merge level concurrently too)."""
    x = np.ascontiguousarray(x, dtype=np.int32)
    if x.size == 0:
        return x.copy()
    cuts = np.linspace(0, x.size, parts + 1).astype(np.int64)
    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        runs = list(ex.map(lambda i: oracle.sort(x[cuts[i]:cuts[i + 1]]), range(parts)))
        while len(runs) > 1:
            pairs = [(runs[i], runs[i + 1]) for i in range(0, len(runs) - 1, 2)]
            merged = list(ex.map(lambda ab: oracle.merge(ab[0], ab[1]), pairs))
            if len(runs) % 2:
                merged.append(runs[-1])
            runs = merged
    return runs[0]
