"""Optional thread parallelism over the oracle's independent loops (test infrastructure).

Algorithm 1 runs steps 7-10 as a parallel loop over the active blocks, each block touching
only its own v_i, v~_i and statistics; the Psi^dagger of Sec. III is one analysis per
basis, each independent of the others.  ``pmap`` runs such a loop on a thread pool when
more than one worker is set (numpy releases the interpreter lock inside its array
loops), and serially otherwise.  Each item's arithmetic is the same either way, and the
caller combines the results in item order, so the results are bitwise identical for any
worker count.  The default is one worker.
"""
import concurrent.futures as cf

_workers = 1


def set_workers(n: int) -> None:
    global _workers
    _workers = max(1, int(n))


def workers() -> int:
    return _workers


def pmap(fn, items):
    items = list(items)
    if _workers <= 1 or len(items) <= 1:
        return [fn(i) for i in items]
    with cf.ThreadPoolExecutor(max_workers=min(_workers, len(items))) as ex:
        return list(ex.map(fn, items))
