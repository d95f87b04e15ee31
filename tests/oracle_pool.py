"""Process pool that runs oracle candidate evaluations in parallel (tests and
the CPU-baseline leg of the benchmark).  Workers are started with 'spawn', so
they never inherit a GPU runtime."""
import multiprocessing as mp
import os

from oracle import search as S


def _keys(args):
    job, lo, hi = args
    return [S.candidate(job, i)[0] for i in range(lo, hi)]


def _results(args):
    job, lo, hi = args
    out = []
    for i in range(lo, hi):
        _, r = S.candidate(job, i)
        out.append((r.key, r.cost_km, r.makespan_s, r.flags))
    return out


def _results_at(args):
    job, idx = args
    out = []
    for i in idx:
        _, r = S.candidate(job, int(i))
        out.append((r.key, r.cost_km, r.makespan_s, r.flags))
    return out


def n_procs():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


class OraclePool:
    def __init__(self, procs=None):
        self.procs = procs or n_procs()
        self._pool = mp.get_context("spawn").Pool(self.procs)

    def _chunks(self, job, n, lo=0):
        step = max(1, n // (self.procs * 4))
        return [(job, a, min(lo + n, a + step)) for a in range(lo, lo + n, step)]

    def __call__(self, job, n):
        out = []
        for part in self._pool.map(_keys, self._chunks(job, n)):
            out += part
        return out

    def results(self, job, n, lo=0):
        out = []
        for part in self._pool.map(_results, self._chunks(job, n, lo)):
            out += part
        return out

    def results_at(self, job, idx):
        """(key, cost km, makespan s, flags) of the candidates with the given
        indices, in that order."""
        idx = [int(i) for i in idx]
        step = max(1, len(idx) // (self.procs * 4))
        out = []
        for part in self._pool.map(_results_at, [(job, idx[a:a + step]) for a in range(0, len(idx), step)]):
            out += part
        return out

    def results_multi(self, pairs):
        """For each (job, indices) pair, the results of those candidates (as
        results_at), one pair per task."""
        return self._pool.map(_results_at, [(job, [int(i) for i in idx]) for job, idx in pairs])

    def close(self):
        self._pool.terminate()
        self._pool.join()
