"""Helpers shared by the GPU tests: oracle <-> library marshalling and the
element-by-element comparison of candidate results."""
import math

import numpy as np

from oracle import model as M
from oracle import moves as MV
from oracle import search as S
from paper_1909_10286_amd import bl

COST_RTOL = 1e-5   # FP32 cost vs the float64 oracle


def to_csr(sol: M.Solution) -> bl.CSR:
    return bl.CSR.from_lists(sol.tours, sol.fields, sol.hu_tour, sol.su_tour)


def from_csr(c: bl.CSR) -> M.Solution:
    t, f, h, s = c.to_lists()
    return M.Solution(t, f, h, s)


def gate_of(flags: int) -> str:
    if flags & bl.GATE_OFF:
        return M.GATE_OFF
    if flags & bl.GATE_STRICT:
        return M.GATE_STRICT
    return M.GATE_LE


def caps_of(inst, cap_hu=0, cap_su=0):
    d = M.default_caps(inst)
    return (cap_hu or d[0], cap_su or d[1])


def oracle_batch(inst, base, words, t_star, flags=0, caps=None):
    """Oracle results for encoded move words, in the library's output format."""
    gate = gate_of(flags)
    emb = not (flags & bl.NO_EMBEDDED_MIN)
    key = np.empty(len(words), np.uint64)
    cost = np.empty(len(words), np.float64)
    mk = np.empty(len(words), np.int64)
    fl = np.empty(len(words), np.uint8)
    for i, w in enumerate(words):
        r = S.evaluate_move(inst, base, MV.decode(int(w)), i, gate, t_star, caps, emb)
        key[i] = r.key
        cost[i] = r.cost_km
        mk[i] = bl.INF_MAKESPAN if (r.makespan_s == math.inf or r.makespan_s >= bl.INF_MAKESPAN) \
            else int(r.makespan_s)
        fl[i] = r.flags
    return key, cost, mk, fl


def compare(gpu, orc, label=""):
    gk, gc, gm, gf = gpu
    ok, oc, om, of = orc
    bad = np.nonzero(gk != ok)[0]
    assert bad.size == 0, "%s key mismatch at %s: gpu %s oracle %s" % (
        label, bad[:5], gk[bad[:5]], ok[bad[:5]])
    bad = np.nonzero(gf != of)[0]
    assert bad.size == 0, "%s flags mismatch at %s: gpu %s oracle %s" % (
        label, bad[:5], gf[bad[:5]], of[bad[:5]])
    bad = np.nonzero(gm.astype(np.int64) != om)[0]
    assert bad.size == 0, "%s makespan mismatch at %s: gpu %s oracle %s" % (
        label, bad[:5], gm[bad[:5]], om[bad[:5]])
    fin = np.isfinite(oc)
    assert np.array_equal(np.isfinite(gc), fin), label + " cost finiteness mismatch"
    rel = np.abs(gc[fin].astype(np.float64) - oc[fin]) / np.maximum(oc[fin], 1e-300)
    assert rel.size == 0 or rel.max() <= COST_RTOL, "%s cost rel err %g" % (label, rel.max())


def oracle_words(inst, base, seed, it, n, first=0, inst_idx=0, fixed=False):
    return np.array([MV.encode(MV.draw_move(inst, base, seed, it, first + i, inst_idx, fixed))
                     for i in range(n)], dtype=np.uint64)
