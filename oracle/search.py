"""Algorithm 1 (sec. 2.5).  GPU version: n candidates per iteration, argmin
of the path length over the non-discarded ones, reconstruction of the winner
from its random draw, update of x* and x_old.  CPU version: one candidate per
iteration, x_old <- x after every draw (``search_cpu_version``); the GPU
version with one worker is ``search_single_worker``.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Readings of the paper: the start evaluates the initial x with the gate
off and keeps its minimised units; a candidate starts from the units of its
base; x* is replaced only on a strict decrease of C (and then T* becomes the
winner's makespan); when every candidate is discarded x_old becomes the base;
the improvement indicator is 1 or 2 when x* improved through a field or a BP
move (Fig. 3 caption), else 0.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

from . import model as M
from .moves import FIELD, Move, apply_move, draw_move, exploit_draw, is_valid


@dataclasses.dataclass
class CandidateResult:
    key: int
    cost_km: float
    makespan_s: float
    flags: int
    evaluation: Optional[M.Evaluation]


def evaluate_move(inst, base: M.Solution, mv: Move, index: int, gate: str, t_star,
                  caps=None, embedded_min: bool = True) -> CandidateResult:
    if not is_valid(inst, base, mv):
        return CandidateResult(M.INF_KEY, M.INF, M.INF, M.FLAG_INVALID, None)
    ev = M.evaluate_solution(inst, apply_move(base, mv), caps, embedded_min)
    if not ev.feasible:
        return CandidateResult(M.INF_KEY, M.INF, M.INF, ev.flags, ev)
    return CandidateResult(M.candidate_key(ev, index, gate, t_star), ev.cost_km, ev.makespan_s,
                           M.candidate_flags(ev, gate, t_star), ev)


@dataclasses.dataclass
class TraceRow:
    it: int
    use_best: bool
    best_key: int
    cost_m: int          # C* after the iteration
    makespan_s: float    # T* after the iteration
    indicator: int       # 0, 1 (field move improved x*), 2 (BP move improved x*)


@dataclasses.dataclass
class SearchState:
    it: int
    x_best: M.Solution
    cost_best: int
    t_best: float
    x_old: M.Solution
    trace: List[TraceRow]


def with_units(sol: M.Solution, ev: M.Evaluation) -> M.Solution:
    out = sol.copy()
    out.hu_tour = list(ev.hu_tour)
    out.su_tour = list(ev.su_tour)
    return out


def start(inst, x0: M.Solution, caps=None, embedded_min: bool = True) -> SearchState:
    """Start of Alg. 1: summarise the initial solution as x*, cost it, x_old = x*."""
    ev = M.evaluate_solution(inst, x0, caps, embedded_min)
    assert ev.feasible
    xb = with_units(x0, ev)
    return SearchState(0, xb, ev.cost_m, ev.makespan_s, xb.copy(), [])


def candidate(job, i):
    """Key and result of candidate i of one iteration (job = the iteration's
    fixed arguments)."""
    inst, base, seed, it, inst_idx, fixed_field_bp, gate, t_star, caps, embedded_min = job
    mv = draw_move(inst, base, seed, it, i, inst_idx, fixed_field_bp)
    r = evaluate_move(inst, base, mv, i, gate, t_star, caps, embedded_min)
    return r.key, r


def step(inst, st: SearchState, seed: int, n: int, eps_threshold: int, gate: str = M.GATE_LE,
         inst_idx: int = 0, fixed_field_bp: bool = False, caps=None,
         embedded_min: bool = True, map_fn=None) -> SearchState:
    """One iteration of the loop of Algorithm 1 (GPU version).  ``map_fn(job,
    n)`` may return the n candidate keys computed elsewhere (e.g. by a process
    pool running ``candidate``); by default they are computed in turn."""
    it = st.it
    use_best = exploit_draw(seed, it, inst_idx, eps_threshold)
    base = st.x_best if use_best else st.x_old
    best = None
    best_key = M.INF_KEY
    job = (inst, base, seed, it, inst_idx, fixed_field_bp, gate, st.t_best, caps, embedded_min)
    keys = map_fn(job, n) if map_fn is not None else [candidate(job, i)[0] for i in range(n)]
    for i, k in enumerate(keys):
        if k < best_key:
            best_key, best = k, i
    if best is not None:
        mv = draw_move(inst, base, seed, it, best, inst_idx, fixed_field_bp)
        best = (mv, evaluate_move(inst, base, mv, best, gate, st.t_best, caps, embedded_min))
    indicator = 0
    if best is None:
        x_old = base
        xb, cb, tb = st.x_best, st.cost_best, st.t_best
    else:
        mv, r = best
        x_new = with_units(apply_move(base, mv), r.evaluation)
        xb, cb, tb = st.x_best, st.cost_best, st.t_best
        if r.evaluation.cost_m < st.cost_best:
            xb, cb, tb = x_new, r.evaluation.cost_m, r.evaluation.makespan_s
            indicator = 1 if mv.kind == FIELD else 2
        x_old = x_new
    trace = st.trace + [TraceRow(it, use_best, best_key, cb, tb, indicator)]
    return SearchState(it + 1, xb, cb, tb, x_old, trace)


def search(inst, x0: M.Solution, seed: int, n: int, iters: int, eps_threshold: int,
           gate: str = M.GATE_LE, inst_idx: int = 0, fixed_field_bp: bool = False,
           caps=None, embedded_min: bool = True, map_fn=None) -> SearchState:
    st = start(inst, x0, caps, embedded_min)
    for _ in range(iters):
        st = step(inst, st, seed, n, eps_threshold, gate, inst_idx, fixed_field_bp, caps,
                  embedded_min, map_fn)
    return st


def search_single_worker(inst, x0: M.Solution, seed: int, iters: int, eps_threshold: int,
                         gate: str = M.GATE_LE, inst_idx: int = 0, fixed_field_bp: bool = False,
                         caps=None, embedded_min: bool = True) -> SearchState:
    """Algorithm 1, GPU version with a single worker (n = 1), written out: each
    iteration draws one remove-and-reinsert move on the eq. (6) base; a
    candidate that fails eq. (2) or the makespan gate is discarded and x_old
    becomes the base (as when every worker's candidate is discarded);
    otherwise x_old becomes the candidate with its minimised units and x* is
    replaced on a strict decrease of C."""
    st = start(inst, x0, caps, embedded_min)
    for _ in range(iters):
        it = st.it
        use_best = exploit_draw(seed, it, inst_idx, eps_threshold)
        base = st.x_best if use_best else st.x_old
        mv = draw_move(inst, base, seed, it, 0, inst_idx, fixed_field_bp)
        r = evaluate_move(inst, base, mv, 0, gate, st.t_best, caps, embedded_min)
        xb, cb, tb = st.x_best, st.cost_best, st.t_best
        indicator = 0
        if r.key == M.INF_KEY:
            x_old = base
        else:
            x_old = with_units(apply_move(base, mv), r.evaluation)
            if r.evaluation.cost_m < st.cost_best:
                xb, cb, tb = x_old, r.evaluation.cost_m, r.evaluation.makespan_s
                indicator = 1 if mv.kind == FIELD else 2
        trace = st.trace + [TraceRow(it, use_best, r.key, cb, tb, indicator)]
        st = SearchState(it + 1, xb, cb, tb, x_old, trace)
    return st


def cpu_version_step(inst, st: SearchState, seed: int, eps_threshold: int, gate: str = M.GATE_LE,
                     inst_idx: int = 0, fixed_field_bp: bool = False, caps=None,
                     embedded_min: bool = True) -> SearchState:
    """One iteration of Algorithm 1, CPU version, as the algorithm states it:
    x is taken from x_old or x* by the eq. (6) rule; one random vertex of x is
    removed and reinserted; eq. (2) is checked and, if x is feasible, x is
    evaluated (the embedded HU and SU minimisation, path length, makespan
    gate); x* is replaced when x is feasible, not discarded by the gate and
    strictly cheaper; then x_old <- x whatever the checks gave.  x carries its
    minimised units when it was evaluated, else the units of the solution it
    came from; an x_old that breaks eq. (2) is kept, and later moves start
    from it.  The draw of iteration it is Philox block (0, it, inst, 0), as
    for candidate 0 of the GPU version."""
    it = st.it
    use_best = exploit_draw(seed, it, inst_idx, eps_threshold)
    x = st.x_best if use_best else st.x_old
    mv = draw_move(inst, x, seed, it, 0, inst_idx, fixed_field_bp)
    r = evaluate_move(inst, x, mv, 0, gate, st.t_best, caps, embedded_min)
    x = apply_move(x, mv) if is_valid(inst, x, mv) else x
    if r.evaluation is not None and r.evaluation.feasible:
        x = with_units(x, r.evaluation)
    xb, cb, tb = st.x_best, st.cost_best, st.t_best
    indicator = 0
    if r.key != M.INF_KEY and r.evaluation.cost_m < st.cost_best:
        xb, cb, tb = x, r.evaluation.cost_m, r.evaluation.makespan_s
        indicator = 1 if mv.kind == FIELD else 2
    trace = st.trace + [TraceRow(it, use_best, r.key, cb, tb, indicator)]
    return SearchState(it + 1, xb, cb, tb, x, trace)


def search_cpu_version(inst, x0: M.Solution, seed: int, iters: int, eps_threshold: int,
                       gate: str = M.GATE_LE, inst_idx: int = 0, fixed_field_bp: bool = False,
                       caps=None, embedded_min: bool = True) -> SearchState:
    """Algorithm 1, CPU version: the start, then ``iters`` calls of
    ``cpu_version_step``."""
    st = start(inst, x0, caps, embedded_min)
    for _ in range(iters):
        st = cpu_version_step(inst, st, seed, eps_threshold, gate, inst_idx, fixed_field_bp, caps,
                              embedded_min)
    return st


def eps_threshold(eps: float) -> int:
    """floor(eps * 2^32), in [0, 2^32]."""
    return int(eps * (1 << 32))
