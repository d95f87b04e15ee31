"""Initial solution of Algorithm 1 (sec. 2.5): BPs to tours, fields to BPs,
field order.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Readings of the paper: the BP-to-tour split gives each tour floor(N_B / N_T) BPs of
one nearest-neighbour chain from HQ, the last tour the residual (the symbol in
the paper's sentence is garbled); fields go to BPs in id order (the
deterministic rule the paper names); nearest means smallest road distance,
ties to the lowest id; every BP's field chain starts at HQ; units start in
contiguous id blocks of floor(N / N_T), residual to the last tour, unless the
instance fixes per-tour counts.
"""
from __future__ import annotations

from typing import Optional

from .model import HQ, Solution, bp_vertex, dist, field_vertex, supply_kg


def _nearest(inst, cur: int, pool, vertex_of):
    return min(pool, key=lambda k: (dist(inst, cur, vertex_of(inst, k)), k))


def bp_chain(inst):
    """BPs to tours: sequential nearest-neighbour search over BPs from HQ."""
    chain, left, cur = [], list(range(inst.n_bps)), HQ
    while left:
        b = _nearest(inst, cur, left, bp_vertex)
        chain.append(b)
        left.remove(b)
        cur = bp_vertex(inst, b)
    return chain


def split_blocks(n: int, n_tours: int, counts=None):
    """Owner tour of items 0..n-1 in contiguous blocks."""
    if counts is None:
        per = n // n_tours
        counts = [per] * (n_tours - 1) + [n - per * (n_tours - 1)]
    owner = []
    for g, c in enumerate(counts):
        owner += [g] * int(c)
    assert len(owner) == n
    return owner


def assign_fields(inst):
    """Fields to BPs: in id order to the closest BP whose demand is not yet
    met; once every demand is met, to the closest BP.  Returns the per-BP
    field lists (id order) or None if some demand stays unmet."""
    supplied = [0] * inst.n_bps
    fields = [[] for _ in range(inst.n_bps)]
    for f in range(inst.n_fields):
        unmet = [b for b in range(inst.n_bps) if supplied[b] < int(inst.bp_demand_kg[b])]
        pool = unmet if unmet else list(range(inst.n_bps))
        b = _nearest(inst, field_vertex(inst, f), pool, bp_vertex)
        fields[b].append(f)
        supplied[b] += supply_kg(inst, f)
    if any(supplied[b] < int(inst.bp_demand_kg[b]) for b in range(inst.n_bps)):
        return None
    return fields


def order_fields(inst, fs):
    """Field order: nearest-neighbour chain over one BP's fields, from HQ."""
    out, left, cur = [], list(fs), HQ
    while left:
        f = _nearest(inst, cur, left, field_vertex)
        out.append(f)
        left.remove(f)
        cur = field_vertex(inst, f)
    return out


def init_solution(inst) -> Optional[Solution]:
    chain = bp_chain(inst)
    NT = inst.n_tours
    per = inst.n_bps // NT
    tours = [chain[g * per:(g + 1) * per] for g in range(NT - 1)] + [chain[(NT - 1) * per:]]
    fields = assign_fields(inst)
    if fields is None:
        return None
    fields = [order_fields(inst, fs) for fs in fields]
    hu = split_blocks(inst.n_hus, NT, inst.init_hus_per_tour)
    su = split_blocks(inst.n_sus, NT, inst.init_sus_per_tour)
    return Solution(tours, fields, hu, su)


def init_feasible(inst) -> bool:
    """Acceptance predicate for the instance generator (the greedy field-to-BP assignment meets
    every demand)."""
    return assign_fields(inst) is not None
