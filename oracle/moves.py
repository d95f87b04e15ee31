"""The move of Algorithm 1: remove one vertex (field or BP) and reinsert it
(sec. 2.5), drawn from the counter-based generator.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Readings of the paper: the vertex is uniform over the N_F + N_B
vertices; a field goes to a uniform BP (its own included; with the fixed
field-to-BP variant of sec. 2.6 it stays in its own BP), a BP to a uniform tour
(its own included) and carries all of its fields; the slot is uniform over the
positions of the destination list after the removal.  Uniform words map to
ranges by multiply-shift.  Candidate i of iteration t of instance k uses the
Philox-4x32-10 block with counter (i, t, k, 0); the exploration draw of
eq. (6) uses counter (0, t, k, 1).

Move record (64 bits): bits 0-14 vertex (field id or BP id), bit 15 kind
(0 field, 1 BP), bits 16-31 destination (BP or tour), bits 32-47 slot,
bits 48-63 zero.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

from .model import Solution
from .philox import draw_words, scale

FIELD = 0
BP = 1


@dataclasses.dataclass(frozen=True)
class Move:
    kind: int
    vertex: int
    dst: int
    slot: int


def encode(mv: Move) -> int:
    return mv.vertex | (mv.kind << 15) | (mv.dst << 16) | (mv.slot << 32)


def decode(word: int) -> Move:
    return Move((word >> 15) & 1, word & 0x7FFF, (word >> 16) & 0xFFFF, (word >> 32) & 0xFFFF)


def bp_of_field(sol: Solution, f: int) -> int:
    for b, fs in enumerate(sol.fields):
        if f in fs:
            return b
    raise KeyError(f)


def tour_of_bp(sol: Solution, b: int) -> int:
    for g, bs in enumerate(sol.tours):
        if b in bs:
            return g
    raise KeyError(b)


def draw_move(inst, sol: Solution, seed: int, it: int, i: int, inst_idx: int = 0,
              fixed_field_bp: bool = False) -> Move:
    w = draw_words(seed, i, it, inst_idx, 0)
    v = scale(w[0], inst.n_fields + inst.n_bps)
    if v < inst.n_fields:
        src = bp_of_field(sol, v)
        dst = src if fixed_field_bp else scale(w[1], inst.n_bps)
        room = len(sol.fields[dst]) - (1 if dst == src else 0)
        return Move(FIELD, v, dst, scale(w[2], room + 1))
    b = v - inst.n_fields
    src = tour_of_bp(sol, b)
    dst = scale(w[1], inst.n_tours)
    room = len(sol.tours[dst]) - (1 if dst == src else 0)
    return Move(BP, b, dst, scale(w[2], room + 1))


def exploit_draw(seed: int, it: int, inst_idx: int, eps_threshold: int) -> bool:
    """eq. (6): the base is x* when u < eps.  u is the first word of block
    (0, t, k, 1); eps_threshold = floor(eps * 2^32) in [0, 2^32]."""
    return draw_words(seed, 0, it, inst_idx, 1)[0] < eps_threshold


def is_valid(inst, sol: Solution, mv: Move) -> bool:
    if mv.kind == FIELD:
        if mv.vertex >= inst.n_fields or mv.dst >= inst.n_bps:
            return False
        src = bp_of_field(sol, mv.vertex)
        room = len(sol.fields[mv.dst]) - (1 if mv.dst == src else 0)
    else:
        if mv.vertex >= inst.n_bps or mv.dst >= inst.n_tours:
            return False
        src = tour_of_bp(sol, mv.vertex)
        room = len(sol.tours[mv.dst]) - (1 if mv.dst == src else 0)
    return mv.slot <= room


def apply_move(sol: Solution, mv: Move) -> Solution:
    """Remove the vertex from its list and insert it at the slot of the
    destination list (a BP keeps its whole field list)."""
    out = sol.copy()
    if mv.kind == FIELD:
        src = bp_of_field(out, mv.vertex)
        out.fields[src].remove(mv.vertex)
        out.fields[mv.dst].insert(mv.slot, mv.vertex)
    else:
        src = tour_of_bp(out, mv.vertex)
        out.tours[src].remove(mv.vertex)
        out.tours[mv.dst].insert(mv.slot, mv.vertex)
    return out


def noop_move(sol: Solution) -> Optional[Move]:
    """A move that leaves x unchanged: some field reinserted where it was."""
    for b, fs in enumerate(sol.fields):
        if fs:
            return Move(FIELD, fs[0], b, 0)
    return None
