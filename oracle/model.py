"""Cost model, constraints and the embedded HU/SU minimisation (paper sec. 2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Every quantity is an exact Python integer: distances in metres, supplies in
kg, areas in 0.01 ha, working rates in 0.01 ha/h, speeds in m/h, times in
seconds.  "Infinite" times are ``math.inf``.  Every division is a floor
division of non-negative integers.

Readings of passages the paper leaves open:
  * supply s_f = area_f * yield_f (eq. (3) with a per-field yield);
  * shuttle drives n_f = ceil(s_f / c_bar) with c_bar the fleet-mean SU
    capacity, floor division (eq. (4) gives one count per SU class);
  * path length: every unit of tour g drives that tour's HU route
    HQ -> fields (BP order, field order) -> HQ, plus 2 * n_f * D[f][b_f] of
    shuttle driving per field (sec. 2.2);
  * completion time of a tour = road time of its route at the HU road speed
    plus its harvested area over the summed working rates of its HUs;
  * waiting time (eq. (5) and Alg. 2's mean BP distance): round trip of the mean
    field-to-BP distance of the tour at the critical SU's speed, minus the
    fill times of the other SUs of the tour divided by the tour's HU count;
    the critical SU has the largest fill time;
  * units are ranked HUs by (rate, id) and SUs by (fill time, -id); the
    critical SU is the last SU of its tour in that rank;
  * one generic min-max rebalancing routine serves both the HU step (sec. 2.5,
    first evaluation step, and its non-uniform variant) and Alg. 2.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

INF = math.inf
INF_KEY = (1 << 64) - 1

# Candidate flags (same bit values as the C interface documents).
FLAG_INFEASIBLE = 1
FLAG_GATED = 2
FLAG_CAP_HU = 4
FLAG_CAP_SU = 8
FLAG_INVALID = 16
FLAG_INF_MAKESPAN = 32

GATE_LE = "le"          # discard when T_max > T*  (default reading)
GATE_STRICT = "strict"  # discard when T_max >= T* (literal reading)
GATE_OFF = "off"        # no makespan gate (Case 2, and Alg. 1's start)

HQ = 0


@dataclasses.dataclass
class Solution:
    """The generic solution vector x (sec. 2.5, Alg. 1).

    tours[g]  : BP ids visited by tour g, in order          (levels i, ii)
    fields[b] : field ids assigned to BP b, in harvest order (levels iii, iv)
    hu_tour[h]: tour of HU h                                 (level v)
    su_tour[s]: tour of SU s                                 (level vi)
    """
    tours: List[List[int]]
    fields: List[List[int]]
    hu_tour: List[int]
    su_tour: List[int]

    def copy(self) -> "Solution":
        return Solution([list(t) for t in self.tours], [list(f) for f in self.fields],
                        list(self.hu_tour), list(self.su_tour))


def bp_vertex(inst, b: int) -> int:
    return 1 + b


def field_vertex(inst, f: int) -> int:
    return 1 + inst.n_bps + f


def dist(inst, u: int, v: int) -> int:
    return int(inst.dist_m[u][v])


# ---------------------------------------------------------------- supplies --

def supply_kg(inst, f: int) -> int:
    """eq. (3): s_f = c_f * h_f; 0.01 ha * 0.1 t/ha = 1 kg."""
    return int(inst.field_area[f]) * int(inst.field_yield[f])


def mean_capacity_kg(inst) -> int:
    return sum(int(c) for c in inst.su_cap_kg) // inst.n_sus


def shuttle_drives(inst, f: int) -> int:
    """eq. (4): ceil(s_f / capacity), with the fleet-mean capacity."""
    c = mean_capacity_kg(inst)
    return -(-supply_kg(inst, f) // c)


def shuttle_distance(inst, f: int, b: int) -> int:
    """sec. 2.2: each shuttle drive counts twice (field -> BP -> field)."""
    return 2 * shuttle_drives(inst, f) * dist(inst, field_vertex(inst, f), bp_vertex(inst, b))


def bp_supply(inst, sol: Solution, b: int) -> int:
    return sum(supply_kg(inst, f) for f in sol.fields[b])


def is_feasible(inst, sol: Solution) -> bool:
    """eq. (2): every BP receives at least its minimum demand."""
    return all(bp_supply(inst, sol, b) >= int(inst.bp_demand_kg[b]) for b in range(inst.n_bps))


# ---------------------------------------------------------------- geometry --

def tour_route(sol: Solution, g: int) -> List[int]:
    """Fields of tour g in visiting order: BPs in tour order, each BP's fields
    in harvest order.  HUs never visit BPs (sec. 2.1)."""
    return [f for b in sol.tours[g] for f in sol.fields[b]]


def is_active(sol: Solution, g: int) -> bool:
    return len(tour_route(sol, g)) > 0


def tour_length(inst, sol: Solution, g: int) -> int:
    """HQ -> first field -> ... -> last field -> HQ, metres; 0 if inactive."""
    route = tour_route(sol, g)
    if not route:
        return 0
    vs = [HQ] + [field_vertex(inst, f) for f in route] + [HQ]
    return sum(dist(inst, vs[k], vs[k + 1]) for k in range(len(vs) - 1))


def tour_area(inst, sol: Solution, g: int) -> int:
    return sum(int(inst.field_area[f]) for f in tour_route(sol, g))


def mean_bp_distance(inst, sol: Solution, b: int) -> int:
    """Mean field-to-BP distance of the fields of BP b (inner mean of Alg. 2's
    mean BP distance), floor division; the BP must hold at least one field."""
    fs = sol.fields[b]
    return sum(dist(inst, field_vertex(inst, f), bp_vertex(inst, b)) for f in fs) // len(fs)


def tour_mean_distance(inst, sol: Solution, g: int) -> int:
    """Outer mean of Alg. 2's mean BP distance over the BPs of tour g that hold fields."""
    bs = [b for b in sol.tours[g] if sol.fields[b]]
    if not bs:
        return 0
    return sum(mean_bp_distance(inst, sol, b) for b in bs) // len(bs)


# ------------------------------------------------------------------- times --

def hu_rank(inst, h: int):
    return (int(inst.hu_rate[h]), h)


def su_rank(inst, s: int):
    return (int(inst.su_fill_s[s]), -s)


def completion_time(inst, length_m: int, area: int, hus) -> float:
    """Completion time of a tour in seconds: road time of the route plus the
    harvested area over the tour's summed HU working rates; infinite for an
    active tour without HUs."""
    rate = sum(int(inst.hu_rate[h]) for h in hus)
    if rate == 0:
        return INF
    return (3600 * length_m) // inst.hu_speed_mph + (3600 * area) // rate


def critical_su(inst, sus) -> int:
    """The SU with the largest fill time (eq. (5), l^largest); ties go to the
    lowest id."""
    return max(sus, key=lambda s: su_rank(inst, s))


def waiting_time(inst, mean_dist_m: int, sus, n_hu: int) -> float:
    """HU waiting time of a tour (eq. (5) with the distance averaged as in Alg. 2), in
    seconds: round trip of the mean field-BP distance at the critical SU's
    speed, minus the summed fill times of the other SUs over the HU count."""
    if not sus or n_hu == 0:
        return INF
    s = critical_su(inst, sus)
    load = sum(int(inst.su_fill_s[u]) for u in sus)
    return (7200 * mean_dist_m) // int(inst.su_speed_mph[s]) - (load - int(inst.su_fill_s[s])) // n_hu


# ------------------------------------------------------------ rebalancing --

def rebalance(n_tours: int, active: List[bool], units: List[set],
              value: Callable[[int, set], float], rank: Callable[[int], tuple],
              cap: int):
    """Min-max rebalancing of units over tours (sec. 2.5 for HUs; Alg. 2 for
    SUs).  Returns (units per tour, rounds, cap_hit).

    One round: g_max is the active tour with the largest value and g2 the
    runner-up among the other active tours; the donor g_min is the tour with
    the smallest value (inactive tours count as -inf) among the tours other
    than g_max and g2 that hold units, else among those other than g_max.  The
    donor's units are tried in rank order: the first one whose move makes
    g_max's value drop below g2's value is moved, else the last one.  The round
    is kept if the largest value over active tours fell, otherwise it is undone
    and the loop ends.  At most ``cap`` rounds run; wanting another one sets
    cap_hit.
    """
    units = [set(u) for u in units]
    rounds = 0
    cap_hit = False
    while True:
        vals = {g: value(g, units[g]) for g in range(n_tours) if active[g]}
        if not vals:
            break
        top = max(vals.values())
        g_max = min(g for g in vals if vals[g] == top)
        rest = {g: v for g, v in vals.items() if g != g_max}
        g2 = None
        if rest:
            second = max(rest.values())
            g2 = min(g for g in rest if rest[g] == second)
        donors = [g for g in range(n_tours) if g not in (g_max, g2) and units[g]]
        if not donors:
            donors = [g for g in range(n_tours) if g != g_max and units[g]]
        if not donors:
            break
        if rounds == cap:
            cap_hit = True
            break
        dkey = {g: (vals[g] if active[g] else -INF) for g in donors}
        low = min(dkey.values())
        g_min = min(g for g in donors if dkey[g] == low)
        order = sorted(units[g_min], key=rank)
        for j, u in enumerate(order):
            trial = value(g_max, units[g_max] | {u})
            if g2 is None or trial < vals[g2] or j == len(order) - 1:
                break
        units[g_min].remove(u)
        units[g_max].add(u)
        rounds += 1
        new_top = max(value(g, units[g]) for g in range(n_tours) if active[g])
        if new_top < top:
            continue
        units[g_max].remove(u)
        units[g_min].add(u)
        break
    return units, rounds, cap_hit


def default_caps(inst):
    return inst.n_hus + inst.n_tours, inst.n_sus + inst.n_tours


# --------------------------------------------------------------- evaluate --

@dataclasses.dataclass
class Evaluation:
    feasible: bool
    cost_m: int = 0
    makespan_s: float = 0
    flags: int = 0
    hu_tour: Optional[List[int]] = None
    su_tour: Optional[List[int]] = None
    length_m: Optional[List[int]] = None
    area: Optional[List[int]] = None
    active: Optional[List[bool]] = None
    t_compl: Optional[List[float]] = None
    t_wait: Optional[List[float]] = None
    tour_cost_m: Optional[List[int]] = None
    hu_rounds: int = 0
    su_rounds: int = 0

    @property
    def cost_km(self) -> float:
        return self.cost_m / 1000.0


def evaluate_solution(inst, sol: Solution, caps=None, embedded_min: bool = True) -> Evaluation:
    """Evaluate x (sec. 2.5): check eq. (2); if feasible, minimise the maximum
    completion time by moving HUs, then the maximum waiting time by moving SUs
    (Alg. 2), starting from the units x carries; then the path length C."""
    if not is_feasible(inst, sol):
        return Evaluation(feasible=False, flags=FLAG_INFEASIBLE)
    NT = inst.n_tours
    cap_hu, cap_su = caps if caps is not None else default_caps(inst)
    active = [is_active(sol, g) for g in range(NT)]
    L = [tour_length(inst, sol, g) for g in range(NT)]
    A = [tour_area(inst, sol, g) for g in range(NT)]
    Dm = [tour_mean_distance(inst, sol, g) for g in range(NT)]
    hus = [{h for h in range(inst.n_hus) if sol.hu_tour[h] == g} for g in range(NT)]
    sus = [{s for s in range(inst.n_sus) if sol.su_tour[s] == g} for g in range(NT)]
    flags = 0
    hu_rounds = su_rounds = 0
    if embedded_min:
        hus, hu_rounds, hit = rebalance(
            NT, active, hus, lambda g, u: completion_time(inst, L[g], A[g], u),
            lambda h: hu_rank(inst, h), cap_hu)
        flags |= FLAG_CAP_HU if hit else 0
    t_compl = [completion_time(inst, L[g], A[g], hus[g]) if active[g] else None for g in range(NT)]
    n_hu = [len(hus[g]) for g in range(NT)]
    if embedded_min:
        sus, su_rounds, hit = rebalance(
            NT, active, sus, lambda g, u: waiting_time(inst, Dm[g], u, n_hu[g]),
            lambda s: su_rank(inst, s), cap_su)
        flags |= FLAG_CAP_SU if hit else 0
    t_wait = [waiting_time(inst, Dm[g], sus[g], n_hu[g]) if active[g] else None for g in range(NT)]
    tour_cost = []
    for g in range(NT):
        shuttle = sum(shuttle_distance(inst, f, b) for b in sol.tours[g] for f in sol.fields[b])
        tour_cost.append((len(hus[g]) + len(sus[g])) * L[g] + shuttle)
    makespan = max(t_compl[g] for g in range(NT) if active[g])
    if makespan == INF:
        flags |= FLAG_INF_MAKESPAN
    hu_tour = [0] * inst.n_hus
    su_tour = [0] * inst.n_sus
    for g in range(NT):
        for h in hus[g]:
            hu_tour[h] = g
        for s in sus[g]:
            su_tour[s] = g
    return Evaluation(True, sum(tour_cost), makespan, flags, hu_tour, su_tour, L, A, active,
                      t_compl, t_wait, tour_cost, hu_rounds, su_rounds)


def gated(makespan, gate: str, t_star) -> bool:
    """sec. 2.5, third evaluation step: candidates that do not decrease the
    best-so-far maximum completion time are discarded."""
    if gate == GATE_OFF:
        return False
    if gate == GATE_STRICT:
        return makespan >= t_star
    return makespan > t_star


def candidate_key(ev: Evaluation, index: int, gate: str, t_star) -> int:
    """Ranking key: (path length in metres) * 2^24 + candidate index, or
    INF_KEY for discarded candidates.  The minimum key is the arg-min of the
    path length with the lowest index winning ties (Alg. 1, GPU version)."""
    if not ev.feasible or gated(ev.makespan_s, gate, t_star):
        return INF_KEY
    return (ev.cost_m << 24) | index


def candidate_flags(ev: Evaluation, gate: str, t_star) -> int:
    f = ev.flags
    if ev.feasible and gated(ev.makespan_s, gate, t_star):
        f |= FLAG_GATED
    return f
