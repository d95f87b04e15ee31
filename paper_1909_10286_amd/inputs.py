"""Seeded synthetic problem instances for the biomass-logistics search.

This module only draws raw instance data (coordinates, road distances, field
areas and yields, plant demands, the harvester and support-unit fleets).  It
holds none of the method's arithmetic: supplies, shuttle counts, completion
and waiting times, costs and every decision of the search are computed
independently by the CPU oracle (``oracle/``) and by the HIP library.  Both
sides take their inputs from here.

Recipes (all quantities are integers so that every decision of the method is
exact on both sides):

* Vertices: 0 is the headquarter (HQ), 1..N_B are the biogas plants (BPs),
  N_B+1..N_B+N_F are the fields.  The HQ sits at the origin, at the centre of
  an L x L square (paper sec. 3.1 places it at the origin; Fig. 1 draws it in
  the middle of the tours).
* Points are drawn uniformly in the square, or, for the clustered workload,
  as 20 Gaussian clusters (sigma 5 km) around uniform centres, field f in
  cluster f mod 20, clamped to the square.  Coordinates are rounded to metres.
* Road distance: rint(road_factor * Euclidean distance) in metres (the paper
  uses straight-line edges, sec. 3.1; the synthetic workloads add a 1.3 road
  factor).
* Field area in 0.01 ha, yield in 0.1 t/ha, so area*yield is the supply in kg
  exactly.  HU working rates in 0.01 ha/h; SU capacity in kg; SU road speed in
  m/h rounded to 100 m/h; HU road speed 40 km/h (Table 1).
* SU fill time proportional to capacity (sec. 2.1, seventh item): 6 min per
  12.5 t of Table 1, i.e. floor(capacity_kg * 288 / 10000) seconds.
* BP demands: 80 % of the total supply split equally, floor division (sec. 3.1
  gives equal demands per plant).

Draw order inside one numpy ``Generator(Philox(key))`` stream: BP xy, cluster
centres (clustered only), field xy, area, yield, HU rate, SU capacity, SU speed.
A redraw (when the caller's acceptance predicate rejects the instance, e.g. the
greedy initialisation cannot meet every demand) uses key = seed + attempt*2^64.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

HU_SPEED_MPH = 40_000          # Table 1: v_HU^edge = 40 km/h
FILL_S_PER_KG_NUM = 288        # Table 1: 6 min per 12.5 t = 28.8 s/t
FILL_S_PER_KG_DEN = 10_000


@dataclasses.dataclass
class Instance:
    """Raw instance data; every array is an integer numpy array."""
    name: str
    seed: int
    attempt: int
    n_fields: int
    n_bps: int
    n_tours: int
    n_hus: int
    n_sus: int
    xy_m: np.ndarray            # (V, 2) int64, metres; row 0 = HQ
    dist_m: np.ndarray          # (V, V) uint32, metres
    field_area: np.ndarray      # (N_F,) uint32, 0.01 ha
    field_yield: np.ndarray     # (N_F,) uint32, 0.1 t/ha
    bp_demand_kg: np.ndarray    # (N_B,) uint32
    hu_rate: np.ndarray         # (N_HU,) uint32, 0.01 ha/h
    su_cap_kg: np.ndarray       # (N_SU,) uint32
    su_speed_mph: np.ndarray    # (N_SU,) uint32, m/h
    su_fill_s: np.ndarray       # (N_SU,) uint32, s
    hu_speed_mph: int = HU_SPEED_MPH
    # Initial units per tour (contiguous id blocks).  None: equal split with the
    # residual on the last tour.
    init_hus_per_tour: Optional[np.ndarray] = None
    init_sus_per_tour: Optional[np.ndarray] = None

    @property
    def n_vertices(self) -> int:
        return 1 + self.n_bps + self.n_fields


@dataclasses.dataclass(frozen=True)
class InstanceSpec:
    name: str
    square_m: int
    n_fields: int
    n_bps: int
    n_tours: int
    n_hus: int
    n_sus: int
    clusters: int = 0
    sigma_m: float = 5_000.0
    road_factor: float = 1.3
    area_ha: tuple = (5.0, 50.0)
    yield_tpha: tuple = (35.0, 50.0)
    hu_rate_hah: tuple = (1.5, 3.0)
    su_cap_t: tuple = (15.0, 30.0)
    su_speed_kmh: tuple = (30.0, 50.0)
    demand_frac_num: int = 8
    demand_frac_den: int = 10


# The synthetic workloads.  Search sizes (candidates per iteration, iterations)
# are attached in WORKLOADS below.
# tiny12: 12 fields, 3 BPs, 2 tours, 4 HUs, 8 SUs, 50 km square.
# mid100: 100 fields, 10 BPs, 5 tours, 12 HUs, 40 SUs, 100 km square.
# clust500: 500 fields in 20 Gaussian clusters, 20 BPs, 10 tours, 30 HUs,
#           120 SUs, 200 km square.
SPECS = {
    "tiny12": InstanceSpec("tiny12", 50_000, 12, 3, 2, 4, 8),
    "mid100": InstanceSpec("mid100", 100_000, 100, 10, 5, 12, 40),
    "clust500": InstanceSpec("clust500", 200_000, 500, 20, 10, 30, 120, clusters=20),
}

WORKLOADS = {
    "tiny12": dict(n_cand=4096, iters=100),
    "mid100": dict(n_cand=1 << 20, iters=200),
    "clust500": dict(n_cand=1 << 22, iters=300),
    "batch256": dict(n_cand=1 << 16, iters=100, n_instances=256),
}


def _uniform_q(rng, lo, hi, size, scale):
    """Uniform draw in [lo, hi] quantised to 1/scale units (rint)."""
    return np.rint(rng.uniform(lo, hi, size) * scale).astype(np.int64)


def _distances(xy: np.ndarray, road_factor: float) -> np.ndarray:
    d = xy[:, None, :].astype(np.float64) - xy[None, :, :].astype(np.float64)
    e = np.sqrt((d * d).sum(axis=2))
    D = np.rint(road_factor * e).astype(np.uint32)
    return D


def _draw(spec: InstanceSpec, seed: int, attempt: int,
          hus_per_tour=None, sus_per_tour=None) -> Instance:
    rng = np.random.Generator(np.random.Philox(key=seed + (attempt << 64)))
    half = spec.square_m / 2.0
    NB, NF = spec.n_bps, spec.n_fields
    bp_xy = rng.uniform(-half, half, (NB, 2))
    if spec.clusters:
        centres = rng.uniform(-half, half, (spec.clusters, 2))
        off = rng.normal(0.0, spec.sigma_m, (NF, 2))
        field_xy = centres[np.arange(NF) % spec.clusters] + off
        field_xy = np.clip(field_xy, -half, half)
    else:
        field_xy = rng.uniform(-half, half, (NF, 2))
    area = _uniform_q(rng, *spec.area_ha, NF, 100)
    yld = _uniform_q(rng, *spec.yield_tpha, NF, 10)
    hu_rate = _uniform_q(rng, *spec.hu_rate_hah, spec.n_hus, 100)
    su_cap = _uniform_q(rng, *spec.su_cap_t, spec.n_sus, 1000)
    su_speed = _uniform_q(rng, *spec.su_speed_kmh, spec.n_sus, 10) * 100
    xy = np.concatenate([np.zeros((1, 2)), bp_xy, field_xy]).round().astype(np.int64)
    D = _distances(xy, spec.road_factor)
    total = int((area * yld).sum())
    demand = (spec.demand_frac_num * total) // (spec.demand_frac_den * NB)
    fill = (su_cap * FILL_S_PER_KG_NUM) // FILL_S_PER_KG_DEN
    return Instance(
        name=spec.name, seed=seed, attempt=attempt,
        n_fields=NF, n_bps=NB, n_tours=spec.n_tours, n_hus=spec.n_hus,
        n_sus=spec.n_sus, xy_m=xy, dist_m=D,
        field_area=area.astype(np.uint32), field_yield=yld.astype(np.uint32),
        bp_demand_kg=np.full(NB, demand, dtype=np.uint32),
        hu_rate=hu_rate.astype(np.uint32), su_cap_kg=su_cap.astype(np.uint32),
        su_speed_mph=su_speed.astype(np.uint32), su_fill_s=fill.astype(np.uint32),
        init_hus_per_tour=None if hus_per_tour is None else np.asarray(hus_per_tour, np.int64),
        init_sus_per_tour=None if sus_per_tour is None else np.asarray(sus_per_tour, np.int64),
    )


Accept = Callable[[Instance], bool]


def _first_accepted(draw, accept: Optional[Accept], max_attempts: int = 256) -> Instance:
    for attempt in range(max_attempts):
        inst = draw(attempt)
        if accept is None or accept(inst):
            return inst
    raise RuntimeError("no accepted instance within %d attempts" % max_attempts)


def make_instance(name: str, seed: int = 0, accept: Optional[Accept] = None) -> Instance:
    """Instance of one of the named single-instance workloads (SPECS)."""
    spec = SPECS[name]
    return _first_accepted(lambda a: _draw(spec, seed, a), accept)


def batch_member_spec(k: int) -> tuple:
    """Sizes of member k of the 256-instance batch workload.

    Fields U{20..300}, BPs U{3..15}, tours U{2..min(8, BPs)}, 2-3 HUs and
    4-10 SUs per tour, drawn from a stream keyed by (3 << 32) | k.
    """
    rng = np.random.Generator(np.random.Philox(key=(3 << 32) | k))
    nf = int(rng.integers(20, 301))
    nb = int(rng.integers(3, 16))
    nt = int(rng.integers(2, min(8, nb) + 1))
    hpt = rng.integers(2, 4, nt)
    spt = rng.integers(4, 11, nt)
    return nf, nb, nt, hpt, spt


def make_batch_instance(k: int, accept: Optional[Accept] = None) -> Instance:
    nf, nb, nt, hpt, spt = batch_member_spec(k)
    spec = InstanceSpec("batch256[%d]" % k, 50_000, nf, nb, nt, int(hpt.sum()), int(spt.sum()))
    seed = (3 << 32) | k
    return _first_accepted(lambda a: _draw(spec, seed + (1 << 40), a, hpt, spt), accept)


def make_custom_instance(name: str, seed: int, square_m: int, n_fields: int, n_bps: int,
                         n_tours: int, n_hus: int, n_sus: int, clusters: int = 0,
                         accept: Optional[Accept] = None, **kw) -> Instance:
    """Instance with the uniform-distribution recipe at arbitrary sizes (tests)."""
    spec = InstanceSpec(name, square_m, n_fields, n_bps, n_tours, n_hus, n_sus,
                        clusters=clusters, **kw)
    return _first_accepted(lambda a: _draw(spec, seed, a), accept)


def make_replica_instance(seed: int, accept: Optional[Accept] = None) -> Instance:
    """Paper-scale replica (sec. 3.1, Table 1): 1200 fields of 3 + 4u ha,
    20 BPs at 250 ha of demand, 80 km x 80 km, straight-line edges, 7 tours,
    7 HUs at 2.5 ha/h, 14 SUs of 12.5 t / 6 min and 28 SUs of 16.5 t / 8 min,
    40 km/h for every unit, 40 t/ha for every field."""
    def draw(attempt):
        rng = np.random.Generator(np.random.Philox(key=seed + (attempt << 64) + (2 << 96)))
        half = 40_000.0
        bp_xy = rng.uniform(-half, half, (20, 2))
        field_xy = rng.uniform(-half, half, (1200, 2))
        area = np.rint((3.0 + 4.0 * rng.uniform(0.0, 1.0, 1200)) * 100).astype(np.int64)
        xy = np.concatenate([np.zeros((1, 2)), bp_xy, field_xy]).round().astype(np.int64)
        D = _distances(xy, 1.0)
        # Ids in blocks of 6 per tour (2 small then 4 large), so that the
        # contiguous initial split gives Case 1's 2 + 4 SUs per tour.
        cap = np.array(([12_500] * 2 + [16_500] * 4) * 7, dtype=np.int64)
        fill = np.array(([360] * 2 + [480] * 4) * 7, dtype=np.int64)
        return Instance(
            name="replica", seed=seed, attempt=attempt, n_fields=1200, n_bps=20,
            n_tours=7, n_hus=7, n_sus=42, xy_m=xy, dist_m=D,
            field_area=area.astype(np.uint32),
            field_yield=np.full(1200, 400, dtype=np.uint32),
            bp_demand_kg=np.full(20, 250 * 40 * 1000, dtype=np.uint32),
            hu_rate=np.full(7, 250, dtype=np.uint32), su_cap_kg=cap.astype(np.uint32),
            su_speed_mph=np.full(42, 40_000, dtype=np.uint32),
            su_fill_s=fill.astype(np.uint32),
            init_hus_per_tour=np.ones(7, np.int64),
            init_sus_per_tour=np.full(7, 6, np.int64),
        )
    return _first_accepted(draw, accept)


SURROGATE_PARAMS = 16 * 128 + 128 * 128 + 136 * 64 + 64 * 2


def surrogate_init_words(seed: int) -> np.ndarray:
    """Uniform [0, 1) draws for the initial weights of the learned screen
    (W1 16x128, W2 128x128, W3 136x64, W4 64x2, row-major, in that order);
    the weights themselves are formed from these draws by each side."""
    rng = np.random.Generator(np.random.Philox(key=seed + (5 << 96)))
    return rng.random(SURROGATE_PARAMS)
