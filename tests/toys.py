"""Hand-built instances for the CPU tests (explicit arrays, no generator)."""
import json
import os

import numpy as np

from paper_1909_10286_amd.inputs import HU_SPEED_MPH, Instance

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def build(xy, n_bps, n_tours, area, yld, demand, hu_rate, su_cap, su_speed, su_fill,
          road_factor=1.0, name="toy", hus_per_tour=None, sus_per_tour=None):
    xy = np.asarray(xy, dtype=np.int64)
    d = xy[:, None, :].astype(np.float64) - xy[None, :, :].astype(np.float64)
    D = np.rint(road_factor * np.sqrt((d * d).sum(axis=2))).astype(np.uint32)
    nf = len(xy) - 1 - n_bps
    u32 = lambda a: np.asarray(a, dtype=np.uint32)
    return Instance(name=name, seed=0, attempt=0, n_fields=nf, n_bps=n_bps, n_tours=n_tours,
                    n_hus=len(hu_rate), n_sus=len(su_cap), xy_m=xy, dist_m=D,
                    field_area=u32(area), field_yield=u32(yld), bp_demand_kg=u32(demand),
                    hu_rate=u32(hu_rate), su_cap_kg=u32(su_cap), su_speed_mph=u32(su_speed),
                    su_fill_s=u32(su_fill), hu_speed_mph=HU_SPEED_MPH,
                    init_hus_per_tour=hus_per_tour, init_sus_per_tour=sus_per_tour)
