"""Pins of the float64 surrogate reference: analytic gradients against
central finite differences, and a hand-set network whose output is a
hand-computed function of the features."""
import numpy as np
import pytest

from oracle import init as OI
from oracle import model as M
from oracle import search as S
from oracle import surrogate as SG
from paper_1909_10286_amd import inputs

from .toys import build, load_golden


def _setup(name="tiny12", seed=0):
    inst = inputs.make_instance(name, seed, accept=OI.init_feasible)
    x0 = OI.init_solution(inst)
    st = S.start(inst, x0)
    sc = SG.scales(inst, st.cost_best, st.t_best)
    return inst, st.x_best, sc


@pytest.mark.parametrize("name", ["tiny12", "mid100"])
def test_gradient_matches_finite_differences(name):
    inst, x, sc = _setup(name)
    p = SG.init_params(inputs.surrogate_init_words(3))
    # Non-zero biases so that every ReLU sees both signs.
    rng = np.random.default_rng(0)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    ev = M.evaluate_solution(inst, x)
    L, g = SG.example_loss_and_grad(p, inst, x, sc, ev.cost_m, ev.makespan_s)
    eps = 1e-6
    for name_, idx in [("W1", (3, 5)), ("W1", (7, 100)), ("b1", (9,)), ("W2", (10, 20)),
                       ("W2", (127, 0)), ("b2", (64,)), ("W3", (5, 7)), ("W3", (130, 3)),
                       ("b3", (11,)), ("W4", (3, 0)), ("W4", (60, 1)), ("b4", (0,)), ("b4", (1,))]:
        q = {k: v.copy() for k, v in p.items()}
        q[name_][idx] += eps
        lp, _ = SG.example_loss_and_grad(q, inst, x, sc, ev.cost_m, ev.makespan_s)
        q[name_][idx] -= 2 * eps
        lm, _ = SG.example_loss_and_grad(q, inst, x, sc, ev.cost_m, ev.makespan_s)
        fd = (lp - lm) / (2 * eps)
        an = g[name_][idx]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9, (name_, idx, fd, an)


def test_hand_set_network_on_collinear_toy():
    """W1 = W2 = identity on the features, W3 routes the pooled leg feature
    (7) and the field-count feature (u4) to two hidden units, W4 reads them
    out: P = mean leg / Ds = (2000 + 3000 + 2000) / 3 / 10000, M = fields(g) /
    N_F = 1."""
    g = load_golden("collinear_toy.json")
    inst = build(g["xy_m"], g["n_bps"], g["n_tours"], g["field_area"], g["field_yield"],
                 g["bp_demand_kg"], g["hu_rate"], g["su_cap_kg"], g["su_speed_mph"],
                 g["su_fill_s"], road_factor=g["road_factor"])
    s = g["solution"]
    sol = M.Solution(s["tours"], s["fields"], s["hu_tour"], s["su_tour"])
    sc = SG.scales(inst, 1.0, 1.0)
    assert sc.d_s == 10000
    p = {"W1": np.zeros((16, 128)), "b1": np.zeros(128), "W2": np.eye(128), "b2": np.zeros(128),
         "W3": np.zeros((136, 64)), "b3": np.zeros(64), "W4": np.zeros((64, 2)), "b4": np.zeros(2)}
    p["W1"][:16, :16] = np.eye(16)
    p["W3"][7, 0] = 1.0
    p["W3"][128 + 4, 1] = 1.0
    p["W4"][0, 0] = 1.0
    p["W4"][1, 1] = 1.0
    P, Mk = SG.predict(p, inst, sol, sc)
    assert P == pytest.approx(7000 / 3 / 10000, rel=1e-12)
    assert Mk == pytest.approx(1.0, rel=1e-12)


def test_inactive_tours_are_masked():
    """A tour without fields adds nothing to P and is not in the max."""
    inst, x, sc = _setup("tiny12")
    y = x.copy()
    y.tours[1] = y.tours[0] + y.tours[1]
    y.tours[0] = []
    p = SG.init_params(inputs.surrogate_init_words(1))
    p["b4"] = np.array([5.0, 100.0])   # an unmasked empty tour would add 5 and win the max
    phi, u, fbp, btour, active = SG.features(inst, y, sc)
    assert list(active) == [False, True]
    P, Mk, cache = SG.forward(p, phi, u, fbp, btour, active, inst.n_bps)
    assert P == pytest.approx(cache["y"][1, 0]) and Mk == pytest.approx(cache["y"][1, 1])
