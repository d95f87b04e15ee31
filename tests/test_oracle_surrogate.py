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


# ------------------------------------------------------------------- Adam --

def _rand_params(rng):
    return {"W": rng.normal(0, 1, (5, 3)), "b": rng.normal(0, 1, 3)}


def test_adam_first_step_closed_form():
    """Kingma and Ba (2015), Algorithm 1, at t = 1: the bias corrections undo
    the (1 - beta) factors, so the step is -lr g / (|g| + eps) element-wise,
    whatever beta1 and beta2 are."""
    rng = np.random.default_rng(1)
    p, g = _rand_params(rng), _rand_params(rng)
    zero = {k: np.zeros_like(v) for k, v in p.items()}
    for beta1, beta2 in ((0.9, 0.999), (0.5, 0.9)):
        q, m, v = SG.adam_step(p, g, zero, zero, 1, 1e-3, beta1, beta2, 1e-8)
        for k in p:
            np.testing.assert_allclose(q[k] - p[k], -1e-3 * g[k] / (np.abs(g[k]) + 1e-8),
                                       rtol=1e-12, atol=1e-18)
            np.testing.assert_allclose(m[k], (1 - beta1) * g[k], rtol=1e-15)
            np.testing.assert_allclose(v[k], (1 - beta2) * g[k] ** 2, rtol=1e-15)


def test_adam_constant_gradient_steps():
    """With the same gradient every step, m_t = (1 - beta1^t) g and v_t = (1 -
    beta2^t) g^2 exactly (geometric sums), so every step is -lr g / (|g| +
    eps): after k steps p moved by -k lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    p, g = _rand_params(rng), _rand_params(rng)
    m = v = {k: np.zeros_like(x) for k, x in p.items()}
    q = p
    for t in range(1, 8):
        q, m, v = SG.adam_step(q, g, m, v, t, 2e-3, 0.9, 0.99, 1e-6)
    for k in p:
        np.testing.assert_allclose(q[k] - p[k], -7 * 2e-3 * g[k] / (np.abs(g[k]) + 1e-6), rtol=1e-9)


def test_adam_matches_torch_optimizer():
    """The library routine: torch.optim.Adam on float64 CPU tensors (same
    definition, no weight decay, no amsgrad) over six steps of varying
    gradients."""
    import torch
    rng = np.random.default_rng(3)
    p = _rand_params(rng)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=5e-3, betas=(0.8, 0.95), eps=1e-7)
    m = v = {k: np.zeros_like(x) for k, x in p.items()}
    q = p
    for t in range(1, 7):
        g = _rand_params(rng)
        for k in tp:
            tp[k].grad = torch.tensor(g[k], dtype=torch.float64)
        opt.step()
        q, m, v = SG.adam_step(q, g, m, v, t, 5e-3, 0.8, 0.95, 1e-7)
    for k in p:
        np.testing.assert_allclose(q[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15)


def _bf16(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def test_rounding_model_gradient():
    """The error model behind the GPU gradient tolerance.  Without
    perturbation it is the oracle's gradient (its factoring, rows projected
    by W3 before pooling, is the same function).  Its spread covers the
    rounding the device certainly does: the float64 gradient at the
    bf16-rounded W1, W2, W3 rows and features stays within 8 estimated
    standard deviations of the unrounded one, element by element."""
    from oracle import moves as MV

    from .sur_common import draw_moves, flat, rounding_model_gradient, unflat
    inst, _, sc = _setup("tiny12")
    st = S.start(inst, OI.init_solution(inst))
    p = SG.init_params(inputs.surrogate_init_words(3))
    rng = np.random.default_rng(3)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    p = unflat(flat(p))
    pw = dict(p, W1=_bf16(p["W1"]), W2=_bf16(p["W2"]))
    pw["W3"] = np.concatenate([_bf16(p["W3"][:SG.D_H]), p["W3"][SG.D_H:]])
    keys = [0x5EED0000 + 7919 * j for j in range(12)]
    g0, g1, draws = {}, {}, [{} for _ in keys]

    def add(acc, g):
        for k in g:
            acc[k] = acc.get(k, 0) + g[k]
    for mv in draw_moves(inst, st.x_best, 24, seed=11):
        sol = MV.apply_move(st.x_best, mv)
        ev = M.evaluate_solution(inst, sol)
        _, g = SG.example_loss_and_grad(p, inst, sol, sc, ev.cost_m, ev.makespan_s)
        add(g0, g)
        gm = rounding_model_gradient(p, inst, sol, sc, ev.cost_m, ev.makespan_s)
        for k in g:
            np.testing.assert_allclose(gm[k], g[k], rtol=1e-10, atol=1e-12 * np.abs(g[k]).max())
        phi, u, fbp, btour, active = SG.features(inst, sol, sc)
        P, Mk, c = SG.forward(pw, _bf16(phi), u, fbp, btour, active, inst.n_bps)
        add(g1, SG.backward(pw, c, P, Mk, ev.cost_m / sc.c0, ev.makespan_s / sc.t0))
        for d, key in zip(draws, keys):
            add(d, rounding_model_gradient(p, inst, sol, sc, ev.cost_m, ev.makespan_s, key))
    for k in g0:
        sig = np.sqrt(np.mean([(d[k] - g0[k]) ** 2 for d in draws], axis=0))
        assert np.all(np.abs(g1[k] - g0[k]) <= 8.0 * sig + 1e-9 * np.abs(g0[k]).max()), k
