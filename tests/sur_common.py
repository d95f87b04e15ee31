"""Helpers shared by the GPU tests of the learned screen: a surrogate with
seeded weights on an instance whose search has started from its initial
solution, and oracle-drawn moves."""
import numpy as np

from oracle import init as OI
from oracle import model as M
from oracle import moves as MV
from oracle import search as S
from oracle import surrogate as SG
from paper_1909_10286_amd import bl, inputs

from .gpu_common import to_csr


def flat(p):
    return np.concatenate([p[k].reshape(-1) for k, _ in bl.SUR_SHAPES]).astype(np.float32)


def unflat(w):
    out, k = {}, 0
    for name, shape in bl.SUR_SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(w[k:k + n], dtype=np.float64).reshape(shape)
        k += n
    return out


def setup(ctx, name, wseed=3, max_examples=512):
    """(instance, search state at start, instance id, surrogate id, float64
    weights rounded to float32, scales)."""
    inst = inputs.make_instance(name, 0, accept=OI.init_feasible)
    st = S.start(inst, OI.init_solution(inst))
    iid = ctx.instance_upload(inst)
    ctx.solution_upload(iid, bl.SLOT_BASE, to_csr(st.x_best))
    p = SG.init_params(inputs.surrogate_init_words(wseed))
    rng = np.random.default_rng(wseed)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    p = unflat(flat(p))
    sur = ctx.sur_create(iid, flat(p), float(st.cost_best), float(st.t_best), max_examples=max_examples)
    sc = SG.scales(inst, st.cost_best, st.t_best)
    return inst, st, iid, sur, p, sc


def draw_moves(inst, base, n, seed=7, feasible_only=True):
    out = []
    i = 0
    while len(out) < n:
        mv = MV.draw_move(inst, base, seed, 0, i)
        i += 1
        if feasible_only and not M.is_feasible(inst, MV.apply_move(base, mv)):
            continue
        out.append(mv)
    return out



# bf16 round to nearest: relative error at most 2^-8 (8 significant bits).
BF16_U = 2.0 ** -8


def value_hash_uniform(x, key):
    """Numbers in [-1, 1) that depend only on the float64 value of each
    element of x and on an integer key (splitmix64 of the value's bits xor
    the key): equal values get equal numbers under one key."""
    z = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64) ^ np.uint64(key)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0


def rounding_model_gradient(p, inst, sol, sc, cost_m, makespan_s, key=None):
    """Loss gradient of one example, in float64, factored as the training
    kernels compute it (each field row projected by the first 128 rows of W3
    before pooling; the same function as oracle.surrogate's, since pooling is
    linear), with a relative perturbation of up to BF16_U at every point where
    the kernels round an operand to bf16: the features, W1, W2, the first 128
    rows of W3, the hidden rows h1 and h2, the per-row projection gradient and
    the error signals dz2 and dz1.  key = None: no perturbation, and the
    result is oracle.surrogate's gradient up to float64 rounding.  With an
    integer key (one per draw of the model, the same for every example of
    the draw), each perturbation is in [-BF16_U, BF16_U] (relative) and
    a function of the value being rounded (value_hash_uniform), as rounding
    is: a field's features, and the hidden rows of fields a move leaves
    unchanged, are the same in every example and round the same way, so their
    errors add up across examples instead of averaging out.  The spread over
    draws is the error model of the device's gradient."""
    from oracle import surrogate as SG

    def r(x):
        return x if key is None else x * (1.0 + BF16_U * value_hash_uniform(x, key))
    phi, u, fbp, btour, active = SG.features(inst, sol, sc)
    nb, nt, H = inst.n_bps, inst.n_tours, SG.D_H
    w1, w2, w3e = r(p["W1"]), r(p["W2"]), r(p["W3"][:H])
    x = r(phi)
    z1 = x @ w1 + p["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ w2 + p["b2"]
    h2 = r(np.maximum(z2, 0.0))
    prow = h2 @ w3e
    cb = np.bincount(fbp, minlength=nb).astype(np.float64)
    cg = np.bincount(btour, minlength=nt).astype(np.float64)
    eb = np.zeros((nb, prow.shape[1]))
    np.add.at(eb, fbp, prow)
    eb /= np.maximum(cb, 1)[:, None]
    eg = np.zeros((nt, prow.shape[1]))
    np.add.at(eg, btour, eb)
    eg /= np.maximum(cg, 1)[:, None]
    z3 = eg + u @ p["W3"][H:] + p["b3"]
    a = np.maximum(z3, 0.0)
    y = a @ p["W4"] + p["b4"]
    act = np.nonzero(active)[0]
    P = y[act, 0].sum()
    gm = act[np.argmax(y[act, 1])]
    dy = np.zeros_like(y)
    dy[act, 0] = 2.0 * (P - cost_m / sc.c0)
    dy[gm, 1] += 2.0 * (y[gm, 1] - makespan_s / sc.t0)
    g = {"W4": a.T @ dy, "b4": dy.sum(0)}
    dz3 = (dy @ p["W4"].T) * (z3 > 0)
    g["b3"] = dz3.sum(0)
    deb = dz3[btour] / np.maximum(cg[btour], 1)[:, None] * (cg[btour] > 0)[:, None]
    dprow = r(deb[fbp] / cb[fbp][:, None])
    g["W3"] = np.concatenate([h2.T @ dprow, u.T @ dz3], axis=0)
    dz2f = (dprow @ w3e.T) * (h2 > 0)
    g["b2"] = dz2f.sum(0)
    dz2 = r(dz2f)
    g["W2"] = h1.T @ dz2
    dz1f = (dz2 @ w2.T) * (h1 > 0)
    g["b1"] = dz1f.sum(0)
    g["W1"] = x.T @ r(dz1f)
    return g
