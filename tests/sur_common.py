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
