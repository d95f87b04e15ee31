"""The paper-scale replica workload (sec. 3.1, Table 1: 1200 fields, 20 BPs,
7 tours, 7 HUs of one rate, SUs in two classes of one fill time each) on the
GPU against the oracle.  Its fleet is the one workload where the tie rules
of the unit moves decide: every HU has the same rate, and 14 and 28 SUs
share two fill times.  Cases 2-4 of sec. 3.2 as instance flags."""
import sys

import numpy as np
import pytest

from oracle import init as OI
from oracle import model as M
from oracle import moves as MV
from oracle import search as S
from paper_1909_10286_amd import bl, inputs

from .gpu_common import compare, from_csr, to_csr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# Case 2: fields stay with their BP, units never move, no makespan gate;
# Case 3: fields stay with their BP; Case 4: the plain method.
CASES = {2: bl.FIXED_FIELD_BP | bl.NO_EMBEDDED_MIN | bl.GATE_OFF, 3: bl.FIXED_FIELD_BP, 4: 0}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _replica():
    return inputs.make_replica_instance(0, accept=OI.init_feasible)


def _gate(flags):
    return M.GATE_OFF if flags & bl.GATE_OFF else M.GATE_LE


def _pool_batch(pool, inst, base, seed, it, n, flags, t_star):
    """Oracle results of candidates 0..n-1 of (seed, it) against `base`,
    in the library's output format."""
    job = (inst, base, seed, it, 0, bool(flags & bl.FIXED_FIELD_BP), _gate(flags), t_star, None,
           not (flags & bl.NO_EMBEDDED_MIN))
    rs = pool.results(job, n)
    key = np.array([r[0] for r in rs], np.uint64)
    cost = np.array([r[1] for r in rs], np.float64)
    mk = np.array([bl.INF_MAKESPAN if r[2] == M.INF or r[2] >= bl.INF_MAKESPAN else int(r[2]) for r in rs],
                  np.int64)
    fl = np.array([r[3] for r in rs], np.uint8)
    return key, cost, mk, fl


def test_replica_init_matches_oracle(ctx):
    _say("replica init")
    inst = _replica()
    iid = ctx.instance_upload(inst)
    assert from_csr(ctx.init_solution(iid)) == OI.init_solution(inst)


@pytest.mark.parametrize("case", [2, 3, 4])
@pytest.mark.parametrize("walked", [False, True])
def test_replica_evaluate_parity(ctx, pool, case, walked):
    """evaluate_batch on 4096 oracle-drawn moves, element by element, from
    Alg. 1's start (x with its minimised units) and from a base a few
    iterations of the case's own search further on."""
    flags = CASES[case]
    _say("replica evaluate", case, walked)
    inst = _replica()
    x0 = OI.init_solution(inst)
    emb = not (flags & bl.NO_EMBEDDED_MIN)
    st = S.start(inst, x0, embedded_min=emb)
    if walked:
        st = S.search(inst, x0, 8, 64, 6, S.eps_threshold(0.5), gate=_gate(flags),
                      fixed_field_bp=bool(flags & bl.FIXED_FIELD_BP), embedded_min=emb, map_fn=pool)
    base = st.x_old
    iid = ctx.instance_upload(inst, flags=flags)
    ctx.solution_upload(iid, bl.SLOT_BASE, to_csr(base))
    n, seed, it = 4096, 42, 3
    d = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.generate(iid, seed, it, 0, 0, n, d)
    words = np.array([MV.encode(MV.draw_move(inst, base, seed, it, i, 0, bool(flags & bl.FIXED_FIELD_BP)))
                      for i in range(n)], dtype=np.uint64)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy().view(np.uint64), words)
    t_star = (1 << 40) if flags & bl.GATE_OFF else int(st.t_best)
    d_key = torch.empty(n, dtype=torch.int64, device="cuda")
    d_cost = torch.empty(n, dtype=torch.float32, device="cuda")
    d_mk = torch.empty(n, dtype=torch.int32, device="cuda")
    d_fl = torch.empty(n, dtype=torch.uint8, device="cuda")
    ctx.evaluate_batch(iid, d, n, t_star, d_key, d_cost, d_mk, d_fl)
    torch.cuda.synchronize()
    gpu = (d_key.cpu().numpy().view(np.uint64), d_cost.cpu().numpy(), d_mk.cpu().numpy(), d_fl.cpu().numpy())
    orc = _pool_batch(pool, inst, base, seed, it, n, flags, t_star)
    compare(gpu, orc, "replica case %d" % case)
    assert (orc[0] != bl.INF_KEY).any()


def test_replica_batched_trajectory(ctx, pool):
    """Cases 2, 3 and 4 of one replica instance as members of one batched
    search (one persistent launch per iteration): every member's trajectory
    equals the oracle's search of that case, with the member's position as
    the Philox instance word."""
    _say("replica batch")
    inst = _replica()
    x0 = OI.init_solution(inst)
    ids = []
    for case in (2, 3, 4):
        iid = ctx.instance_upload(inst, flags=CASES[case])
        ctx.solution_upload(iid, bl.SLOT_BASE, to_csr(x0))
        ids.append(iid)
    n, iters, thr, seed = 512, 4, S.eps_threshold(0.5), 6
    b = ctx.batch_create(ids, n)
    ctx.batch_start(b, iters)
    for _ in range(iters):
        ctx.batch_step(b, seed, thr)
    torch.cuda.synchronize()
    for k, (case, iid) in enumerate(zip((2, 3, 4), ids)):
        flags = CASES[case]
        st = S.search(inst, x0, seed, n, iters, thr, gate=_gate(flags), inst_idx=k,
                      fixed_field_bp=bool(flags & bl.FIXED_FIELD_BP),
                      embedded_min=not (flags & bl.NO_EMBEDDED_MIN), map_fn=pool)
        rows = [(r["it"], r["best_key"], r["cost_m"], r["indicator"], bool(r["use_best"]))
                for r in ctx.search_trace(iid)]
        assert rows == [(r.it, r.best_key, r.cost_m, r.indicator, r.use_best) for r in st.trace], case
        assert from_csr(ctx.solution_download(iid, bl.SLOT_BEST)) == st.x_best
        assert from_csr(ctx.solution_download(iid, bl.SLOT_OLD)) == st.x_old
