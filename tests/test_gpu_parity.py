"""Parity of the HIP library (through the C interface) with the CPU oracle.

Inputs of the oracle never come from the GPU: move records are drawn by the
oracle itself and uploaded; the GPU's own generator is compared with them
separately.  Decisions (moves, keys, flags, makespans, units, trajectories)
must be bit-exact; FP32 costs within 1e-5 relative of the float64 oracle.
"""
import sys

import numpy as np
import pytest

from oracle import init as OI
from oracle import model as M
from oracle import moves as MV
from oracle import search as S
from paper_1909_10286_amd import bl, inputs

from .gpu_common import caps_of, compare, from_csr, oracle_batch, oracle_words, to_csr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def _gpu_eval(ctx, iid, words, t_star):
    n = len(words)
    d_mv = _dev(words.astype(np.uint64))
    d_key = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
    d_cost = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
    d_mk = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    d_fl = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
    ctx.evaluate_batch(iid, d_mv, n, t_star, d_key, d_cost, d_mk, d_fl)
    torch.cuda.synchronize()
    return (d_key.cpu().numpy().view(np.uint64)[:n], d_cost.cpu().numpy()[:n],
            d_mk.cpu().numpy()[:n], d_fl.cpu().numpy()[:n])


# Instances past the one-candidate-per-lane limit of 12 tours: the segment
# version at its widths of 32 and 64 lanes (17-32 and 33-64 tours).
_WIDE = {"tours20": (200, 30, 20, 40, 80), "tours40": (240, 48, 40, 64, 120)}


def _instance(name, seed=0):
    if name.startswith("batch"):
        return inputs.make_batch_instance(int(name[5:]), accept=OI.init_feasible)
    if name in _WIDE:
        nf, nb, nt, nh, ns = _WIDE[name]
        return inputs.make_custom_instance(name, seed, 100_000, nf, nb, nt, nh, ns, accept=OI.init_feasible)
    return inputs.make_instance(name, seed, accept=OI.init_feasible)


def _setup(ctx, inst, base, flags=0, cap_hu=0, cap_su=0):
    iid = ctx.instance_upload(inst, flags=flags, cap_hu=cap_hu, cap_su=cap_su)
    ctx.solution_upload(iid, bl.SLOT_BASE, to_csr(base))
    return iid


# ------------------------------------------------------------------ init ---

@pytest.mark.parametrize("name", ["tiny12", "mid100", "clust500", "batch7", "batch100"])
def test_init_solution_matches_oracle(ctx, name):
    _say("init", name)
    inst = _instance(name)
    iid = ctx.instance_upload(inst)
    got = from_csr(ctx.init_solution(iid))
    want = OI.init_solution(inst)
    assert got == want


# -------------------------------------------------------------- generate ---

@pytest.mark.parametrize("name,n,first,fixed", [
    ("tiny12", 4096, 0, False), ("mid100", 3001, 17, False), ("clust500", 1500, 5, False),
    ("mid100", 2000, 0, True), ("batch3", 777, 1000, False)])
def test_generate_bitexact(ctx, name, n, first, fixed):
    _say("generate", name, n, first, fixed)
    inst = _instance(name)
    base = OI.init_solution(inst)
    iid = _setup(ctx, inst, base, flags=bl.FIXED_FIELD_BP if fixed else 0)
    d = torch.empty(n, dtype=torch.int64, device="cuda")
    seed, it = 0x1234_5678_9ABC_DEF0, 7
    ctx.generate(iid, seed, it, 3, first, n, d)
    torch.cuda.synchronize()
    got = d.cpu().numpy().view(np.uint64)
    want = oracle_words(inst, base, seed, it, n, first, 3, fixed)
    assert np.array_equal(got, want)


# ------------------------------------------------------------- evaluate ----

def _walk_base(inst, x, seed, steps):
    """A base reached by a few oracle moves (feasible or not), to leave the
    initial solution's structure."""
    for i in range(steps):
        mv = MV.draw_move(inst, x, seed, 999, i)
        y = MV.apply_move(x, mv)
        if M.is_feasible(inst, y):
            x = y
    ev = M.evaluate_solution(inst, x)
    return S.with_units(x, ev)


def _inactive_tour_base(inst):
    """All BPs of tour 0 moved to tour 1: tour 0 inactive but keeps units."""
    x = OI.init_solution(inst)
    x = x.copy()
    x.tours[1] = x.tours[0] + x.tours[1]
    x.tours[0] = []
    return x


def _empty_bp_base(inst):
    """BP 0's fields appended to the next BP of the same tour (or of the
    next tour): BP 0 keeps its place in its tour with no fields."""
    x = OI.init_solution(inst).copy()
    dst = next(b for t in x.tours for b in t if b != 0)
    x.fields[dst] = x.fields[dst] + x.fields[0]
    x.fields[0] = []
    return x


def _no_hu_base(inst):
    """Tour 0 active without HUs (its HUs moved to tour 1)."""
    x = OI.init_solution(inst)
    x = x.copy()
    x.hu_tour = [1 if g == 0 else g for g in x.hu_tour]
    return x


CASES = [
    # name, n, base kind, flags, caps, t_star kind
    ("tiny12", 4096, "init", 0, (0, 0), "base"),
    ("tiny12", 1000, "inactive", 0, (0, 0), "base"),
    ("tiny12", 1000, "init", bl.GATE_STRICT, (0, 0), "base"),
    ("tiny12", 700, "init", bl.GATE_OFF | bl.NO_EMBEDDED_MIN | bl.FIXED_FIELD_BP, (0, 0), "base"),
    ("mid100", 2085, "init", 0, (0, 0), "base"),
    ("mid100", 600, "walk", 0, (0, 0), "big"),
    ("mid100", 600, "nohu", 0, (0, 0), "big"),
    ("mid100", 600, "init", 0, (1, 1), "big"),
    ("mid100", 500, "inactive", 0, (0, 0), "big"),
    ("clust500", 257, "init", 0, (0, 0), "base"),
    ("clust500", 129, "walk", 0, (2, 3), "big"),
    ("batch0", 500, "init", 0, (0, 0), "base"),
    ("batch11", 500, "walk", 0, (0, 0), "base"),
    ("batch42", 500, "init", 0, (0, 0), "big"),
    # The full walk of every route (BL_FULL_WALK) against the same oracle.
    ("tiny12", 1000, "inactive", bl.FULL_WALK, (0, 0), "base"),
    ("mid100", 2085, "init", bl.FULL_WALK, (0, 0), "base"),
    ("clust500", 129, "walk", bl.FULL_WALK, (2, 3), "big"),
    # A base with an emptied BP (infeasible): moves that refill it are the only
    # feasible ones.
    ("tiny12", 2000, "emptybp", 0, (0, 0), "big"),
    ("mid100", 2000, "emptybp", 0, (0, 0), "big"),
    ("mid100", 2000, "emptybp", bl.FULL_WALK, (0, 0), "big"),
    # 64-bit rebalancing keys where 32-bit ones would do.
    ("tiny12", 1000, "init", bl.WIDE_KEYS, (0, 0), "base"),
    ("mid100", 2085, "walk", bl.WIDE_KEYS, (0, 0), "big"),
    ("clust500", 129, "init", bl.WIDE_KEYS | bl.FULL_WALK, (2, 3), "base"),
    ("batch31", 500, "init", bl.WIDE_KEYS, (1, 1), "big"),
    # The segment version (one tour per lane) where one lane per candidate is the default.
    ("mid100", 2085, "walk", bl.SEGMENT_EVAL, (0, 0), "big"),
    ("tiny12", 1000, "inactive", bl.SEGMENT_EVAL, (0, 0), "base"),
    # More than 12 tours: segments of 32 and 64 lanes, 64-bit keys.
    ("tours20", 600, "walk", 0, (0, 0), "big"),
    ("tours20", 600, "init", 0, (0, 0), "base"),
    ("tours40", 400, "walk", 0, (0, 0), "big"),
    ("tours40", 400, "init", bl.FULL_WALK, (2, 3), "base"),
]


@pytest.mark.parametrize("name,n,kind,flags,caps,tk", CASES)
def test_evaluate_batch_parity(ctx, name, n, kind, flags, caps, tk):
    _say("evaluate", name, n, kind, flags, caps, tk)
    inst = _instance(name)
    base = {"init": lambda: OI.init_solution(inst), "walk": lambda: _walk_base(inst, OI.init_solution(inst), 5, 40),
            "inactive": lambda: _inactive_tour_base(inst), "nohu": lambda: _no_hu_base(inst),
            "emptybp": lambda: _empty_bp_base(inst)}[kind]()
    iid = _setup(ctx, inst, base, flags, *caps)
    fixed = bool(flags & bl.FIXED_FIELD_BP)
    words = oracle_words(inst, base, 42, 3, n, fixed=fixed)
    ev = M.evaluate_solution(inst, base, caps_of(inst, *caps), not (flags & bl.NO_EMBEDDED_MIN))
    t_star = (1 << 40) if tk == "big" or not ev.feasible or ev.makespan_s == M.INF else int(ev.makespan_s)
    gpu = _gpu_eval(ctx, iid, words, t_star)
    orc = oracle_batch(inst, base, words, t_star, flags, caps_of(inst, *caps))
    compare(gpu, orc, name)
    if kind == "init" and not flags and not name.startswith("batch"):
        # The sample exercises both discarded and ranked candidates.
        assert (orc[3] & bl.CAND_INFEASIBLE).any() and (orc[0] != bl.INF_KEY).any()


@pytest.mark.parametrize("name,kind", [("mid100", "walk"), ("clust500", "walk"), ("batch77", "init"),
                                       ("mid100", "emptybp"), ("tiny12", "inactive")])
def test_delta_equals_full_walk(ctx, name, kind):
    """The default evaluation (base aggregates plus the legs a move changes;
    one candidate per lane up to 12 tours, else 32-bit rebalancing keys on a
    segment of lanes), the segment version, the full walk and the 64-bit keys
    agree bit for bit on 2^16 generated moves."""
    _say("delta vs walk", name, kind)
    inst = _instance(name)
    base = {"init": lambda: OI.init_solution(inst), "walk": lambda: _walk_base(inst, OI.init_solution(inst), 5, 40),
            "inactive": lambda: _inactive_tour_base(inst), "emptybp": lambda: _empty_bp_base(inst)}[kind]()
    a = _setup(ctx, inst, base)
    b = _setup(ctx, inst, base, bl.FULL_WALK)
    w = _setup(ctx, inst, base, bl.WIDE_KEYS)
    g = _setup(ctx, inst, base, bl.SEGMENT_EVAL)
    n = 1 << 16
    d_mv = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.generate(a, 77, 5, 0, 0, n, d_mv)
    words = d_mv.cpu().numpy().view(np.uint64)
    for t_star in (1 << 40, int(M.evaluate_solution(inst, base).makespan_s) if kind != "emptybp" else 0):
        ga = _gpu_eval(ctx, a, words, t_star)
        for other in (b, w, g):
            go = _gpu_eval(ctx, other, words, t_star)
            for x, y in zip(ga, go):
                assert np.array_equal(x, y)
    assert (ga[3] & bl.CAND_INFEASIBLE).any()


@pytest.mark.parametrize("name", ["mid100", "clust500"])
def test_deferred_list_overflow(ctx, name):
    """A batch of 2^21 copies of a move whose SU rebalancing runs several
    rounds: the evaluation's second pass takes the first 2^20 deferred
    candidates, the rest finish in the first pass, and every copy gets the
    oracle's result (with its own index in the key)."""
    _say("deferred overflow", name)
    inst = _instance(name)
    base = _walk_base(inst, OI.init_solution(inst), 5, 40)
    iid = _setup(ctx, inst, base)
    words = oracle_words(inst, base, 42, 3, 600)
    best_w, best_r = None, 0
    for i, w in enumerate(words):
        r = S.evaluate_move(inst, base, MV.decode(int(w)), i, M.GATE_LE, 1 << 40)
        if r.evaluation is not None and r.evaluation.feasible and r.evaluation.su_rounds > best_r:
            best_w, best_r = w, r.evaluation.su_rounds
    assert best_r >= 4, "no move with a long SU tail in the sample"
    n = 1 << 21
    gk, gc, gm, gf = _gpu_eval(ctx, iid, np.full(n, best_w, np.uint64), 1 << 40)
    ok, oc, om, of = oracle_batch(inst, base, np.array([best_w], np.uint64), 1 << 40)
    assert np.array_equal(gk >> np.uint64(24), np.full(n, ok[0] >> np.uint64(24), np.uint64))
    assert np.array_equal(gk & np.uint64((1 << 24) - 1), np.arange(n, dtype=np.uint64))
    assert (gm == om[0]).all() and (gf == of[0]).all()
    assert np.allclose(gc, oc[0], rtol=1e-5)


@pytest.mark.parametrize("name,caps", [("mid100", (0, 0)), ("clust500", (0, 0)),
                                       ("mid100", (0, 3)), ("clust500", (2, 3))])
def test_two_pass_equals_segment(ctx, name, caps):
    """At 2^20 candidates the lane evaluation runs its two passes (long SU
    tails deferred to the second); its outputs equal the segment version's
    (one pass, one tour per lane) element for element, also where the SU cap
    (3 rounds) lies just past the deferral limit (1 round), so that deferred
    candidates hit it in the second pass."""
    _say("two passes vs segment", name, caps)
    inst = _instance(name)
    base = _walk_base(inst, OI.init_solution(inst), 5, 40)
    a = _setup(ctx, inst, base, 0, *caps)
    g = _setup(ctx, inst, base, bl.SEGMENT_EVAL, *caps)
    n = 1 << 20
    d_mv = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.generate(a, 91, 2, 0, 0, n, d_mv)
    words = d_mv.cpu().numpy().view(np.uint64)
    ga = _gpu_eval(ctx, a, words, 1 << 40)
    gg = _gpu_eval(ctx, g, words, 1 << 40)
    for x, y in zip(ga, gg):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("name,flags,lane,table", [("mid100", 0, 1, 1), ("clust500", 0, 1, 1),
                                                   ("clust500", bl.SEGMENT_EVAL, 0, 0), ("tours40", 0, 0, 0)])
def test_instance_info_names_the_kernels(ctx, name, flags, lane, table):
    """bl_instance_info_get reports one candidate per lane up to 12 tours
    (with the LDS-table second pass where it keeps the workgroups per CU),
    the segment version beyond or on request, and the image size."""
    _say("instance info", name, flags)
    inst = _instance(name)
    info = ctx.instance_info(ctx.instance_upload(inst, flags=flags))
    assert (info["lane_eval"], info["tail_table"]) == (lane, table)
    assert info["wg_per_cu"] >= 1 and info["image_bytes"] > 22 * inst.n_fields


@pytest.mark.parametrize("name,iters", [("mid100", 6), ("clust500", 3)])
def test_winner_record_equals_reevaluation(ctx, name, iters, monkeypatch):
    """Searches at full candidate counts (two lane passes): where the second
    pass forms the winner's units for the commit (default upload), the
    trajectory, trace and solutions equal those of the same search whose
    commit evaluates the winner again (BL_LANE_TAIL=0 at upload: no record)."""
    _say("winner record vs re-evaluation", name)
    inst = _instance(name)
    x0 = to_csr(OI.init_solution(inst))
    n = inputs.WORKLOADS[name]["n_cand"]
    out = []
    for tail in (None, "0"):
        if tail is None:
            monkeypatch.delenv("BL_LANE_TAIL", raising=False)
        else:
            monkeypatch.setenv("BL_LANE_TAIL", tail)
        iid = ctx.instance_upload(inst)
        monkeypatch.delenv("BL_LANE_TAIL", raising=False)
        assert ctx.instance_info(iid)["tail_table"] == (1 if tail is None else 0)
        ctx.solution_upload(iid, bl.SLOT_BASE, x0)
        ctx.search_start(iid, iters)
        for _ in range(iters):
            ctx.search_step(iid, 17, 1 << 31, n)
        out.append((ctx.search_state(iid), ctx.search_trace(iid),
                    from_csr(ctx.solution_download(iid, bl.SLOT_OLD)),
                    from_csr(ctx.solution_download(iid, bl.SLOT_BEST))))
    assert out[0][0] == out[1][0]
    assert out[0][1] == out[1][1]
    assert out[0][2] == out[1][2] and out[0][3] == out[1][3]


@pytest.mark.parametrize("name,caps", [("mid100", (0, 0)), ("clust500", (0, 0)), ("clust500", (2, 3))])
def test_tail_table_equals_registers(ctx, name, caps, monkeypatch):
    """The second lane pass with every thread's SU masks in an LDS table
    gives the outputs of the same pass with the masks in registers
    (BL_LANE_TAIL=0 at upload), element for element, at 2^20 candidates."""
    _say("tail table vs registers", name, caps)
    inst = _instance(name)
    base = _walk_base(inst, OI.init_solution(inst), 5, 40)
    a = _setup(ctx, inst, base, 0, *caps)
    monkeypatch.setenv("BL_LANE_TAIL", "0")
    r = _setup(ctx, inst, base, 0, *caps)
    monkeypatch.delenv("BL_LANE_TAIL")
    ia, ir = ctx.instance_info(a), ctx.instance_info(r)
    assert ia["lane_eval"] == 1 and ia["tail_table"] == 1 and ir["tail_table"] == 0
    assert ia["wg_per_cu"] == ir["wg_per_cu"]
    n = 1 << 20
    d_mv = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.generate(a, 93, 2, 0, 0, n, d_mv)
    words = d_mv.cpu().numpy().view(np.uint64)
    ga = _gpu_eval(ctx, a, words, 1 << 40)
    gr = _gpu_eval(ctx, r, words, 1 << 40)
    for x, y in zip(ga, gr):
        assert np.array_equal(x, y)
    assert (ga[0] != bl.INF_KEY).any()
    if caps[1]:
        assert (ga[3] & bl.CAND_CAP_SU).any()


def test_evaluate_invalid_and_ragged(ctx):
    _say("evaluate invalid")
    inst = _instance("tiny12")
    base = OI.init_solution(inst)
    iid = _setup(ctx, inst, base)
    good = oracle_words(inst, base, 1, 0, 5)
    bad = np.array([
        MV.encode(MV.Move(0, inst.n_fields, 0, 0)),        # field id out of range
        MV.encode(MV.Move(0, 0, inst.n_bps, 0)),           # BP out of range
        MV.encode(MV.Move(1, inst.n_bps, 0, 0)),           # BP id out of range
        MV.encode(MV.Move(1, 0, inst.n_tours, 0)),         # tour out of range
        MV.encode(MV.Move(0, 0, 0, 500)),                  # slot beyond the list
    ], dtype=np.uint64)
    words = np.concatenate([good, bad])
    gpu = _gpu_eval(ctx, iid, words, 1 << 40)
    orc = oracle_batch(inst, base, words, 1 << 40)
    compare(gpu, orc, "invalid")
    assert (gpu[3][5:] == bl.CAND_INVALID).all()
    # n = 0 is a no-op; n = 1 works.
    ctx.evaluate_batch(iid, 0, 0, 0, 0)
    compare(_gpu_eval(ctx, iid, words[:1], 1 << 40), oracle_batch(inst, base, words[:1], 1 << 40))


def test_select_best(ctx):
    _say("select")
    rng = np.random.default_rng(0)
    for n in (1, 63, 64, 1000, 1 << 20):
        keys = rng.integers(0, 2**63, n, dtype=np.uint64) | np.uint64(1 << 63)
        keys[rng.integers(0, n, max(1, n // 3))] = np.uint64(bl.INF_KEY)
        d_k = _dev(keys)
        d_b = torch.empty(1, dtype=torch.int64, device="cuda")
        ctx.select_best(d_k, n, d_b)
        torch.cuda.synchronize()
        assert d_b.cpu().numpy().view(np.uint64)[0] == keys.min()
    d_b = torch.empty(1, dtype=torch.int64, device="cuda")
    ctx.select_best(0, 0, d_b)
    torch.cuda.synchronize()
    assert d_b.cpu().numpy().view(np.uint64)[0] == np.uint64(bl.INF_KEY)


# --------------------------------------------------------------- search ----

def _gpu_search(ctx, inst, x0, seed, n, iters, eps_thr, flags=0):
    iid = _setup(ctx, inst, x0, flags)
    ctx.search_start(iid, iters)
    for _ in range(iters):
        ctx.search_step(iid, seed, eps_thr, n)
    torch.cuda.synchronize()
    return iid, ctx.search_trace(iid), ctx.search_state(iid)


def _compare_trace(gtr, otr):
    assert len(gtr) == len(otr)
    for g, o in zip(gtr, otr):
        mk = bl.INF_MAKESPAN if o.makespan_s == M.INF else o.makespan_s
        assert (g["it"], g["best_key"], g["cost_m"], g["makespan_s"], g["indicator"], bool(g["use_best"])) == \
            (o.it, o.best_key, o.cost_m, mk, o.indicator, o.use_best), (g, o)


def test_search_trajectory_tiny12(ctx, pool):
    """Full tiny workload: 4096 candidates x 100 iterations, seed 0, eps 0.5."""
    _say("search tiny12 full")
    inst = _instance("tiny12")
    x0 = OI.init_solution(inst)
    thr = S.eps_threshold(0.5)
    iid, gtr, gst = _gpu_search(ctx, inst, x0, 0, 4096, 100, thr)
    st = S.search(inst, x0, 0, 4096, 100, thr, map_fn=pool)
    _compare_trace(gtr, st.trace)
    assert gst["cost_best_m"] == st.cost_best
    assert from_csr(ctx.solution_download(iid, bl.SLOT_BEST)) == st.x_best
    assert from_csr(ctx.solution_download(iid, bl.SLOT_OLD)) == st.x_old


@pytest.mark.parametrize("name,n,iters,eps,flags", [
    ("mid100", 2048, 6, 0.5, 0), ("mid100", 1500, 4, 0.0, bl.FIXED_FIELD_BP),
    ("batch5", 1024, 5, 1.0, 0), ("tiny12", 512, 20, 0.25, bl.GATE_STRICT),
    ("tiny12", 256, 10, 0.5, bl.GATE_OFF | bl.NO_EMBEDDED_MIN | bl.FIXED_FIELD_BP),
    ("mid100", 1024, 4, 0.5, bl.FULL_WALK), ("batch9", 512, 5, 0.5, bl.FULL_WALK),
    ("mid100", 1024, 4, 0.5, bl.WIDE_KEYS), ("tiny12", 512, 12, 0.5, bl.WIDE_KEYS | bl.GATE_STRICT)])
def test_search_trajectory_reduced(ctx, pool, name, n, iters, eps, flags):
    _say("search", name, n, iters, eps, flags)
    inst = _instance(name)
    x0 = OI.init_solution(inst)
    thr = S.eps_threshold(eps)
    gate = M.GATE_OFF if flags & bl.GATE_OFF else (M.GATE_STRICT if flags & bl.GATE_STRICT else M.GATE_LE)
    iid, gtr, gst = _gpu_search(ctx, inst, x0, 9, n, iters, thr, flags)
    st = S.search(inst, x0, 9, n, iters, thr, gate=gate, fixed_field_bp=bool(flags & bl.FIXED_FIELD_BP),
                  embedded_min=not (flags & bl.NO_EMBEDDED_MIN), map_fn=pool)
    _compare_trace(gtr, st.trace)
    assert from_csr(ctx.solution_download(iid, bl.SLOT_BEST)) == st.x_best


@pytest.mark.parametrize("name,iters", [("tiny12", 300), ("mid100", 120)])
def test_single_worker_search(ctx, name, iters):
    """The GPU version of Algorithm 1 with one worker (the oracle's
    `search_single_worker`, one candidate per iteration) equals the
    device-resident iteration with n = 1."""
    _say("single worker", name, iters)
    inst = _instance(name)
    x0 = OI.init_solution(inst)
    thr = S.eps_threshold(0.5)
    iid, gtr, gst = _gpu_search(ctx, inst, x0, 4, 1, iters, thr)
    st = S.search_single_worker(inst, x0, 4, iters, thr)
    _compare_trace(gtr, st.trace)
    assert from_csr(ctx.solution_download(iid, bl.SLOT_BEST)) == st.x_best
    assert from_csr(ctx.solution_download(iid, bl.SLOT_OLD)) == st.x_old


def test_search_deterministic(ctx):
    """Unique (cost, index) keys make the argmin order-free: two runs agree
    bit for bit."""
    _say("search determinism")
    inst = _instance("mid100")
    x0 = OI.init_solution(inst)
    a = _gpu_search(ctx, inst, x0, 3, 1 << 18, 10, S.eps_threshold(0.5))[1]
    b = _gpu_search(ctx, inst, x0, 3, 1 << 18, 10, S.eps_threshold(0.5))[1]
    assert a == b


@pytest.mark.parametrize("name,n,samples", [("mid100", 1 << 20, 400), ("clust500", 1 << 22, 120)])
def test_full_size_iteration_sampled(ctx, pool, name, n, samples):
    """At the full candidate count: one device-resident iteration; the winner
    re-evaluated by the oracle reproduces the iteration's key, and no sampled
    candidate (oracle) beats it.  Sampled candidates are also evaluated by
    evaluate_batch on GPU-generated moves and compared one by one."""
    _say("full size", name, n)
    inst = _instance(name)
    x0 = OI.init_solution(inst)
    thr = S.eps_threshold(0.5)
    iid, gtr, gst = _gpu_search(ctx, inst, x0, 0, n, 1, thr)
    st0 = S.start(inst, x0)
    use_best = MV.exploit_draw(0, 0, 0, thr)
    base = st0.x_best if use_best else st0.x_old
    k = gtr[0]["best_key"]
    assert k != bl.INF_KEY
    i_star = int(k) & 0xFFFFFF
    job = (inst, base, 0, 0, 0, False, M.GATE_LE, st0.t_best, None, True)
    assert S.candidate(job, i_star)[0] == k
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(n, samples, replace=False))
    okeys = [S.candidate(job, int(i))[0] for i in idx]
    assert min(okeys) >= k
    # GPU generator + evaluate_batch at full size, sampled comparison.
    iid2 = _setup(ctx, inst, base)
    d_mv = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.generate(iid2, 0, 0, 0, 0, n, d_mv)
    d_key = torch.empty(n, dtype=torch.int64, device="cuda")
    d_cost = torch.empty(n, dtype=torch.float32, device="cuda")
    d_mk = torch.empty(n, dtype=torch.int32, device="cuda")
    d_fl = torch.empty(n, dtype=torch.uint8, device="cuda")
    ctx.evaluate_batch(iid2, d_mv, n, st0.t_best, d_key, d_cost, d_mk, d_fl)
    d_best = torch.empty(1, dtype=torch.int64, device="cuda")
    ctx.select_best(d_key, n, d_best)
    torch.cuda.synchronize()
    assert int(d_best.cpu().numpy().view(np.uint64)[0]) == k
    words = np.array([MV.encode(MV.draw_move(inst, base, 0, 0, int(i))) for i in idx], np.uint64)
    assert np.array_equal(d_mv.cpu().numpy().view(np.uint64)[idx], words)
    orc = oracle_batch(inst, base, words, st0.t_best)
    orc = (np.array([(w if w == bl.INF_KEY else ((int(w) >> 24) << 24) | int(i)) for w, i in zip(orc[0], idx)],
                    dtype=np.uint64),) + orc[1:]
    gpu = (d_key.cpu().numpy().view(np.uint64)[idx], d_cost.cpu().numpy()[idx],
           d_mk.cpu().numpy()[idx], d_fl.cpu().numpy()[idx])
    compare(gpu, orc, name + " sampled")
