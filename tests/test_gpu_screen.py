"""The learned screen's incremental inference and the screened iteration on
the GPU.

* Scores: the screen recomputes only the rows, BP means and tours a proposal
  changes; its predicted path must equal the library's full forward pass
  (bl_sur_predict, itself checked against the float64 reference) on the same
  proposals up to float32 summation order, and its discards must be exactly
  the proposals that break eq. (2) (an integer decision) or whose predicted
  makespan is above the gate.
* Shortlist: exactly the n_shortlist smallest scores, lowest index first
  among equal scores (index work: bit-exact).
* Screened iteration: given the shortlist, the iteration is the oracle's
  iteration with every other proposal left out (keys, trace, solutions
  bit-exact); with the fallback forced it is the plain iteration.
"""
import math
import sys

import numpy as np
import pytest

from oracle import model as M
from oracle import moves as MV
from oracle import search as S
from oracle import surrogate as SG

from paper_1909_10286_amd import bl, inputs

from .gpu_common import from_csr, to_csr
from .sur_common import setup

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _screen(ctx, sur, seed, eps, n, k, margin):
    d_short = torch.empty(k, dtype=torch.int32, device="cuda")
    d_score = torch.empty(n, dtype=torch.float32, device="cuda")
    ctx.sur_screen(sur, seed, eps, n, k, d_short, d_score, mk_margin=margin)
    torch.cuda.synchronize()
    return d_short.cpu().numpy().view(np.uint32).astype(np.int64), d_score.cpu().numpy()


def _predict(ctx, iid, sur, seed, n):
    d_mv = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.generate(iid, seed, 0, 0, 0, n, d_mv)
    d_out = torch.empty(2 * n, dtype=torch.float32, device="cuda")
    ctx.sur_predict(sur, d_mv, n, d_out)
    torch.cuda.synchronize()
    return d_mv.cpu().numpy().view(np.uint64), d_out.cpu().numpy().reshape(-1, 2).astype(np.float64)


def _expected_shortlist(score, k):
    return np.sort(np.argsort(score, kind="stable")[:k])


@pytest.mark.parametrize("name,n,k", [("tiny12", 5000, 128), ("mid100", 8192, 512),
                                      ("clust500", 4096, 300)])
def test_screen_scores_match_full_forward(ctx, name, n, k):
    _say("screen scores", name, n, k)
    inst, st, iid, sur, p, sc = setup(ctx, name)
    ctx.search_start(iid, 4)
    seed, eps = 21, 1 << 32          # eps threshold 2^32: the base is x*
    short, score = _screen(ctx, sur, seed, eps, n, k, margin=1e9)
    words, pred = _predict(ctx, iid, sur, seed, n)
    base = st.x_best
    feas = np.array([M.is_feasible(inst, MV.apply_move(base, MV.decode(int(w)))) for w in words])
    # With an unreachable makespan gate, exactly the eq. (2) breakers are discarded.
    assert np.array_equal(np.isfinite(score), feas), np.nonzero(np.isfinite(score) != feas)[0][:10]
    tol = 1e-4 * np.abs(pred[:, 0]).max() + 1e-6
    err = np.abs(score[feas] - pred[feas, 0])
    assert err.max() <= tol, (err.max(), tol)
    assert np.array_equal(short, _expected_shortlist(score, k))
    # And against the float64 reference directly, on a sample (bf16 tolerance
    # of the full-forward test).
    idx = np.nonzero(feas)[0][:48]
    ref = np.array([SG.predict(p, inst, MV.apply_move(base, MV.decode(int(words[i]))), sc)[0] for i in idx])
    assert (np.abs(score[idx] - ref) <= 2e-2 * np.abs(ref).max() + 1e-3).all()

    # The makespan gate: predicted makespan above t_best / t0 + margin drops out.
    margin = float(np.median(pred[feas, 1])) - 1.0   # t0 = t_best: the gate sits at the median
    short2, score2 = _screen(ctx, sur, seed, eps, n, k, margin=margin)
    gate = 1.0 + margin
    mtol = 1e-4 * np.abs(pred[:, 1]).max() + 1e-6
    clear_in = feas & (pred[:, 1] < gate - mtol)
    clear_out = ~feas | (pred[:, 1] > gate + mtol)
    assert np.isfinite(score2[clear_in]).all()
    assert not np.isfinite(score2[clear_out]).any()
    assert np.array_equal(short2, _expected_shortlist(score2, k))


def test_screen_full_size_sampled(ctx):
    """The screen at its full size (2^24 clust500 proposals, the bench's
    launch): sampled scores, spread over the index range and including the
    last proposal, equal the full forward pass of the same proposals; the
    discards among them are exactly the eq. (2) breakers (gate off); and the
    shortlist of 2^18 is the 2^18 smallest scores, lowest index first (its
    boundary checked against the exported scores)."""
    n, k = 1 << 24, 1 << 18
    _say("screen full size", n, k)
    inst, st, iid, sur, p, sc = setup(ctx, "clust500")
    ctx.search_start(iid, 4)
    seed, eps = 3, 1 << 32
    short, score = _screen(ctx, sur, seed, eps, n, k, margin=1e9)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([rng.choice(n, 1500, replace=False), [0, 63, 64, n - 64, n - 1]]))
    d_all = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.generate(iid, seed, 0, 0, 0, n, d_all)
    d_mv = d_all[torch.from_numpy(idx).cuda()].contiguous()
    del d_all
    d_out = torch.empty(2 * len(idx), dtype=torch.float32, device="cuda")
    ctx.sur_predict(sur, d_mv, len(idx), d_out)
    torch.cuda.synchronize()
    pred = d_out.cpu().numpy().reshape(-1, 2).astype(np.float64)
    words = d_mv.cpu().numpy().view(np.uint64)
    base = st.x_best
    feas = np.array([M.is_feasible(inst, MV.apply_move(base, MV.decode(int(w)))) for w in words])
    got = score[idx]
    assert np.array_equal(np.isfinite(got), feas)
    tol = 1e-4 * np.abs(pred[:, 0]).max() + 1e-6
    assert np.abs(got[feas] - pred[feas, 0]).max() <= tol
    # The shortlist: ascending, every member scores at most the k-th score, every
    # non-member at least it, and among equal scores at the boundary the lowest indices.
    assert len(short) == k and np.all(np.diff(short) > 0)
    kth = np.partition(score, k - 1)[k - 1]
    member = np.zeros(n, bool)
    member[short] = True
    assert (score[member] <= kth).all() and (score[~member] >= kth).all()
    ties = np.nonzero(score == kth)[0]
    n_below = int((score < kth).sum())
    assert np.array_equal(np.nonzero(member & (score == kth))[0], ties[:k - n_below])


def _oracle_screened_step(inst, st, seed, n, eps, short, n_control):
    """The oracle's iteration over the shortlist and the control sample, or
    over every proposal when the exact results reject the screen (no gated
    survivor in the shortlist, or the control sample beats it with a cost
    below x*'s)."""
    seen = {}

    def key_of(job, i):
        if i not in seen:
            seen[i] = S.candidate(job, i)[0]
        return seen[i]

    decision = {}

    def keys(job, nn):
        smin = min(key_of(job, int(i)) for i in short)
        cmin = min((key_of(job, i) for i in range(n_control)), default=M.INF_KEY)
        fallback = smin == M.INF_KEY or (cmin < smin and (cmin >> 24) < st.cost_best)
        decision["fallback"] = fallback
        subset = range(nn) if fallback else set(int(i) for i in short) | set(range(n_control))
        out = [M.INF_KEY] * nn
        for i in subset:
            out[i] = key_of(job, i)
        return out
    return S.step(inst, st, seed, n, eps, map_fn=keys), decision["fallback"]


def _compare(ctx, iid, st, row):
    g = ctx.search_trace(iid)[-1]
    o = st.trace[-1]
    mk = bl.INF_MAKESPAN if o.makespan_s == M.INF else o.makespan_s
    assert (g["it"], g["best_key"], g["cost_m"], g["makespan_s"], g["indicator"], bool(g["use_best"])) == \
        (o.it, o.best_key, o.cost_m, mk, o.indicator, o.use_best), (row, g, o)
    assert from_csr(ctx.solution_download(iid, bl.SLOT_OLD)) == st.x_old
    assert from_csr(ctx.solution_download(iid, bl.SLOT_BEST)) == st.x_best


@pytest.mark.parametrize("name,n,k,n_control,iters", [("tiny12", 1024, 64, 0, 4), ("tiny12", 1024, 64, 48, 6),
                                                     ("mid100", 1024, 96, 160, 3)])
def test_screened_iteration_matches_oracle_on_shortlist(ctx, name, n, k, n_control, iters):
    """Each iteration: the shortlist the screen picks, then the oracle's
    iteration over it and the control sample, or the plain iteration when
    the exact results reject the screen."""
    _say("screened iteration", name, n, k, n_control, iters)
    inst, st, iid, sur, p, sc = setup(ctx, name)
    ctx.search_start(iid, iters)
    seed, eps = 5, S.eps_threshold(0.5)
    fallbacks = 0
    for it in range(iters):
        short, score = _screen(ctx, sur, seed, eps, n, k, margin=0.5)
        ctx.sur_search_step(sur, seed, eps, n, k, n, mk_margin=0.5, err_threshold=math.inf,
                            n_control=n_control)
        torch.cuda.synchronize()
        st, fb = _oracle_screened_step(inst, st, seed, n, eps, short, n_control)
        fallbacks += fb
        _compare(ctx, iid, st, it)
    stats = ctx.sur_stats(sur)
    _say("  fallbacks", fallbacks, "of", iters)
    assert stats["iterations"] == iters and stats["fallbacks"] == fallbacks


@pytest.mark.parametrize("name,n,iters", [("tiny12", 2048, 8), ("mid100", 4096, 3)])
def test_forced_fallback_is_the_plain_search(ctx, name, n, iters):
    """err_threshold below any error forces the fallback every iteration;
    with n_fallback = n_proposals the argmin covers every proposal, so the
    trajectory is the plain search's, bit for bit."""
    _say("forced fallback", name, n, iters)
    inst, st, iid, sur, p, sc = setup(ctx, name)
    seed, eps = 11, S.eps_threshold(0.5)
    ctx.search_start(iid, iters)
    for _ in range(iters):
        ctx.search_step(iid, seed, eps, n)
    torch.cuda.synchronize()
    plain = ctx.search_trace(iid)
    ctx.solution_upload(iid, bl.SLOT_BASE, to_csr(st.x_best))
    ctx.search_start(iid, iters)
    for _ in range(iters):
        ctx.sur_search_step(sur, seed, eps, n, 32, n, mk_margin=0.0, err_threshold=-1.0)
    torch.cuda.synchronize()
    assert ctx.search_trace(iid) == plain
    stats = ctx.sur_stats(sur)
    assert stats["iterations"] == iters and stats["fallbacks"] == iters


def test_screen_rejects_bad_sizes(ctx):
    inst, st, iid, sur, p, sc = setup(ctx, "tiny12")
    d = torch.empty(64, dtype=torch.int32, device="cuda")
    with pytest.raises(bl.BlError):
        ctx.sur_screen(sur, 0, 0, 64, 64, d)          # search not started
    ctx.search_start(iid, 0)
    with pytest.raises(bl.BlError):
        ctx.sur_screen(sur, 0, 0, 32, 64, d)          # shortlist longer than the proposals
    with pytest.raises(bl.BlError):
        ctx.sur_screen(sur, 0, 0, 0, 1, d)
    with pytest.raises(bl.BlError):
        ctx.sur_search_step(sur, 0, 0, (1 << 24) + 1, 1, 0)
    with pytest.raises(bl.BlError):
        ctx.sur_search_step(sur, 0, 0, 64, 8, 0, n_control=65)  # control beyond the proposals


def test_screen_refuses_instance_beyond_lds(ctx):
    """An instance whose image fits the evaluation kernel's LDS but not the
    screen's (weights, tables and image in one workgroup) is evaluated, and
    the screen calls refuse it with BL_EINVAL instead of launching."""
    from oracle import init as OI
    inst = inputs.make_custom_instance("big2000", 0, 200_000, 2000, 20, 10, 30, 120,
                                       accept=OI.init_feasible)
    iid = ctx.instance_upload(inst)
    x0 = ctx.init_solution(iid)
    ctx.solution_upload(iid, bl.SLOT_BASE, x0)
    ctx.search_start(iid, 2)
    ctx.search_step(iid, 0, 1 << 31, 4096)          # the evaluation runs
    torch.cuda.synchronize()
    st = ctx.search_state(iid)
    w = bl.sur_glorot_weights(inputs.surrogate_init_words(1))
    sur = ctx.sur_create(iid, w, float(st["cost_best_m"]), float(st["t_best_s"]), max_examples=8)
    d = torch.empty(64, dtype=torch.int32, device="cuda")
    with pytest.raises(bl.BlError) as e:
        ctx.sur_screen(sur, 0, 0, 4096, 64, d)
    assert e.value.status == bl.EINVAL
    with pytest.raises(bl.BlError) as e:
        ctx.sur_search_step(sur, 0, 0, 4096, 64, 0)
    assert e.value.status == bl.EINVAL


def test_trained_screen_beats_random_shortlist(ctx):
    """What the trained network gains over the method without it: after a
    short training on exact labels along a plain trajectory, its shortlist of
    1/16 of the proposals holds cheaper candidates on average than a random
    1/16 (the plain method's view of an equal exact budget) and than the
    untrained network's shortlist, and it holds more of the exact top-k.
    The gain is real but far from what a screen of 2^24 proposals down to
    2^18 needs: in the search itself an unscreened sample of 2^12 usually
    beats the shortlist."""
    _say("trained screen gain")
    inst, st, iid, _, p, sc = setup(ctx, "mid100", max_examples=512)
    # The library's usual start: Glorot-uniform weights, zero biases.
    untrained = bl.sur_glorot_weights(inputs.surrogate_init_words(1))
    sur = ctx.sur_create(iid, untrained, float(st.cost_best), float(st.t_best), max_examples=512)
    ctx.search_start(iid, 0)
    per_base, bases = 4096, 24
    d_mv = torch.empty(per_base, dtype=torch.int64, device="cuda")
    d_key = torch.empty(per_base, dtype=torch.int64, device="cuda")
    d_c = torch.empty(per_base, dtype=torch.float32, device="cuda")
    d_m = torch.empty(per_base, dtype=torch.int32, device="cuda")
    for b in range(bases):
        ctx.search_step(iid, 77, S.eps_threshold(0.5), 1 << 14)
        ctx.generate(iid, 1000 + b, 0, 0, 0, per_base, d_mv)
        ctx.evaluate_batch(iid, d_mv, per_base, 1 << 40, d_key, d_c, d_m, None)
        for _ in range(3):
            for j in range(0, per_base, 512):
                ctx.sur_train_step(sur, d_mv[j:], d_c[j:], d_m[j:], 512)
    trained = ctx.sur_get_weights(sur)
    # A fresh base: the initial solution, proposals of iteration 0.
    ctx.solution_upload(iid, bl.SLOT_BASE, to_csr(st.x_best))
    ctx.search_start(iid, 0)
    n, k, seed = 1 << 16, 1 << 12, 3
    mv = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.generate(iid, seed, 0, 0, 0, n, mv)
    kk = torch.empty(n, dtype=torch.int64, device="cuda")
    cc = torch.empty(n, dtype=torch.float32, device="cuda")
    ctx.evaluate_batch(iid, mv, n, 1 << 40, kk, cc, None, None)
    torch.cuda.synchronize()
    keys = kk.cpu().numpy().view(np.uint64)
    cost = cc.cpu().numpy().astype(np.float64)
    ok = keys != np.uint64(M.INF_KEY)
    top = set(np.argsort(keys)[:k][ok[np.argsort(keys)[:k]]].tolist())

    def quality(sel):
        rec = len(top & set(sel.tolist())) / len(top)
        c = cost[sel[ok[sel]]]
        return rec, c.mean(), c.var(ddof=1) / c.size

    def shortlist(w):
        ctx.sur_set_weights(sur, w)
        return _screen(ctx, sur, seed, 1 << 32, n, k, margin=1e9)[0]

    rec_t, mean_t, v_t = quality(shortlist(trained))
    rec_u, mean_u, v_u = quality(shortlist(untrained))
    rng = np.random.default_rng(0)
    rec_r, mean_r, v_r = quality(rng.choice(n, k, replace=False))
    _say("recall trained %.3f untrained %.3f random %.3f; mean cost trained %.1f untrained %.1f random %.1f"
         % (rec_t, rec_u, rec_r, mean_t, mean_u, mean_r))
    # The trained shortlist holds at least twice the random share of the
    # exact top-k and more of it than the untrained network's; its mean cost
    # lies below the random shortlist's by 0.2 % and below the untrained
    # network's by more than three standard errors of the difference of the
    # two means (each standard error taken from the shortlist's own costs).
    assert rec_t >= 2.0 * max(rec_r, k / n) and rec_t > rec_u
    assert mean_t < 0.998 * mean_r
    se = np.sqrt(v_t + v_u)
    _say("trained vs untrained: %.1f below, standard error of the difference %.1f" % (mean_u - mean_t, se))
    assert mean_t < mean_u - 3.0 * se
