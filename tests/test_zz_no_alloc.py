"""bl_evaluate_batch_static (the evaluation for callers that cannot allocate,
its deferred list in a static device array) against bl_evaluate_batch on
the same moves: identical outputs, on two calls in a row, the second
smaller, at sizes where the launch defers long SU tails to its second pass."""
import sys

import numpy as np
import pytest

from oracle import init as OI
from oracle import model as M
from oracle import moves as MV
from oracle import search as S
from paper_1909_10286_amd import bl, inputs

from .gpu_common import to_csr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _walked(inst, steps=40):
    x = OI.init_solution(inst)
    for i in range(steps):
        y = MV.apply_move(x, MV.draw_move(inst, x, 5, 999, i))
        if M.is_feasible(inst, y):
            x = y
    return S.with_units(x, M.evaluate_solution(inst, x))


def _eval(fn, iid, d_mv, n, t_star):
    out = (torch.full((n,), -1, dtype=torch.int64, device="cuda"),
           torch.full((n,), -1.0, dtype=torch.float32, device="cuda"),
           torch.full((n,), -1, dtype=torch.int32, device="cuda"),
           torch.full((n,), 255, dtype=torch.uint8, device="cuda"))
    fn(iid, d_mv, n, t_star, *out)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


@pytest.mark.parametrize("name", ["mid100", "clust500"])
def test_static_scratch_evaluation_matches(ctx, name):
    _say("static scratch evaluation", name)
    inst = inputs.make_instance(name, 0, accept=OI.init_feasible)
    base = _walked(inst)
    iid = ctx.instance_upload(inst)
    ctx.solution_upload(iid, bl.SLOT_BASE, to_csr(base))
    n1, n2 = 1 << 20, 300007
    d_mv = torch.empty(n1, dtype=torch.int64, device="cuda")
    ctx.generate(iid, 77, 4, 0, 0, n1, d_mv)
    for n in (n1, n2):
        want = _eval(ctx.evaluate_batch, iid, d_mv, n, 1 << 40)
        got = _eval(ctx.evaluate_batch_static, iid, d_mv, n, 1 << 40)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), (name, n)
        assert (want[0] != -1).any() and (want[3] == 0).any()
    with pytest.raises(bl.BlError) as e:
        ctx.evaluate_batch_static(iid, d_mv, (1 << 24) + 1, 0, d_mv)
    assert e.value.status == bl.EINVAL
    ctx.evaluate_batch_static(iid, d_mv, 0, 0, d_mv)
