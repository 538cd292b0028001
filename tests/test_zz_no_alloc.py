"""The allocation-free batched evaluation (acopf_batch_eval_noalloc) against
acopf_batch_eval through the C ABI: bitwise-identical outputs on two calls in
a row, the second on a smaller batch that reuses the device scratch array the
first left behind, plus the f of a multi-chunk instance against the oracle and
the refusal of a batch whose objective partials exceed the array."""
import numpy as np
import pytest

import oracle as O
from paper_2203_10587_amd import synth as S
from tests.parity import assert_close, log

pytestmark = pytest.mark.gpu

SCRATCH_PARTS = 32768  # capacity stated in include/acopf.h


def _torch():
    import torch
    return torch


def _buffers(b, iterates):
    torch = _torch()
    K = b.count
    nx, nc = int(b.x_off[-1]), int(b.c_off[-1])
    x, lam = np.empty(nx), np.empty(nc)
    for k, it in enumerate(iterates):
        x[b.x_off[k]:b.x_off[k + 1]] = it.x
        lam[b.c_off[k]:b.c_off[k + 1]] = it.lam
    d = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")
    ins = dict(x=d(x), sigma=d([it.sigma for it in iterates]), lam=d(lam))

    def outs():
        nan = lambda n: torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        return dict(f=nan(K), gf=nan(nx), c=nan(nc), jv=nan(int(b.j_off[-1])),
                    hv=nan(int(b.h_off[-1])))
    return ins, outs


def _run(A, fn, b, ins, o):
    fn(b, ins["x"], ins["sigma"], ins["lam"], o["f"], o["gf"], o["c"], o["jv"], o["hv"],
       A.ACOPF_ALL)


def _check_batch(A, tag, nets, iterates):
    torch = _torch()
    b = A.acopf_batch_create(nets, tile_be=256, grid_mult=0, xcd_group=1, no_graph=0)
    ins, outs = _buffers(b, iterates)
    got, ref = outs(), outs()
    log(f"[no_alloc] {tag}: {b.count} instances, noalloc then batch_eval")
    _run(A, A.acopf_batch_eval_noalloc, b, ins, got)
    _run(A, A.acopf_batch_eval, b, ins, ref)
    torch.cuda.synchronize()
    for k in got:
        a, r = got[k].cpu().numpy(), ref[k].cpu().numpy()
        assert np.isfinite(a).all(), f"{tag}.{k}: non-finite output"
        np.testing.assert_array_equal(a, r, err_msg=f"{tag}.{k}")
    return b, got


def test_noalloc_matches_batch_eval_twice(gpu_lib):
    from paper_2203_10587_amd import acopf as A
    # 1,050 and 1,250 generators: two objective chunks per instance, so the
    # objective goes through the scratch partials
    ga = S.rgg_grid(4200, seed=7)
    gb = S.rgg_grid(2500, seed=8, gen_frac=0.5)
    g9, it9 = S.ring9(0)
    assert ga.ngen > 1024 and gb.ngen > 1024
    rng = np.random.default_rng(11)
    ita, itb = S.draw_iterate(ga, rng), S.draw_iterate(gb, rng)
    na, nb_, n9 = A.acopf_net_create(ga), A.acopf_net_create(gb), A.acopf_net_create(g9)
    ca1, ca2 = A.acopf_net_create_outage(na, 5), A.acopf_net_create_outage(na, 400)
    # an outage child has two flow rows fewer: its iterate is drawn on its own grid
    ita1 = S.draw_iterate(S.remove_branch(ga, 5), rng)
    ita2 = S.draw_iterate(S.remove_branch(ga, 400), rng)

    # first call: 5 instances, 9 partials
    b1, got1 = _check_batch(A, "call1", [na, n9, ca1, nb_, ca2], [ita, it9, ita1, itb, ita2])
    # second call: a smaller batch whose multi-chunk instance now sits where
    # the first call's instance 0 left its partials
    b2, got2 = _check_batch(A, "call2", [nb_, n9], [itb, it9])
    assert got1["f"][3].item() == got2["f"][0].item()

    # the multi-chunk objective against the oracle
    mdl = O.prepare(gb)
    out = O.evaluate(mdl, itb.x, itb.sigma, itb.lam)
    sc = O.scales(mdl, itb.x, out, itb.sigma, itb.lam)
    assert_close("call2.f", [got2["f"][0].item()], [out["f"]], [sc["f"]])
    b1.close()
    b2.close()


def test_noalloc_refuses_oversized_batch(gpu_lib):
    from paper_2203_10587_amd import acopf as A
    torch = _torch()
    g9, _ = S.ring9(0)
    n9 = A.acopf_net_create(g9)
    count = SCRATCH_PARTS + 1  # one objective partial per 9-bus instance
    b = A.acopf_batch_create([n9] * count, tile_be=256, grid_mult=0, xcd_group=1, no_graph=1)
    x = torch.zeros(int(b.x_off[-1]), dtype=torch.float64, device="cuda")
    f = torch.zeros(count, dtype=torch.float64, device="cuda")
    log(f"[no_alloc] refusal: {count} instances")
    with pytest.raises(A.AcopfError) as ei:
        A.acopf_batch_eval_noalloc(b, x, None, None, f, None, None, None, None, A.ACOPF_F)
    assert ei.value.code == A.ACOPF_EINVAL
    assert "objective partials" in str(ei.value)
    b.close()
