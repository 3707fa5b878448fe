"""Tiles of the single-problem fused passes (Sec. 3: the thread-block
partition is a runtime parameter): the autotuner's choices, forced odd
choices (marching tiles and every block tile shape) and the rules give the
same bits in the cycle, the FP64 solve, the mixed solve and the post pass's
residual norm, and a tuned solve captured before a table change is captured
again with the new tiles."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_0904_4152_amd as mg
    mg.lib()
    return mg


@pytest.fixture(scope="module")
def ctx(mg):
    return mg.Context(0)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def run_all(mg, h, L, b64):
    """Bits that must not depend on the tiles: one FP32 and one FP64 fused
    cycle, the post pass's residual norm, a mixed and an FP64 solve."""
    n = h.n
    rng = np.random.default_rng(L)
    x0 = rng.standard_normal(n) * 0.1
    x0[~synth.interior_mask(L)] = 0.0
    out = []
    for dt in (torch.float32, torch.float64):
        x = torch.from_numpy(x0).to(dt).cuda()
        h.vcycle(L, b64.to(dt), x, fused=True)
        out.append(host(x))
        xo = torch.empty_like(x)
        nc = ((1 << (L - 1)) + 1) ** 2
        xc = torch.from_numpy(rng.standard_normal(nc) * 0.01).to(dt).cuda()
        out.append(np.array([h.post_smooth(L, b64.to(dt), x, xc, xo, norm=True)]))
        out.append(host(xo))
    for prec in (mg.MG_PREC_MIXED, mg.MG_PREC_FP64):
        x = torch.zeros_like(b64)
        st = h.solve(b64, x, mg.default_opts(precision=prec, rel_tol=1e-8))
        assert st.status == 0 and st.rel_res <= 1e-8
        out.append(host(x))
        out.append(np.array([st.cycles, st.outer_steps, st.rel_res]))
    return out


@pytest.mark.parametrize("L", [7, 11])
def test_single_tiles_change_no_bit(mg, ctx, L):
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=700 + L)
    b = torch.from_numpy(synth.rhs_uniform(L, 710 + L)).cuda()
    mg.batch_clear_tiles()
    ref = run_all(mg, h, L, b)
    rows = h.autotune(reps=2)
    levels = sorted(r["level"] for r in rows)
    assert levels == list(range(6, L + 1)), levels
    for r in rows:
        assert r["problems"] == 1 and r["us"] > 0.0
        if r["tile_cols"]:
            assert r["level"] <= 10 and r["tile_cols"] == 32 and r["tile_rows"] in (8, 16, 32)
        else:
            assert r["tile_rows"] in (4, 8, 12, 16, 24, 32, 40, 48, 64, 80, 96, 128, 160,
                                      192, 256)
            assert r["row_waves"] in (1, 2, 3, 4)
    tuned = run_all(mg, h, L, b)
    # forced choices no rule picks, every level at once
    forced = []
    for waves, rows_, cols in ((1, 128, 0), (3, 4, 0), (2, 32, 0), (2, 12, 0), (1, 44, 0),
                               (4, 8, 32), (0, 16, 32), (4, 32, 32)):
        for lv in levels:
            mg.batch_set_tiles([{"level": lv, "problems": 1, "tile_rows": rows_,
                                 "row_waves": waves, "tile_cols": cols}])
        forced.append(run_all(mg, h, L, b))
    mg.batch_clear_tiles()
    again = run_all(mg, h, L, b)
    for got in [tuned, again] + forced:
        assert len(got) == len(ref)
        for a, c in zip(got, ref):
            np.testing.assert_array_equal(a, c)
    h.close()
