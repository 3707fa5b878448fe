"""The bench's step at full size: the L = 12 problem (4097 x 4097 nodes,
jitter 0.2 h, geometry seed 1003, Gaussian right-hand side seed 2003) solved
on the device in mixed precision and in FP64, each checked against the
oracle's FP64 solve of the same problem (Sec. 6.2: the mixed scheme reaches
the accuracy of the double-precision solver).

The oracle takes about 20 s for this solve on one host thread.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

L, A_JIT, GSEED, RSEED = 12, 0.2, 1003, 2003


@pytest.fixture(scope="module")
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_0904_4152_amd as mg
    mg.lib()
    return mg


def test_level_12_solves_match_oracle(mg, orc):
    N = (1 << L) + 1
    b = synth.rhs_gaussian(L, RSEED)
    oh = orc.Hierarchy(L, synth.coords(L, A_JIT, GSEED))
    xo, sto = oh.solve_fp64(b, o=orc.opts(rel_tol=1e-8))
    bands = oh.bands(L)
    ctx = mg.Context(0)
    h = mg.Hierarchy(ctx, L, jitter=A_JIT, seed=GSEED)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    # mixed: the oracle's operator confirms the 1e-8 residual; the solution
    # agrees with the FP64 one to about the condition number times 1e-8
    st = h.solve(bd, x, mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8))
    xm = x.cpu().numpy()
    r = orc.norm2(orc.defect(N, bands, b, xm)) / orc.norm2(b)
    assert st.status == 0 and r <= 1.05e-8, (st.status, r)
    assert abs(r - st.rel_res) <= 1e-3 * r
    rel_m = np.linalg.norm(xm - xo) / np.linalg.norm(xo)
    assert rel_m <= 1e-7, rel_m
    # FP64: the same cycles as the oracle, the same solution to rounding
    x.zero_()
    s64 = h.solve(bd, x, mg.default_opts(precision=mg.MG_PREC_FP64, rel_tol=1e-8))
    assert s64.status == 0 and s64.cycles == sto.cycles
    rel_f = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
    assert rel_f <= 1e-10, rel_f
    print("L=12: mixed %d outer / %d inner, rel_res %.2e, |x-x_oracle| %.2e; "
          "FP64 %d cycles, |x-x_oracle| %.2e" % (st.outer_steps, st.cycles, r, rel_m,
                                                s64.cycles, rel_f))
    oh.close()
    h.close()
