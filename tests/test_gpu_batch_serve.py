"""Batched solves and the serving loop on the device.

A problem's arithmetic is the same whichever other problems share the
launches (same per-tile device functions, per-problem reductions in a fixed
order, stop decisions per problem), so its result must be bit-identical
alone, in a batch, in the server's live mix and in the single-problem solver.
Convergence is checked independently with the CPU oracle's operator.
"""
import numpy as np
import pytest

import synth
from gpu_common import U64, abs_band_product

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


def make_problems(mg, ctx, levels, seed0=4100):
    probs = []
    amps = synth.batch_jitter(len(levels), 0.25, 4005)
    for k, L in enumerate(levels):
        h = mg.Hierarchy(ctx, int(L), jitter=float(amps[k]), seed=seed0 + k)
        b = torch.empty(h.n, dtype=torch.float64, device="cuda")
        h.rhs_uniform(4200 + k, b)
        probs.append((h, b, float(amps[k]), seed0 + k))
    return probs


LEVELS = [5, 2, 8, 3, 7, 6, 4, 8, 1, 6]


def test_batch_equals_single_solver_bitwise(mg, ctx):
    probs = make_problems(mg, ctx, LEVELS)
    opts = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8)
    xs = [torch.zeros_like(b) for _, b, _, _ in probs]
    stats = mg.solve_batch([p[0] for p in probs], [p[1] for p in probs], xs, opts)
    for k, (h, b, _, _) in enumerate(probs):
        x1 = torch.zeros_like(b)
        s1 = h.solve(b, x1, opts)
        assert stats[k].status == 0 and stats[k].rel_res <= 1e-8
        assert (stats[k].cycles, stats[k].outer_steps) == (s1.cycles, s1.outer_steps)
        np.testing.assert_array_equal(host(xs[k]), host(x1))
        assert stats[k].rel_res == s1.rel_res


def test_batch_warm_and_cold_starts_equal_single(mg, ctx):
    """Problems started from a nonzero iterate (their first defect reads x)
    and from zero (their first defect is b itself, without the bands) in one
    batch: each equals the single-problem solver from the same start, bit
    for bit."""
    levels = [6, 7, 5, 8, 6, 7]
    probs = make_problems(mg, ctx, levels, seed0=960)
    opts = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-9)
    rng = np.random.default_rng(961)
    x0s = []
    for k, L in enumerate(levels):
        x0 = np.zeros(probs[k][0].n)
        if k % 2 == 0:
            x0 = rng.standard_normal(x0.size) * 0.01
            x0[~synth.interior_mask(L)] = 0.0
        x0s.append(x0)
    xs = [torch.from_numpy(x0.copy()).cuda() for x0 in x0s]
    stats = mg.solve_batch([p[0] for p in probs], [p[1] for p in probs], xs, opts)
    for k, (h, b, _, _) in enumerate(probs):
        x1 = torch.from_numpy(x0s[k].copy()).cuda()
        s1 = h.solve(b, x1, opts)
        assert stats[k].status == 0 and stats[k].rel_res <= 1e-9
        assert (stats[k].cycles, stats[k].outer_steps) == (s1.cycles, s1.outer_steps)
        assert stats[k].rel_res == s1.rel_res
        np.testing.assert_array_equal(host(xs[k]), host(x1))
    for h, _, _, _ in probs:
        h.close()


def test_batch_alone_equals_in_the_mix(mg, ctx):
    probs = make_problems(mg, ctx, LEVELS, seed0=900)
    opts = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-10)
    xs = [torch.zeros_like(b) for _, b, _, _ in probs]
    mg.solve_batch([p[0] for p in probs], [p[1] for p in probs], xs, opts)
    for k in (0, 2, 8):
        h, b, _, _ = probs[k]
        x1 = torch.zeros_like(b)
        st = mg.solve_batch([h], [b], [x1], opts)
        np.testing.assert_array_equal(host(xs[k]), host(x1))
        assert st[0].status == 0


def test_batch_composition_changes_tiling_not_bits(mg, ctx):
    # The fused passes pick each level's chunk height from how many problems
    # share the level, and the batch machinery is reused between calls; a
    # problem's result must not change with either.  Problem 0 (L = 9) is
    # solved among 40, among 10 and alone (chunk heights 32, 8 and 4 rows at
    # L = 9), in calls of shrinking size, and by the single-problem solver.
    crowd = make_problems(mg, ctx, [9] * 40, seed0=3000)
    opts = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8)
    h0, b0 = crowd[0][0], crowd[0][1]
    results = []
    for group in (crowd, crowd[:10], crowd[:1]):
        xs = [torch.zeros_like(p[1]) for p in group]
        st = mg.solve_batch([p[0] for p in group], [p[1] for p in group], xs, opts)
        assert all(s.status == 0 and s.rel_res <= 1e-8 for s in st)
        results.append((host(xs[0]), st[0].cycles, st[0].rel_res))
    for x, cyc, rel in results[1:]:
        np.testing.assert_array_equal(x, results[0][0])
        assert (cyc, rel) == results[0][1:]
    x1 = torch.zeros_like(b0)
    s1 = h0.solve(b0, x1, opts)
    np.testing.assert_array_equal(host(x1), results[0][0])
    assert s1.cycles == results[0][1]
    for h, _, _, _ in crowd:
        h.close()


def test_batch_per_problem_tolerances_checked_by_oracle(mg, ctx, orc):
    levels = [6, 7, 5, 8]
    tols = [1e-6, 1e-8, 1e-10, 1e-8]
    probs = make_problems(mg, ctx, levels, seed0=300)
    opts = [mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=t) for t in tols]
    xs = [torch.zeros_like(b) for _, b, _, _ in probs]
    stats = mg.solve_batch([p[0] for p in probs], [p[1] for p in probs], xs, opts)
    for k, (h, b, a, gs) in enumerate(probs):
        L = levels[k]
        N = (1 << L) + 1
        bands = orc.assemble(N, synth.coords(L, a, gs))
        bh = host(b)
        bref = synth.rhs_uniform(L, 4200 + k)
        np.testing.assert_array_equal(bh, bref)  # device RHS generator = host generator
        r = orc.norm2(orc.defect(N, bands, bh, host(xs[k]))) / orc.norm2(bh)
        assert stats[k].status == 0
        assert r <= 1.05 * tols[k], (k, r, tols[k])


def test_batch_of_config_shape(mg, ctx):
    """Levels drawn from {5..9} (seed 4004), jitter U[0, 0.25) per problem:
    every problem reaches 1e-8."""
    levels = synth.batch_levels(48, 5, 9, 4004)
    probs = make_problems(mg, ctx, levels)
    opts = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8)
    xs = [torch.zeros_like(b) for _, b, _, _ in probs]
    stats = mg.solve_batch([p[0] for p in probs], [p[1] for p in probs], xs, opts)
    for s in stats:
        assert s.status == 0 and s.rel_res <= 1e-8
        assert 3 <= s.outer_steps <= 6


def test_batch_of_config_shape_256_checked_by_oracle(mg, ctx, orc):
    """The benchmark's batch at full shape: 256 problems, levels from {5..9}
    (seed 4004), jitter U[0, 0.25) h (seed 4005), geometry seeds 4100 + p,
    uniform right-hand sides 4200 + p.  Every problem's right-hand side equals
    the host generator's and its final residual, recomputed with the oracle's
    operator on the host coordinates, is within 1e-8 of ||b||; for 32 problems
    (every level) the solution is compared with the oracle's FP64 solution."""
    count = 256
    levels = synth.batch_levels(count, 5, 9, 4004)
    probs = make_problems(mg, ctx, levels)
    opts = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8)
    xs = [torch.zeros_like(b) for _, b, _, _ in probs]
    print("batch of 256: levels %s" % np.bincount(levels, minlength=10)[5:].tolist(), flush=True)
    stats = mg.solve_batch([p[0] for p in probs], [p[1] for p in probs], xs, opts)
    sample = set()
    for L in range(5, 10):
        sample.update(np.nonzero(levels == L)[0][:7 if L < 9 else 4].tolist())
    worst_res, worst_err = 0.0, 0.0
    for k, (h, b, a, gs) in enumerate(probs):
        L = int(levels[k])
        N = (1 << L) + 1
        xy = synth.coords(L, a, gs)
        bh = host(b)
        np.testing.assert_array_equal(bh, synth.rhs_uniform(L, 4200 + k))
        xk = host(xs[k])
        bands = orc.assemble(N, xy)
        bn = orc.norm2(bh)
        r = orc.norm2(orc.defect(N, bands, bh, xk)) / bn
        assert stats[k].status == 0 and stats[k].rel_res <= 1e-8, k
        assert r <= 1.05e-8, (k, L, r)
        # the device's residual norm against the oracle's: the defect's
        # forward error (9-term products, bands within 64 ulp of the
        # oracle's) bounds the difference, whatever the residual's size
        scale = np.linalg.norm(abs_band_product(N, bands, xk) + np.abs(bh))
        assert abs(r - stats[k].rel_res) * bn <= 80 * U64 * scale, (k, r, stats[k].rel_res)
        worst_res = max(worst_res, r)
        if k in sample:
            oh = orc.Hierarchy(L, xy)
            xo, so = oh.solve_fp64(bh, o=orc.opts(rel_tol=1e-12))
            oh.close()
            err = float(np.linalg.norm(xk - xo) / np.linalg.norm(xo))
            assert err <= 1e-6, (k, L, err)
            worst_err = max(worst_err, err)
    assert len(sample) == 32
    print("batch of 256: worst oracle residual %.3e, worst solution error %.3e (32 problems)"
          % (worst_res, worst_err))
    for h, _, _, _ in probs:
        h.close()


def test_batch_errors(mg, ctx):
    probs = make_problems(mg, ctx, [4, 5])
    xs = [torch.zeros_like(b) for _, b, _, _ in probs]
    with pytest.raises(mg.MgError) as e:
        mg.solve_batch([p[0] for p in probs], [p[1] for p in probs], xs,
                       mg.default_opts(precision=mg.MG_PREC_FP64))
    assert e.value.status == mg.MG_ERR_INVALID
    with pytest.raises(mg.MgError) as e:
        mg.solve_batch([probs[0][0], probs[0][0]], [probs[0][1]] * 2, xs,
                       mg.default_opts(precision=mg.MG_PREC_MIXED))
    assert e.value.status == mg.MG_ERR_INVALID
    # the problems work in place: no shared x, no x that is another's b
    hs2 = [probs[0][0], probs[1][0]]
    same = [torch.zeros_like(probs[1][1])] * 2
    for bs_, xs_ in (([probs[0][1], probs[1][1]], same),
                     ([probs[0][1], xs[0]], [xs[0], xs[1]])):
        with pytest.raises(mg.MgError) as e:
            mg.solve_batch(hs2, bs_, xs_, mg.default_opts(precision=mg.MG_PREC_MIXED))
        assert e.value.status == mg.MG_ERR_INVALID


def test_batch_zero_rhs_and_early_stop_give_zero_x(mg, ctx):
    """A zero right-hand side gives x = 0 (whatever x held); a zero guess
    whose first defect already meets the tolerance gives x = 0 too; the
    other problems of the batch are unaffected."""
    probs = make_problems(mg, ctx, [5, 6, 7])
    hs = [p[0] for p in probs]
    bs = [p[1] for p in probs]
    bs[0] = torch.zeros_like(bs[0])
    ref = torch.zeros_like(bs[2])
    st_ref = hs[2].solve(bs[2], ref, mg.default_opts(precision=mg.MG_PREC_MIXED))
    for zg in (0, 1):
        xs = [torch.full_like(b, 3.0) for b in bs]
        xs[2].zero_()
        opts = [mg.default_opts(precision=mg.MG_PREC_MIXED, zero_guess=zg),
                mg.default_opts(precision=mg.MG_PREC_MIXED, zero_guess=1, rel_tol=10.0),
                mg.default_opts(precision=mg.MG_PREC_MIXED, zero_guess=zg)]
        st = mg.solve_batch(hs, bs, xs, opts)
        torch.cuda.synchronize()
        assert all(s.status == 0 for s in st)
        assert not xs[0].cpu().numpy().any() and not xs[1].cpu().numpy().any()
        assert st[1].outer_steps == 0
        np.testing.assert_array_equal(xs[2].cpu().numpy(), ref.cpu().numpy())
        assert (st[2].cycles, st[2].rel_res) == (st_ref.cycles, st_ref.rel_res)


def test_server_result_same_alone_and_in_the_mix(mg, ctx, orc):
    """Requests that overlap on the device (more requests than slots, so they
    are admitted as slots free up) give bit-identical results to the same
    problem solved alone."""
    srv = mg.Server(ctx, slots=4, budget_bytes=8 << 30, max_level=9)
    reqs = []
    rng = np.random.default_rng(5)
    for r in range(10):
        L = int(rng.integers(4, 10))
        tol = [1e-6, 1e-8, 1e-10][r % 3]
        a = float(rng.uniform(0, 0.25))
        t = srv.submit(L, tol, a, 5100 + r, 5200 + r, keep_x=True)
        reqs.append((t, L, tol, a, 5100 + r, 5200 + r))
    results = {}
    for t, L, *_ in reqs:
        while True:
            rc, st, x = srv.poll(t, n=((1 << L) + 1) ** 2)
            if rc != mg.MG_ERR_BUSY:
                break
            import time
            time.sleep(0.002)
        results[t] = (rc, st, x)
    info = srv.info()
    srv.close()
    assert info.completed == 10
    for t, L, tol, a, gs, rs in reqs:
        rc, st, x = results[t]
        assert rc == 0 and st.rel_res <= tol
        assert st.seconds >= st.queue_seconds >= 0.0
        # the served solution against the oracle's operator on the host
        # coordinates and right-hand side of the request
        N = (1 << L) + 1
        bh = synth.rhs_uniform(L, rs)
        r = orc.norm2(orc.defect(N, orc.assemble(N, synth.coords(L, a, gs)), bh, x))
        assert r <= 1.05 * tol * orc.norm2(bh), (t, L, tol, r)
        h = mg.Hierarchy(ctx, L, jitter=a, seed=gs)
        b = torch.empty(h.n, dtype=torch.float64, device="cuda")
        h.rhs_uniform(rs, b)
        x1 = torch.zeros_like(b)
        s1 = mg.solve_batch([h], [b], [x1], mg.default_opts(precision=mg.MG_PREC_MIXED,
                                                            rel_tol=tol))
        np.testing.assert_array_equal(x, host(x1))
        assert (st.cycles, st.outer_steps) == (s1[0].cycles, s1[0].outer_steps)


def test_server_budget_admission(mg, ctx):
    one = mg.Hierarchy.bytes_needed(9)
    srv = mg.Server(ctx, slots=8, budget_bytes=int(one * 1.5), max_level=9)
    with pytest.raises(mg.MgError) as e:  # can never fit: rejected at submission
        mg.Server(ctx, slots=1, budget_bytes=one // 2, max_level=9).submit(9, 1e-8, 0.1, 1, 2)
    assert e.value.status == mg.MG_ERR_NOMEM
    tickets = [srv.submit(9, 1e-8, 0.1, 10 + k, 20 + k) for k in range(4)]
    got = []
    while len(got) < 4:
        r = srv.next(timeout=5.0)
        assert r is not None
        got.append(r)
    info = srv.info()
    srv.close()
    assert sorted(t for t, _, _ in got) == sorted(tickets)
    assert all(rc == 0 for _, rc, _ in got)
    assert info.bytes_high_water <= int(one * 1.5)


def test_autotuned_tiles_change_no_bit(mg, ctx, tmp_path):
    """The autotuner picks a tile per level of this composition (a marching
    tile's height and workgroup width, or a block tile's shape); the batch
    solved with the tuned table, with forced odd choices (rows and widths no
    rule picks, every block shape) and with the rules' choices gives the
    same bits, and the table round-trips through a file."""
    probs = make_problems(mg, ctx, [9, 8, 7, 6, 5, 9, 8, 7] * 3, seed0=5000)
    opts = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8)
    hs, bs_ = [p[0] for p in probs], [p[1] for p in probs]

    def run():
        xs = [torch.zeros_like(b) for b in bs_]
        st = mg.solve_batch(hs, bs_, xs, opts)
        assert all(s.status == 0 and s.rel_res <= 1e-8 for s in st)
        return [host(x) for x in xs], [(s.cycles, s.outer_steps, s.rel_res) for s in st]

    mg.batch_clear_tiles()
    ref_x, ref_s = run()
    rows = mg.batch_autotune(hs, opts, reps=3)
    assert sorted(r["level"] for r in rows) == [5, 6, 7, 8, 9]
    for r in rows:
        assert r["us"] > 0.0
        if r["tile_cols"]:
            assert r["tile_cols"] == 32 and r["tile_rows"] in (8, 16, 32)
            assert r["row_waves"] == 4
        else:
            assert r["tile_rows"] in (4, 8, 12, 16, 24, 32, 48, 64, 96)
            assert r["row_waves"] in (1, 2, 3, 4)
    # problems per level: levels above the coarse tail (5) run for every
    # problem that has them, level 5 only as a finest level
    by_level = {r["level"]: r["problems"] for r in rows}
    assert by_level == {9: 6, 8: 12, 7: 18, 6: 21, 5: 3}
    x1, s1 = run()
    path = str(tmp_path / "tiles.json")
    mg.save_tiles(rows, path)
    mg.batch_clear_tiles()
    assert mg.load_tiles(path) == rows
    x2, s2 = run()
    mg.batch_set_tiles([{"level": 9, "problems": 6, "tile_rows": 128}])  # not a tuner candidate
    x3, s3 = run()
    # every width at every level of the composition, with odd heights
    outs = [(x1, s1), (x2, s2), (x3, s3)]
    for waves, rows_ in ((1, 8), (3, 16), (2, 64), (4, 4), (2, 12), (1, 40), (3, 100)):
        mg.batch_set_tiles([{"level": l, "problems": p, "tile_rows": rows_, "row_waves": waves}
                            for l, p in by_level.items()])
        outs.append(run())
    # block tiles at every level, and block and marching tiles mixed
    for rows_ in (8, 16, 32):
        mg.batch_set_tiles([{"level": l, "problems": p, "tile_rows": rows_, "tile_cols": 32}
                            for l, p in by_level.items()])
        outs.append(run())
    mg.batch_set_tiles([{"level": l, "problems": p, "tile_rows": 16, "tile_cols": 32 * (l % 2)}
                        for l, p in by_level.items()])
    outs.append(run())
    for xs, ss in outs:
        assert ss == ref_s
        for a, b in zip(xs, ref_x):
            np.testing.assert_array_equal(a, b)
    with pytest.raises(mg.MgError):
        mg.batch_set_tiles([{"level": 9, "problems": 6, "tile_rows": 14}])
    for bad_rows in (0, 2, 260):
        with pytest.raises(mg.MgError):
            mg.batch_set_tiles([{"level": 9, "problems": 6, "tile_rows": bad_rows}])
    with pytest.raises(mg.MgError):
        mg.batch_set_tiles([{"level": 9, "problems": 6, "tile_rows": 16, "row_waves": 5}])
    for bad in ({"tile_rows": 64, "tile_cols": 32}, {"tile_rows": 16, "tile_cols": 16},
                {"tile_rows": 16, "tile_cols": 32, "row_waves": 2}):
        with pytest.raises(mg.MgError):
            mg.batch_set_tiles([dict(level=9, problems=6, **bad)])
    mg.batch_clear_tiles()
    for h, _, _, _ in probs:
        h.close()
