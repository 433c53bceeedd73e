"""Serving pool: solves stepped together in batched launches give the same results
as the same solves run alone, admission respects the memory arena, and requests
submitted while others run are admitted as memory frees up."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2604_06309_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests(n, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        a2 = rng.dirichlet([1.0, 1.0, 1.0])
        L = int(rng.choice([64, 96, 128]))
        p = pk.make_params({2: a2[0], 3: a2[1], 4: a2[2]}, float(rng.uniform(0.4, 1.2)),
                           t_max=float(np.exp(rng.uniform(np.log(4.0), np.log(8.0)))), L=L, M_cap=1500,
                           eps=1e-7, dt0=1e-3, dt_min=1e-10)
        out.append(p)
    return out


def _solo(p):
    s = pk.Solver(p)
    st, info = s.step(float("inf"))
    res = (s.read(pk.F_T_GRID), s.read(pk.F_C), s.read(pk.F_R), info.accepted, info.rejected)
    s.close()
    return res


def test_pool_matches_solo_runs_and_admits_by_memory():
    say("pool vs solo")
    reqs = _requests(10)
    solo = [_solo(p) for p in reqs]
    fp = max(pk.dmfe_footprint(p) for p in reqs)
    arena = 3 * fp + 4096  # room for three of the largest solves, not for all six of the first batch
    pool = pk.Pool(arena, max_instances=8)
    ids = [pool.submit(p) for p in reqs[:6]]
    st = pool.run(50)
    assert st.bytes_total - st.bytes_free <= arena
    assert st.running >= 1 and st.queued >= 1 and st.running + st.queued + st.finished_unreleased == 6
    ids += [pool.submit(p) for p in reqs[6:]]  # arrive while others run
    done = {}
    for _ in range(100000):
        st = pool.run(200)
        for rid in pool.poll():
            info, tm = pool.result(rid)
            k = ids.index(rid)
            assert tm.status == pk.DONE, (rid, tm.status)
            L = reqs[k].L
            done[rid] = (pool.read(rid, pk.F_T_GRID), pool.read(rid, pk.F_C, L=L), pool.read(rid, pk.F_R, L=L),
                         info.accepted, info.rejected, tm.total_s)
            pool.release(rid)
        assert st.bytes_total - st.bytes_free <= arena
        if len(done) == len(reqs):
            break
    assert len(done) == len(reqs)
    for k, rid in enumerate(ids):
        t, C, R, acc, rej, tts = done[rid]
        t0, C0, R0, acc0, rej0 = solo[k]
        assert (acc, rej) == (acc0, rej0)
        np.testing.assert_array_equal(t, t0)
        np.testing.assert_array_equal(C, C0)
        np.testing.assert_array_equal(R, R0)
    say(f"  {len(reqs)} solves identical to solo runs; ticks={st.ticks}")
    pool.close()


def test_pool_rejects_what_cannot_fit():
    p = _requests(1)[0]
    pool = pk.Pool(pk.dmfe_footprint(p) // 2, max_instances=2)
    with pytest.raises(pk.DmfeError) as e:
        pool.submit(p)
    assert e.value.status == pk.ERR_NOMEM
    pool.close()


@pytest.mark.parametrize("precision", [pk.FP64, pk.FP32_COMP])
def test_sixteen_large_instances_stepped_together(precision):
    """The large-grid stress case: 16 identical solves of the 2+4 model (a2^2 = 0.3,
    a4^2 = 0.7, T = 0.45, t_max = 1e7) on a 8192-point grid with history cap 8192,
    all admitted at once and stepped together in batched launches.  After the
    same number of ticks every instance holds bitwise the same history, equal to
    the same solve run alone for the same number of steps."""
    say(f"16 instances at L=8192, precision={precision}")
    p = pk.make_params({2: 0.3, 4: 0.7}, 0.45, t_max=1e7, L=8192, M_cap=8192, eps=1e-8, dt0=1e-3, dt_min=1e-12,
                       precision=precision)
    fp = pk.dmfe_footprint(p)
    pool = pk.Pool(16 * fp + 4096, max_instances=16)
    ids = [pool.submit(p) for _ in range(16)]
    st = pool.run(6 * 25)
    assert st.running == 16 and st.queued == 0
    infos = [pool.result(rid)[0] for rid in ids]
    steps = infos[0].accepted + infos[0].rejected
    assert steps >= 20 and all((i.accepted, i.rejected, i.M, i.t) == (infos[0].accepted, infos[0].rejected,
                                                                        infos[0].M, infos[0].t) for i in infos)
    ref = [pool.read(ids[0], f, L=8192) for f in (pk.F_T_GRID, pk.F_C, pk.F_R)]
    for rid in ids[1:]:
        for f, r in zip((pk.F_T_GRID, pk.F_C, pk.F_R), ref):
            np.testing.assert_array_equal(pool.read(rid, f, L=8192), r)
    pool.close()
    s = pk.Solver(p)
    _, info = s.step(float("inf"), steps)
    assert (info.accepted, info.rejected, info.M) == (infos[0].accepted, infos[0].rejected, infos[0].M)
    np.testing.assert_array_equal(s.read(pk.F_T_GRID), ref[0])
    np.testing.assert_array_equal(s.read(pk.F_C), ref[1])
    np.testing.assert_array_equal(s.read(pk.F_R), ref[2])
    s.close()
    say(f"  16 instances bitwise equal to each other and to the solo solve after {steps} steps, M={info.M}")


@pytest.mark.parametrize("precision", [pk.FP64, pk.FP32_COMP])
def test_sixteen_large_instances_with_a_long_history(precision):
    """The large-grid stress case with a history of 400 stored slices: the solve is
    first run alone for 400 steps; its stored history then resumes the 16 pooled
    solves (dmfe_pool_set_history) and, once more, the solve alone
    (dmfe_set_history); all are stepped for 60 ticks' worth of stages.  Every
    pooled instance stays bitwise equal to the others and to the solo solve after
    the same number of steps."""
    say(f"16 instances at L=8192 with 400 stored slices, precision={precision}")
    L, M = 8192, 401
    p = pk.make_params({2: 0.3, 4: 0.7}, 0.45, t_max=1e7, L=L, M_cap=512, eps=1e-8, dt0=1e-3, dt_min=1e-12,
                       precision=precision)
    s = pk.Solver(p)
    _, info0 = s.step(float("inf"), M - 1)
    assert info0.M == M and info0.nb_valid == M
    times, C, R, dC, dR = (s.read(f) for f in (pk.F_T_GRID, pk.F_C, pk.F_R, pk.F_DC, pk.F_DR))
    dt0 = info0.dt
    pool = pk.Pool(16 * pk.dmfe_footprint(p) + 4096, max_instances=16)
    ids = [pool.submit(p) for _ in range(16)]
    st = pool.run(0)  # admission only
    assert st.running == 16
    for rid in ids:
        pool.set_history(rid, times, C, R, dC, dR, dt=dt0, scheme=pk.SCHEME_DP5)
    st = pool.run(60)
    assert st.running == 16
    infos = [pool.result(rid)[0] for rid in ids]
    steps = infos[0].accepted + infos[0].rejected
    assert steps >= 5 and infos[0].M >= M
    ref = [pool.read(ids[0], f, L=L) for f in (pk.F_T_GRID, pk.F_C, pk.F_R, pk.F_DC)]
    for rid in ids[1:]:
        for f, r in zip((pk.F_T_GRID, pk.F_C, pk.F_R, pk.F_DC), ref):
            np.testing.assert_array_equal(pool.read(rid, f, L=L), r)
    pool.close()
    s.set_history(times, C, R, dC, dR, dt=dt0, scheme=pk.SCHEME_DP5)
    a0 = s.info()
    _, info = s.step(float("inf"), steps)
    assert (info.accepted - a0.accepted, info.rejected - a0.rejected, info.M) == (infos[0].accepted,
                                                                                  infos[0].rejected, infos[0].M)
    for f, r in zip((pk.F_T_GRID, pk.F_C, pk.F_R, pk.F_DC), ref):
        np.testing.assert_array_equal(s.read(f), r)
    s.close()
    say(f"  16 instances bitwise equal to each other and to the solo solve after {steps} steps, M={info.M}")
