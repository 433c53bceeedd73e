#!/usr/bin/env python3
"""RK steps/s of the MI355X DMFE solver at theta-grid length L = 4096.

Workload: the mixed spherical 3+4 model (a_3^2 = a_4^2 = 1/2) at T = 0.55 with
t_max = 1e7 (gamma = 19.066), L = 4096, history capacity 4096 slices,
tolerance 1e-8, DP5 then SSPRK(10,4), automatic sparsification.  Inputs are
the model parameters: the history is produced by the solver itself.

Phases: (1) untimed fill from t = 0 until the history first reaches its
capacity and an automatic sparsification pass has run (the steady state of
the method), (2) W untimed warm-up steps, (3) exactly K timed steps between
device synchronisations.  Per-kernel durations are HIP events recorded by the
library on its own stream during (3).  The line's value is the --precision
solve (FP64 by default); the same three phases then run for the other
precision (FP32-compensated history by default) and are reported beside it.
Then come the end-to-end run of the uniform-grid configuration (p=3, N=1000,
with the oracle timed beside it), the serving sweep and the CPU baseline (the
oracle).  --c2 adds the L=2048 configuration from t=0 to t_max=1e4, --aging
the paper's energy-exponent experiment (pure p=3 quenched to T=0).

One JSON line is printed on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "RK steps/s at grid L=4096 (FP64 vs FP32-comp); sweep solves/s + p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def calibration_copies(torch, nbytes: int = 256 << 20, reps: int = 2):
    """Plain device copies of known size (a blit and an elementwise kernel that
    read and write nbytes each), run right after the timed launches so that
    hardware byte counters of a profiled run can be scaled to bytes."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    return {"bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}


def traffic_record(L: int, precision: str):
    """HBM bytes per launch of the history-integral kernel, from the committed
    counter summary, if it was taken on the kernel source as it is now."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hist_integral_L{L}_{precision}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2604_06309_amd", "csrc", "kernels_theta.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("kernel_source_sha256") != sha:
        return None
    return float(rec["traffic_bytes_per_launch"])


def workload_params(pk, precision):
    return pk.make_params({3: 0.5, 4: 0.5}, 0.55, t_max=1e7, L=4096, M_cap=4096, eps=1e-8, dt0=1e-3,
                          dt_min=1e-12, precision=precision)


def touched_points(th, thc, tgrid, t, gamma, s: int = 10) -> int:
    """(slice, node) points of the stored history that one right-hand side at
    stage time t reads: for every pair (i, j) the s-point stencil around
    x(psi_ij) on the two slices bracketing phi_ij t (the last slice only when
    phi_ij t is inside the current step), and every node of the two slices
    bracketing theta_j t for row j.  The index map is the inverse of eq. (theta)
    at alpha = 0, evaluated here in numpy as a measurement aid."""
    import numpy as np
    L = th.size
    M = tgrid.size
    D = np.arctan(np.sinh(gamma))
    xs, eg, egi = (L - 1) / (2 * gamma), np.exp(gamma), np.exp(-gamma)

    def xmap(a, ac):
        lo = a <= 0.5
        T = np.tan(np.where(lo, a, ac) * D)
        x = xs * (np.log1p(eg * T) - np.log1p(-egi * T))
        return np.where(lo, x, L - 1 - x)

    mark = np.zeros((M, L), dtype=bool)
    tb = tgrid[-1]
    for j0 in range(0, L, 256):
        thj, thcj = th[j0:j0 + 256, None], thc[j0:j0 + 256, None]
        phi = thj + thcj * th[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            psi = np.where(phi > 0, thj / phi, 0.0)
            psic = np.where(phi > 0, thcj * th[None, :] / phi, 1.0)
        b = np.clip(np.floor(xmap(psi, psic)).astype(np.int64) - (s - 1) // 2, 0, L - s)
        sv = phi * t
        m = np.clip(np.searchsorted(tgrid, sv, side="right") - 1, 0, M - 1)
        inside = sv > tb
        for k in range(s):
            mark[m, b + k] = True
            mm1 = np.where(inside, m, np.minimum(m + 1, M - 1))
            mark[mm1, b + k] = True
        # row Hermite: slices bracketing theta_j t
        tp = th[j0:j0 + 256] * t
        mr = np.clip(np.searchsorted(tgrid, tp, side="right") - 1, 0, M - 1)
        mark[mr, :] = True
        mark[np.minimum(mr + 1, M - 1), :] = True
    return int(mark.sum())


PEAK_FP64_TFLOPS = 78.6  # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz


def hist_integral_flops(L: int, s: int = 10) -> float:
    """FP64 operations of one history-integral launch: L^2 pairs of (24 s + 110)
    (interpolation 24 s + 32, f' and f'' about 42, the nine sums about 36)."""
    return float(L) * L * (24 * s + 110)


def hist_integral_bytes(L: int, slices: float, fp32: bool = False) -> float:
    """Bytes of one history-integral launch counting `slices` full slices of the
    history (C, R, dC/dt, dR/dt: 32 bytes per point in FP64, 16 in FP32) once,
    the stage slice and the output (2 doubles each per grid point) and theta,
    1-theta, nu.  With every stored slice this is an upper bound: a launch reads
    only the points its stencils touch (touched_points)."""
    return slices * L * (16.0 if fp32 else 32.0) + L * (16.0 + 16.0 + 24.0)


def cpu_baseline(L: int, M: int, evals_per_step: float, budget_s: float = 20.0):
    """The oracle's right-hand side on a synthetic history of the same shape,
    timed over the rows of up to one RK step's evaluations (about 10-20 s of
    host work at L = 4096) and scaled to one RK step."""
    import numpy as np

    import oracle

    ts = oracle.ThetaSetup(L, 1e7)
    m = oracle.make_model({3: 0.5, 4: 0.5}, T=0.55)
    rng = np.random.default_rng(20260406)
    times = np.concatenate([[0.0], np.geomspace(1e-2, 3000.0, M - 1)])
    k = 0.5 + 0.2 * rng.random()
    C = np.exp(-k * np.outer(times, ts.thc))
    R = np.exp(-1.3 * k * np.outer(times, ts.thc))
    dC = -k * ts.thc * C
    dR = -1.3 * k * ts.thc * R
    t = 3000.0 * 1.0005
    yC = np.exp(-k * t * ts.thc)
    yR = np.exp(-1.3 * k * t * ts.thc)
    threads = oracle.num_threads()
    done, elapsed, nrows = 0, 0.0, 16
    target = int(round(evals_per_step * L))
    order = np.tile(rng.permutation(L), int(np.ceil(evals_per_step)) + 1)
    while done < target and elapsed < budget_s:
        rows = order[done:min(done + nrows, target)]
        t0 = time.perf_counter()
        oracle.theta_rhs(m, ts, times, C, R, dC, dR, M, t, yC, yR, rows=rows)
        elapsed += time.perf_counter() - t0
        done += rows.size
        nrows = min(nrows * 2, L)
        log(f"cpu baseline: {done} rows in {elapsed:.1f} s")
    per_eval = elapsed / done * L
    return {"value": 1.0 / (per_eval * evals_per_step), "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} rows ({done / L:.2f} right-hand-side evaluations) at L={L}, M={M} "
                      f"(synthetic smooth history), {elapsed:.1f} s, scaled to {evals_per_step:.2f} evaluations per step; "
                      f"the oracle as written, whose t-bracket search walks the stored slices one by one "
                      f"(O(L^2 M) per evaluation)"}


def sweep_requests(pk, n: int, seed: int, precision: int, tmax_range=(10.0, 100.0)):
    """Parameter-sweep requests: T ~ U[0.4, 1.2], (a2^2, a3^2, a4^2) ~ Dirichlet(1,1,1),
    t_max log-uniform on tmax_range, L uniform on {512, 1024, 2048, 4096}, history cap L."""
    import numpy as np
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n):
        a2 = rng.dirichlet([1.0, 1.0, 1.0])
        L = int(rng.choice([512, 1024, 2048, 4096]))
        tmax = float(np.exp(rng.uniform(np.log(tmax_range[0]), np.log(tmax_range[1]))))
        reqs.append(pk.make_params({2: a2[0], 3: a2[1], 4: a2[2]}, float(rng.uniform(0.4, 1.2)), t_max=tmax, L=L,
                                   M_cap=L, eps=1e-6, dt0=1e-3, dt_min=1e-12, precision=precision))
    return reqs


def serving_sweep(pk, n: int = 24, seed: int = 20260406):
    """Solves/s and time-to-solution of the serving pool (FP32-comp histories) on a
    scaled sweep, next to the same requests solved one after another in FP64."""
    import numpy as np
    import torch

    out = {}
    # (a) the same requests as plain FP64 solves, one after another
    t0 = time.perf_counter()
    for p in sweep_requests(pk, n, seed, pk.FP64):
        s = pk.Solver(p)
        s.step(float("inf"))
        s.close()
    torch.cuda.synchronize()
    t_seq64 = time.perf_counter() - t0
    out["sequential_fp64_solves_per_s"] = n / t_seq64
    log(f"serving: {n} sequential FP64 solves in {t_seq64:.1f} s")
    reqs = sweep_requests(pk, n, seed, pk.FP32_COMP)
    arena = int(0.5 * torch.cuda.mem_get_info()[0])
    # (b) closed batch: all requests at once -> capacity
    pool = pk.Pool(arena, max_instances=256)
    t0 = time.perf_counter()
    ids = [pool.submit(p) for p in reqs]
    done = 0
    while done < n:
        pool.run(50)
        for rid in pool.poll():
            pool.release(rid)
            done += 1
    t_batch = time.perf_counter() - t0
    cap = n / t_batch
    out["batch_solves_per_s"] = cap
    log(f"serving: closed batch of {n} in {t_batch:.1f} s ({cap:.2f} solves/s)")
    pool.close()
    # (c) Poisson arrivals at 0.8 x capacity: time to solution
    rng = np.random.default_rng(seed + 1)
    arrivals = np.cumsum(rng.exponential(1.0 / (0.8 * cap), n))
    pool = pk.Pool(arena, max_instances=256)
    t0 = time.perf_counter()
    nxt, tts, status = 0, [], []
    t_log = t0
    while len(tts) < n:
        now = time.perf_counter() - t0
        if time.perf_counter() - t_log > 20.0:
            t_log = time.perf_counter()
            log(f"c4 poisson: {len(tts)} of {n} done, {nxt} arrived after {now:.0f} s")
        while nxt < n and arrivals[nxt] <= now:
            pool.submit(reqs[nxt])
            nxt += 1
        st = pool.run(20)
        for rid in pool.poll():
            _, tm = pool.result(rid)
            tts.append(tm.total_s)
            status.append(tm.status)
            pool.release(rid)
        if st.running == 0 and st.queued == 0 and nxt < n:
            time.sleep(max(0.0, min(arrivals[nxt] - (time.perf_counter() - t0), 0.05)))
    t_open = time.perf_counter() - t0
    pool.close()
    tts = np.array(tts)
    out.update({
        "poisson_solves_per_s": n / t_open,
        "arrival_rate_per_s": 0.8 * cap,
        "p50_time_to_solution_s": float(np.percentile(tts, 50)),
        "p99_time_to_solution_s": float(np.percentile(tts, 99)),
        "all_reached_t_max": bool(all(x == pk.DONE for x in status)),
        "speedup_vs_sequential_fp64": cap / out["sequential_fp64_solves_per_s"],
        "sweep": f"{n} requests: T~U[0.4,1.2], (a2^2,a3^2,a4^2)~Dirichlet(1,1,1), t_max~logU[10,100], "
                 f"L~U{{512,1024,2048,4096}}, history cap L, eps=1e-6, FP32-comp histories, seed {seed}",
    })
    log(f"serving: Poisson run {t_open:.1f} s, p50 {out['p50_time_to_solution_s']:.2f} s, "
        f"p99 {out['p99_time_to_solution_s']:.2f} s")
    return out


def c4_sweep(pk, torch, n: int = 128, tmax_range=(1e2, 1e3), seed: int = 20260406, part: str = "all") -> dict:
    """The serving sweep (C4 shape, scaled in t_max): n requests with T ~ U[0.4, 1.2],
    (a2^2, a3^2, a4^2) ~ Dirichlet(1,1,1), L uniform on {512, 1024, 2048, 4096}, history
    cap L, eps = 1e-6, t_max log-uniform on tmax_range (the stated C4 range [1e2, 1e6]
    is GPU-hours).  (a) FP32-comp: closed batch (all n submitted at once) -> capacity in
    solves/s; then Poisson arrivals at 0.8 x capacity -> p50/p99 time to solution over
    all n.  (b) FP64: closed batch.  (c) The batching gain on the small half
    (L in {512, 1024}): the same requests pooled (closed batch) and one after another
    (one solver each), in FP64 and in FP32-comp."""
    import numpy as np
    out = {"sweep": f"{n} requests: T~U[0.4,1.2], (a2^2,a3^2,a4^2)~Dirichlet(1,1,1), t_max~logU"
                    f"[{tmax_range[0]:g},{tmax_range[1]:g}], L~U{{512,1024,2048,4096}}, history cap L, eps=1e-6, "
                    f"seed {seed}"}
    arena = int(0.6 * torch.cuda.mem_get_info()[0])

    def closed(reqs, label):
        pool = pk.Pool(arena, max_instances=256)
        t0 = time.perf_counter()
        ids = [pool.submit(p) for p in reqs]
        done, status, svc, tts = 0, [], [], []
        t_log = t0
        while done < len(reqs):
            pool.run(50)
            if time.perf_counter() - t_log > 20.0:
                t_log = time.perf_counter()
                log(f"c4 {label}: {done} of {len(reqs)} done after {t_log - t0:.0f} s")
            for rid in pool.poll():
                _, tm = pool.result(rid)
                status.append(tm.status)
                svc.append(tm.service_s)
                tts.append(tm.total_s)
                pool.release(rid)
                done += 1
        wall = time.perf_counter() - t0
        ticks = pool.run(0).ticks
        pool.close()
        log(f"c4 {label}: closed batch of {len(reqs)} in {wall:.1f} s ({len(reqs) / wall:.2f} solves/s, {ticks} ticks)")
        return {"solves": len(reqs), "wall_s": wall, "solves_per_s": len(reqs) / wall, "ticks": int(ticks),
                "all_reached_t_max": bool(all(x == pk.DONE for x in status)),
                "p50_service_s": float(np.percentile(svc, 50)), "p99_service_s": float(np.percentile(svc, 99))}

    def sequential(reqs, label):
        t0 = time.perf_counter()
        status = []
        for p in reqs:
            s = pk.Solver(p)
            try:
                st, _ = s.step(float("inf"))
            except pk.DmfeError as e:
                st = e.status
            status.append(st)
            s.close()
            if len(status) % 16 == 0:
                log(f"c4 {label}: {len(status)} of {len(reqs)} solved after {time.perf_counter() - t0:.0f} s")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        log(f"c4 {label}: {len(reqs)} sequential solves in {wall:.1f} s ({len(reqs) / wall:.2f} solves/s)")
        return {"solves": len(reqs), "wall_s": wall, "solves_per_s": len(reqs) / wall,
                "all_reached_t_max": bool(all(x == pk.DONE for x in status))}

    r32 = sweep_requests(pk, n, seed, pk.FP32_COMP, tmax_range)
    r64 = sweep_requests(pk, n, seed, pk.FP64, tmax_range)
    out["part"] = part
    if part in ("all", "fp32"):
        out.update(_c4_fp32(pk, torch, closed, r32, n, seed, arena))
    if part in ("all", "fp64"):
        out["fp64_closed"] = closed(r64, "fp64")
        small = [k for k, p in enumerate(r64) if p.L <= 1024]
        for name, reqs in (("fp64", r64), ("fp32c", r32)):
            sub = [reqs[k] for k in small]
            pooled = closed(sub, f"{name} small half pooled")
            seq = sequential(sub, f"{name} small half sequential")
            out[f"{name}_small_half"] = {"L": [512, 1024], "pooled": pooled, "sequential": seq,
                                         "batching_gain": pooled["solves_per_s"] / seq["solves_per_s"]}
    return out


def pool_ticks(pk, torch, Ls=(512, 1024), ns=(1, 4, 16, 64, 128), ticks: int = 300, solo: bool = True) -> dict:
    """Cost of one serving tick against the number of admitted solves (FP64, 2+3+4 model,
    a_p^2 = 0.3, 0.4, 0.3, T = 0.8, history cap L, eps = 1e-6): wall time per tick (one RK
    stage evaluation of every solve: the batched launches, the descriptor upload, one
    synchronisation and the host controller) and per stage evaluation (counted from the
    solves' own counters), after 120 untimed ticks; beside it
    one solve stepped alone (wall and kernel time per stage, from the library's HIP
    events).  Under rocprofv3 --kernel-trace, a run restricted to one L and one count
    (which skips the solve alone) gives the GPU time per tick; the rest of the wall time
    is the host's."""
    out = {"ticks": ticks, "rows": []}
    for L in Ls:
        p = pk.make_params({2: 0.3, 3: 0.4, 4: 0.3}, 0.8, t_max=1e6, L=L, M_cap=L, eps=1e-6, dt0=1e-3, dt_min=1e-12)
        if not solo:
            solo_row = {"L": L, "solo_wall_us_per_stage": None, "solo_kernel_us_per_stage": None}
        else:
            solo_row = _solo_stage_cost(pk, torch, p)
            log(f"pool ticks L={L}: one solve alone {solo_row['solo_wall_us_per_stage']:.1f} us per stage")
        for n in ns:
            pool = pk.Pool(n * pk.dmfe_footprint(p) + (1 << 20), max_instances=max(n, 1))
            ids = [pool.submit(p) for _ in range(n)]
            pool.run(120)
            ev0 = sum(int(pool.result(r)[0].rhs_evals) for r in ids)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = pool.run(ticks)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            evals = sum(int(pool.result(r)[0].rhs_evals) for r in ids) - ev0
            pool.close()
            row = {**solo_row, "instances": n, "us_per_tick": wall / ticks * 1e6, "stage_evals": evals,
                   "us_per_stage_eval": wall / evals * 1e6, "running_at_end": int(st.running)}
            if solo:
                row["pooled_vs_alone_per_stage"] = solo_row["solo_wall_us_per_stage"] / row["us_per_stage_eval"]
            out["rows"].append(row)
            log(f"pool ticks L={L} n={n}: {row['us_per_tick']:.1f} us per tick, {row['us_per_stage_eval']:.2f} us "
                f"per stage evaluation")
    return out


def _solo_stage_cost(pk, torch, p) -> dict:
    """Wall and kernel time per RK stage of one solve stepped alone (100 steps after 100)."""
    s = pk.Solver(p)
    s.step(float("inf"), 100)
    s.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(float("inf"), 100)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k = {name: s.timing_read(kid) for name, kid in (("hist_integral", pk.K_HIST_INTEGRAL),
                                                   ("stage_prep", pk.K_STAGE_PREP), ("rk", pk.K_RK))}
    evals = int(k["hist_integral"][0])
    s.close()
    return {"L": p.L, "solo_wall_us_per_stage": wall / evals * 1e6,
            "solo_kernel_us_per_stage": {n: v[1] / max(v[0], 1) * 1e3 for n, v in k.items()}}


def _c4_fp32(pk, torch, closed, r32, n, seed, arena):
    """FP32-comp closed batch, then Poisson arrivals at 0.8 x its capacity."""
    import numpy as np
    out = {}
    out["fp32c_closed"] = closed(r32, "fp32c")
    cap = out["fp32c_closed"]["solves_per_s"]
    rng = np.random.default_rng(seed + 1)
    arrivals = np.cumsum(rng.exponential(1.0 / (0.8 * cap), n))
    pool = pk.Pool(arena, max_instances=256)
    t0 = time.perf_counter()
    nxt, tts, status = 0, [], []
    t_log = t0
    while len(tts) < n:
        now = time.perf_counter() - t0
        if time.perf_counter() - t_log > 20.0:
            t_log = time.perf_counter()
            log(f"c4 poisson: {len(tts)} of {n} done, {nxt} arrived after {now:.0f} s")
        while nxt < n and arrivals[nxt] <= now:
            pool.submit(r32[nxt])
            nxt += 1
        st = pool.run(20)
        for rid in pool.poll():
            _, tm = pool.result(rid)
            tts.append(tm.total_s)
            status.append(tm.status)
            pool.release(rid)
        if st.running == 0 and st.queued == 0 and nxt < n:
            time.sleep(max(0.0, min(arrivals[nxt] - (time.perf_counter() - t0), 0.05)))
    wall = time.perf_counter() - t0
    pool.close()
    tts = np.array(tts)
    out["fp32c_poisson"] = {"arrival_rate_per_s": 0.8 * cap, "solves_per_s": n / wall, "wall_s": wall,
                            "p50_time_to_solution_s": float(np.percentile(tts, 50)),
                            "p99_time_to_solution_s": float(np.percentile(tts, 99)),
                            "max_time_to_solution_s": float(tts.max()),
                            "all_reached_t_max": bool(all(x == pk.DONE for x in status))}
    log(f"c4 poisson: {n / wall:.2f} solves/s, p50 {out['fp32c_poisson']['p50_time_to_solution_s']:.2f} s, "
        f"p99 {out['fp32c_poisson']['p99_time_to_solution_s']:.2f} s")
    return out


def kernel_bench(pk, args) -> dict:
    """The history-integral kernel alone at the workload's full size: a seeded
    smooth synthetic history of M slices at geometrically spaced times up to
    t = 200 and a stage at t = 200.08, the time and step of the solver's own
    steady state on this workload (the shared input generator of the tests),
    one right-hand-side evaluation per step.  A plain device copy of known size runs beside it, so hardware
    byte counters of the kernel can be calibrated against the copy."""
    import numpy as np
    import torch

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import inputs

    prec = pk.FP64 if args.precision == "fp64" else pk.FP32_COMP
    L, M = 4096, args.kernel_slices
    params = pk.make_params({3: 0.5, 4: 0.5}, 0.55, t_max=1e7, L=L, M_cap=M, eps=1e-8, dt0=1e-3, dt_min=1e-12,
                            precision=prec)
    s = pk.Solver(params)
    th = s.read(pk.F_THETA)
    t_last, t = 200.0, 200.08
    times = inputs.geometric_times(M, t_last, t_first=0.01)
    C, R, dC, dR = inputs.smooth_history(th, times, 1)
    s.set_history(times, C, R, dC, dR)
    del C, R, dC, dR
    yC, yR = inputs.smooth_stage(th, t, 1)
    yC, yR = torch.tensor(yC, device="cuda"), torch.tensor(yR, device="cuda")
    for _ in range(args.warmup):
        s.rhs(t, yC, yR, M)
    s.timing(True)
    for _ in range(args.steps):
        s.rhs(t, yC, yR, M)
    torch.cuda.synchronize()
    n, ms, slices = s.timing_read(pk.K_HIST_INTEGRAL)
    s.timing(False)
    s.close()
    cal = calibration_copies(torch)
    avg_us = ms / n * 1e3
    alg = hist_integral_bytes(L, slices / n, fp32=prec == pk.FP32_COMP)
    return {"kernel": "hist_integral", "L": L, "M": M, "precision": args.precision, "launches": n,
            "avg_launch_us": avg_us, "algorithmic_bytes_per_launch": alg,
            "achieved_GBps": alg / (avg_us * 1e-6) / 1e9, "calibration_copies": cal}


def sparsify_bench(pk, torch, L: int = 4096, M: int = 4096, reps: int = 10) -> dict:
    """The sparsification residual kernel (Sec. 3.6) alone: one pass over a full
    history of M slices at L = 4096 (the workload's capacity): seeded uniform
    random values at geometrically spaced times, whose residuals are far above
    the tiny tolerance used, so no slice is removed and every pass sees the
    same M - 12 candidates (the kernel's cost does not depend on the values).
    Algorithmic bytes: the four FP64 (or FP32) fields of every stored point
    read once."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import inputs
    out = {}
    for name, prec in (("fp64", pk.FP64), ("fp32c", pk.FP32_COMP)):
        s = pk.Solver(pk.make_params({3: 0.5, 4: 0.5}, 0.55, t_max=1e7, L=L, M_cap=M, eps=1e-300, dt0=1e-3,
                                     dt_min=1e-310, precision=prec))
        th = s.read(pk.F_THETA)
        times = inputs.geometric_times(M, 200.0, t_first=0.01)
        rng = np.random.default_rng(20260406)
        C, R = rng.uniform(0.0, 1.0, (2, M, L))
        dC, dR = rng.uniform(-1.0, 1.0, (2, M, L))
        s.set_history(times, C, R, dC, dR)
        del C, R, dC, dR
        s.sparsify(1)
        s.timing(True)
        for _ in range(reps):
            assert s.sparsify(1) == 0
        torch.cuda.synchronize()
        n, ms, _ = s.timing_read(pk.K_SPARSIFY)
        s.timing(False)
        s.close()
        us = ms / n * 1e3
        alg = M * L * (32.0 if prec == pk.FP64 else 16.0)
        out[name] = {"avg_pass_us": us, "algorithmic_bytes_per_pass": alg, "achieved_GBps": alg / (us * 1e-6) / 1e9,
                     "frac_of_hbm_peak": alg / (us * 1e-6) / 1e9 / PEAK_HBM_GBS, "passes": n}
        log(f"sparsify {name}: {us:.1f} us per pass at L={L}, M={M}: {alg / (us * 1e-6) / 1e9:.0f} GB/s algorithmic")
    return {"kernel": "sparsify_residual", "L": L, "M": M, **out}


STENCILS = [  # (name, theta_interp, s, fh_d, log_r)
    ("index-lagrange s=10 (default)", 0, 10, 0, False),
    ("theta-lagrange s=10", 1, 10, 0, False),
    ("index-fh s=10 d=5", 2, 10, 5, False),
    ("theta-fh s=10 d=5", 3, 10, 5, False),
    ("theta-fh s=14 d=9", 3, 14, 9, False),
    ("index-lagrange s=10 log-R", 0, 10, 0, True),
]


def stencil_sweep(pk, torch, args) -> dict:
    """Cost against accuracy of the theta-stencils (Sec. 3.3) and the log-R option.
    Cost: the history-integral kernel's average launch at the L = 4096 steady
    state (M = 2500 slices to t = 200, stage at t = 200.08; HIP events).
    Accuracy: the largest error of one right-hand side along fixed theta against
    the exact p = 2 solution at T = 0 (history and stage from its closed form, 800
    slices to t = 8, L = 96 and 192), and end to end the largest energy error of
    the p = 2 quench to T = 0 solved to t = 8 (L = 128, eps = 1e-9)."""
    import numpy as np

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import inputs
    import p2_exact as px

    rows = []
    for name, interp, s_, d, lr in STENCILS:
        L, M, t_last, t = 4096, 2500, 200.0, 200.08
        params = pk.make_params({3: 0.5, 4: 0.5}, 0.55, t_max=1e7, L=L, M_cap=M, eps=1e-8, s=s_,
                                theta_interp=interp, fh_d=d, log_r=lr)
        sv = pk.Solver(params)
        th = sv.read(pk.F_THETA)
        times = inputs.geometric_times(M, t_last, t_first=0.01)
        C, R, dC, dR = inputs.smooth_history(th, times, 1)
        sv.set_history(times, C, R, dC, dR)
        del C, R, dC, dR
        yC, yR = inputs.smooth_stage(th, t, 1)
        yC, yR = torch.tensor(yC, device="cuda"), torch.tensor(yR, device="cuda")
        for _ in range(3):
            sv.rhs(t, yC, yR, M)
        sv.timing(True)
        for _ in range(10):
            sv.rhs(t, yC, yR, M)
        torch.cuda.synchronize()
        n, ms, _ = sv.timing_read(pk.K_HIST_INTEGRAL)
        sv.close()
        errs = []
        for Lp in (96, 192):
            tp = 8.0
            sp = pk.Solver(pk.make_params({2: 1.0}, 0.0, t_max=1e3, L=Lp, M_cap=820, s=s_, theta_interp=interp,
                                          fh_d=d, log_r=lr))
            thp = sp.read(pk.F_THETA)
            tt = np.concatenate([[0.0], np.geomspace(1e-3, tp - 0.0125, 799)])
            Cp = np.array([px.C0(x, thp * x) for x in tt])
            Rp = np.array([px.R0(x, thp * x) for x in tt])
            dCp = np.array([sum(a * w for a, w in zip(px.dC0(x, thp * x), (1, thp))) for x in tt])
            dRp = np.array([sum(a * w for a, w in zip(px.dR0(x, thp * x), (1, thp))) for x in tt])
            Cp[:, -1] = Rp[:, -1] = 1.0
            sp.set_history(tt, Cp, Rp, dCp, dRp)
            ysC, ysR = px.C0(tp, thp * tp), px.R0(tp, thp * tp)
            ysC[-1] = ysR[-1] = 1.0
            gC, gR, _, _ = sp.rhs(tp, torch.tensor(ysC, device="cuda"), torch.tensor(ysR, device="cuda"), tt.size)
            sp.close()
            a, b = px.dC0(tp, thp * tp)
            exC = a + thp * b
            a, b = px.dR0(tp, thp * tp)
            exR = a + thp * b
            errs.append(float(max(np.abs(gC.cpu().numpy() - exC)[:-1].max(), np.abs(gR.cpu().numpy() - exR)[:-1].max())))
        # end to end: the p = 2 quench to T = 0 solved to t = 8, energy against the closed form
        sp = pk.Solver(pk.make_params({2: 1.0}, 0.0, t_max=1e3, L=128, M_cap=4096, eps=1e-9, dt0=1e-3,
                                      dt_min=1e-12, s=s_, theta_interp=interp, fh_d=d, log_r=lr))
        sp.step(8.0)
        tt, E = sp.read(pk.F_T_GRID), sp.read(pk.F_ENERGY)
        sp.close()
        e2e = float(np.abs(E - px.E0(tt)).max())
        rows.append({"scheme": name, "hist_integral_avg_launch_us": ms / n * 1e3, "p2_rhs_max_error_L96": errs[0],
                     "p2_rhs_max_error_L192": errs[1], "p2_solve_energy_error_L128": e2e})
        log(f"stencil {name}: {ms / n * 1e3:.1f} us per launch; p=2 RHS error {errs[0]:.2e} (L=96), "
            f"{errs[1]:.2e} (L=192); p=2 solve to t=8, energy error {e2e:.2e} (L=128)")
    base = rows[0]["hist_integral_avg_launch_us"]
    for r in rows:
        r["cost_vs_default"] = r["hist_integral_avg_launch_us"] / base
    return {"stencils": rows}


def uniform_c1(pk, torch, with_oracle: bool) -> dict:
    """The uniform-grid baseline: pure p=3 (f = q^3/2), T = 0.5, h = 0.05, N = 1000
    (t_max = 50), classical RK4 with trapezoid history integrals.  Time to
    solution of the library (4000 stages), and of the oracle on the host."""
    p = pk.make_params({3: 1.0}, 0.5, mode=pk.UNIFORM, h=0.05, N=1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = pk.Solver(p)
    s.step(float("inf"))
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t0
    E = s.read(pk.F_ENERGY)
    s.close()
    out = {"config": "p=3, T=0.5, h=0.05, N=1000, RK4 + trapezoid (uniform grid)", "gpu_s": gpu_s,
           "E_final": float(E[-1])}
    if with_oracle:
        import oracle
        t0 = time.perf_counter()
        _, _, Eo = oracle.uniform_solve(oracle.make_model({3: 1.0}, T=0.5), 0.05, 1000)
        out["oracle_s"] = time.perf_counter() - t0
        out["oracle_threads"] = oracle.num_threads()
        out["max_abs_dE_vs_oracle"] = float(abs(Eo - E).max())
    log(f"C1 uniform: GPU {gpu_s:.2f} s" + (f", oracle {out['oracle_s']:.2f} s" if with_oracle else ""))
    return out


def adaptive_c2(pk, torch) -> dict:
    """The L = 2048 workload end to end: 3+4 model, T = 0.6, t_max = 1e4, eps = 1e-8,
    FP64, from t = 0 to t_max, with M(t) sampled every 2000 steps.  The history
    capacity is 8192 slices (0.54 GB): at this tolerance the sparsified history
    needs about 2048 slices by t = 1800 and keeps growing."""
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=2048, M_cap=8192, eps=1e-8, dt0=1e-3, dt_min=1e-12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = pk.Solver(p)
    trace = []
    while True:
        st, info = s.step(float("inf"), 2000)
        trace.append([int(info.accepted + info.rejected), float(info.t), int(info.M), round(time.perf_counter() - t0, 2)])
        log(f"C2: steps={trace[-1][0]} t={info.t:.5g} M={info.M} dt={info.dt:.3g} scheme={info.scheme}")
        if st == pk.DONE:
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    E = s.read(pk.F_ENERGY)
    s.close()
    steps = info.accepted + info.rejected
    return {"config": "3+4, T=0.6, t_max=1e4, L=2048, history cap 8192, eps=1e-8, FP64", "wall_s": wall,
            "steps": int(steps), "accepted": int(info.accepted), "rejected": int(info.rejected),
            "steps_per_s": steps / wall, "rhs_evals": int(info.rhs_evals), "sparsify_calls": int(info.sparsify_calls),
            "removed": int(info.removed), "M_final": int(info.M), "t_final": info.t, "scheme_final": int(info.scheme),
            "E_final": float(E[-1]), "trace_steps_t_M_wall": trace}


def large_grid_c5(pk, torch, M: int = 3000, ticks: int = 60) -> dict:
    """The large-grid stress configuration with a long history: 16 identical solves
    of the 2+4 model (a2^2 = 0.3, a4^2 = 0.7, T = 0.45, t_max = 1e7) on an 8192-point
    grid, history cap 8192, admitted together into one pool and each resumed from
    the same seeded smooth history of M slices (geometric times up to t = 1000)
    through dmfe_pool_set_history; then `ticks` batched ticks (one RK stage of
    every solve per tick) are timed between device synchronisations.  The same
    solve alone on the same history, timed over the same stages, gives the
    one-instance rate.  Algorithmic bytes per stage: the history points one
    evaluation touches (touched_points) plus the stage slice, the output and the
    grid arrays.  FP64 and FP32-comp."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import inputs
    L = 8192
    out = {"config": f"16 x (2+4 model a2^2=0.3, a4^2=0.7, T=0.45, t_max=1e7), L={L}, history cap 8192, eps=1e-8, "
                     f"each resumed from a {M}-slice smooth synthetic history (t up to 1000), one pool, batched ticks"}
    times = inputs.geometric_times(M, 1000.0, t_first=0.01)
    hist = None
    for name, prec in (("fp64", pk.FP64), ("fp32c", pk.FP32_COMP)):
        p = pk.make_params({2: 0.3, 4: 0.7}, 0.45, t_max=1e7, L=L, M_cap=8192, eps=1e-8, dt0=1e-3, dt_min=1e-12,
                           precision=prec)
        sv = pk.Solver(p)
        th, thc = sv.read(pk.F_THETA), sv.read(pk.F_THETA_C)
        if hist is None:
            hist = inputs.smooth_history(th, times, 5)
            touched = touched_points(th, thc, times, times[-1] + 0.05, _gamma_of(1e7))
        # one instance alone on the history: stage evaluations per second over 10 steps
        sv.set_history(times, *hist, dt=0.1)
        sv.step(float("inf"), 2)
        sv.timing(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, i1 = sv.step(float("inf"), 10)
        torch.cuda.synchronize()
        solo_wall = time.perf_counter() - t1
        nh, msh, _ = sv.timing_read(pk.K_HIST_INTEGRAL)
        solo_evals = nh
        sv.close()
        pool = pk.Pool(16 * pk.dmfe_footprint(p) + 4096, max_instances=16)
        ids = [pool.submit(p) for _ in range(16)]
        pool.run(0)
        for rid in ids:
            pool.set_history(rid, times, *hist, dt=0.1)
        pool.run(12)
        torch.cuda.synchronize()
        m0 = pool.result(ids[0])[0].M
        t0 = time.perf_counter()
        st = pool.run(ticks)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        info = pool.result(ids[0])[0]
        assert st.running == 16
        pool.close()
        evals = 16 * ticks
        pb = 32 if prec == pk.FP64 else 16
        alg = touched * pb + L * (16.0 + 16.0 + 24.0)
        out[name] = {"ticks": ticks, "stage_evals": evals, "wall_s": wall, "stage_evals_per_s": evals / wall,
                     "M_window": [int(m0), int(info.M)], "touched_points_per_stage": touched,
                     "algorithmic_bytes_per_stage": alg, "algorithmic_GBps": evals * alg / wall / 1e9,
                     "frac_of_hbm_peak": evals * alg / wall / 1e9 / PEAK_HBM_GBS,
                     "solo_stage_evals_per_s": solo_evals / solo_wall,
                     "solo_hist_integral_avg_launch_us": msh / max(nh, 1) * 1e3,
                     "pooled_vs_solo": (evals / wall) / (solo_evals / solo_wall)}
        log(f"C5 {name}: {evals / wall:.1f} stage-evals/s pooled ({evals} in {wall:.2f} s, M {m0}->{info.M}); "
            f"alone {solo_evals / solo_wall:.1f} (hist_integral {msh / max(nh, 1) * 1e3:.0f} us)")
    return out


def aging_p3(pk, torch, t_end: float = 1e4, eps: float = 1e-10) -> dict:
    """The paper's energy-exponent experiment (Sec. 4.2): pure p=3 (f = q^3/2),
    quench from a random start to T = 0, L = 1024, to t_end at tolerance eps.
    Reports E(t) - E_th at quarter decades of t and the effective exponent between
    them.  A history that outgrows its capacity (DMFE_ERR_CAPACITY) ends the run
    early; the rows reached are reported with the reason."""
    import numpy as np
    cap = 8192 if t_end <= 1e4 else 32768  # the sparsified history grows with t
    p = pk.make_params({3: 1.0}, 0.0, t_max=1e7, L=1024, M_cap=cap, eps=eps, dt0=1e-3, dt_min=1e-14)
    E_th = -np.sqrt(4.0 / 3.0)
    t0 = time.perf_counter()
    s = pk.Solver(p)
    rows, t_next, stopped = [], 1.0, None
    while t_next <= t_end * 1.001:
        try:
            _, info = s.step(t_next)
        except pk.DmfeError as e:
            if e.status != pk.ERR_CAPACITY:
                raise
            info = s.info()
            stopped = f"history capacity {cap} reached at t={info.t:.6g} (M={info.M})"
            log(f"aging: {stopped}")
            break
        E = float(s.read(pk.F_ENERGY)[-1])
        rows.append([info.t, E, E - E_th, int(info.accepted + info.rejected), int(info.M)])
        log(f"aging: t={info.t:.5g} E-E_th={E - E_th:.4e} steps={rows[-1][3]} M={info.M}")
        t_next *= 10 ** 0.25
    s.close()
    t = np.array([r[0] for r in rows])
    d = np.array([r[2] for r in rows])
    alpha = (-np.diff(np.log(d)) / np.diff(np.log(t))).tolist()
    return {"config": f"pure p=3 (f=q^3/2), T=0 after a random start, L=1024, eps={eps:g}, history cap {cap}",
            "E_th": E_th, "wall_s": time.perf_counter() - t0, "rows_t_E_dE_steps_M": rows,
            "alpha_eff_between_rows": alpha, "stopped": stopped}


def _hermite_at(t, tg, Y, dY):
    """Cubic Hermite in t through the stored slices (values Y[n], derivatives dY[n] along
    fixed theta) at time t, node by node: the solver's own interpolation in t."""
    import numpy as np
    n = int(np.searchsorted(tg, t, side="right") - 1)
    n = min(max(n, 0), tg.size - 2)
    h = tg[n + 1] - tg[n]
    u = (t - tg[n]) / h
    h00, h10, h01, h11 = 2 * u**3 - 3 * u**2 + 1, (u**3 - 2 * u**2 + u) * h, -2 * u**3 + 3 * u**2, (u**3 - u**2) * h
    return h00 * Y[n] + h10 * dY[n] + h01 * Y[n + 1] + h11 * dY[n + 1]


def c3_fp32_error(pk, torch, t_end: float = 1000.0) -> dict:
    """Error of the FP32-compensated history against FP64 on the L = 4096 workload
    (3+4 model, T = 0.55, t_max = 1e7, history cap 4096, eps = 1e-8): both solves run
    from t = 0 to t_end through several automatic sparsification passes.  Per
    observable, over the common t range: E(t) and mu(t) of the stored slices (the
    FP32 run's values interpolated to the FP64 run's slice times by a cubic
    spline); C and R along fixed theta, and C(t, t_w) for t_w = 10, 100, at common
    times t = t_end/4, t_end/2 and the last common time (each run's stored slices
    Hermite-interpolated in t, then linearly in theta for C(t, t_w))."""
    import numpy as np
    from scipy.interpolate import CubicSpline
    runs = {}
    for name, prec in (("fp64", pk.FP64), ("fp32c", pk.FP32_COMP)):
        s = pk.Solver(workload_params(pk, prec))
        t0 = time.perf_counter()
        _, info = s.step(t_end)
        wall = time.perf_counter() - t0
        tg = s.read(pk.F_T_GRID)
        runs[name] = {"t": tg, "E": s.read(pk.F_ENERGY), "mu": s.read(pk.F_MU), "C": s.read(pk.F_C),
                      "R": s.read(pk.F_R), "dC": s.read(pk.F_DC), "dR": s.read(pk.F_DR), "th": s.read(pk.F_THETA),
                      "steps": int(info.accepted + info.rejected), "M": int(info.M), "wall_s": wall,
                      "sparsify_calls": int(info.sparsify_calls), "nb": int(info.nb_valid)}
        s.close()
        log(f"c3 error: {name} to t={tg[-1]:.5g} in {info.accepted + info.rejected} steps, M={info.M}, "
            f"{info.sparsify_calls} sparsification passes, {wall:.1f} s")
    a, b = runs["fp64"], runs["fp32c"]
    th = a["th"]
    t_hi = min(a["t"][a["nb"] - 1], b["t"][b["nb"] - 1])
    sel = (a["t"] >= 1.0) & (a["t"] <= t_hi)
    out = {"t_end": t_end, "fp64": {k: a[k] for k in ("steps", "M", "wall_s", "sparsify_calls")},
           "fp32c": {k: b[k] for k in ("steps", "M", "wall_s", "sparsify_calls")}}
    for obs in ("E", "mu"):
        spl = CubicSpline(b["t"], b[obs])
        d = np.abs(spl(a["t"][sel]) - a[obs][sel])
        out[f"max_abs_d{obs}"] = float(d.max())
        out[f"max_abs_d{obs}_t"] = float(a["t"][sel][int(d.argmax())])
    per_t = []
    for tc in (t_end / 4, t_end / 2, t_hi):
        Ca = _hermite_at(tc, a["t"][:a["nb"]], a["C"], a["dC"])
        Cb = _hermite_at(tc, b["t"][:b["nb"]], b["C"], b["dC"])
        Ra = _hermite_at(tc, a["t"][:a["nb"]], a["R"], a["dR"])
        Rb = _hermite_at(tc, b["t"][:b["nb"]], b["R"], b["dR"])
        row = {"t": float(tc), "max_abs_dC_along_theta": float(np.abs(Ca - Cb).max()),
               "max_abs_dR_along_theta": float(np.abs(Ra - Rb).max())}
        for tw in (10.0, 100.0):
            if tw < tc:
                ca, cb = np.interp(tw / tc, th, Ca), np.interp(tw / tc, th, Cb)
                row[f"C(t,{tw:g})_fp64"] = float(ca)
                row[f"abs_dC(t,{tw:g})"] = float(abs(ca - cb))
        per_t.append(row)
    out["fields"] = per_t
    log(f"c3 error: |dE| {out['max_abs_dE']:.2e}, |dmu| {out['max_abs_dmu']:.2e}; fields {per_t}")
    return out


def fdt_chi_vs_c(th, C, R, t):
    """chi(t, theta t) = int_{theta t}^t R(t, s) ds = t int_theta^1 R(t, theta' t) dtheta' on one
    stored slice (trapezoid on the theta grid, summed from theta = 1 down) and C(t, theta t)."""
    import numpy as np
    seg = 0.5 * (R[1:] + R[:-1]) * np.diff(th)
    chi = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]]) * t
    return chi, C


def fdt_slopes(chi, C, q_split: float, fdt_band=(0.85, 0.97), aging_band=(0.15, 0.6)):
    """Least-squares slopes -d chi / d C in the FDT band and the aging band of C, and the C
    where the two fitted lines cross (the break of the chi(C) curve)."""
    import numpy as np
    out = {}
    lines = {}
    for name, (lo, hi) in (("fdt", fdt_band), ("aging", aging_band)):
        sel = (C > lo) & (C < hi)
        if sel.sum() < 4:
            out[name + "_slope"] = None
            continue
        A = np.vstack([C[sel], np.ones(sel.sum())]).T
        (a, b), *_ = np.linalg.lstsq(A, chi[sel], rcond=None)
        out[name + "_slope"] = float(-a)
        lines[name] = (a, b)
    if len(lines) == 2:
        (a1, b1), (a2, b2) = lines["fdt"], lines["aging"]
        out["break_C"] = float((b2 - b1) / (a1 - a2)) if a1 != a2 else None
    return out


def fdt_run(pk, torch, t_points=(100.0, 300.0, 1000.0, 3000.0, 10000.0), L: int = 1024, eps: float = 1e-8,
            cap: int = 16384) -> dict:
    """Fluctuation-dissipation plot of Sec. 4.3 (Fig. RvsC): pure p = 3 with f = q^3
    (a_3^2 = 2 in f = sum a_p^2 q^p / 2), quenched from a random start to T = 1/2,
    solved on the theta grid.  At each t of t_points the newest stored slice gives
    C(t, s) and chi(t, s) = int_s^t R(t, tau) d tau on the theta grid; the slope of
    chi against C is fitted in the FDT band (C in 0.85..0.97, expected 1/T = 2) and in
    the aging band (C in 0.15..0.6, expected to approach x_th = 0.607865), and the
    break of the curve (the crossing of the two lines) is compared with
    q_EA = 0.766911."""
    import numpy as np
    p = pk.make_params({3: 2.0}, 0.5, t_max=1e7, L=L, M_cap=cap, eps=eps, dt0=1e-3, dt_min=1e-14)
    s = pk.Solver(p)
    th = s.read(pk.F_THETA)
    rows = []
    t0 = time.perf_counter()
    for tp in t_points:
        _, info = s.step(tp)
        M = int(info.M)
        C = s.read(pk.F_C, M - 1, 1)[0]
        R = s.read(pk.F_R, M - 1, 1)[0]
        tn = float(s.read(pk.F_T_GRID, M - 1, 1)[0])
        chi, Cc = fdt_chi_vs_c(th, C, R, tn)
        fit = fdt_slopes(chi, Cc, 0.766911)
        rows.append({"t": tn, "M": M, "steps": int(info.accepted + info.rejected), **fit,
                     "wall_s": time.perf_counter() - t0})
        log(f"fdt: t={tn:.5g} M={M} slopes fdt={fit.get('fdt_slope')} aging={fit.get('aging_slope')} "
            f"break C={fit.get('break_C')}")
    s.close()
    return {"config": f"pure p=3, f=q^3 (a3^2=2), T=0.5, random start, L={L}, eps={eps:g}, history cap {cap}",
            "expected": {"fdt_slope": 2.0, "aging_slope_x_th": 0.607865, "q_EA": 0.766911}, "rows": rows}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["fp64", "fp32c"], default="fp64")
    ap.add_argument("--fill-seconds", type=float, default=150.0, help="time budget of the untimed fill phase")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the timed window at the other precision")
    ap.add_argument("--no-configs", action="store_true", help="skip the end-to-end run of the uniform-grid configuration")
    ap.add_argument("--aging", action="store_true",
                    help="also run the energy-exponent experiment (pure p=3 quenched to T=0, to t=1e4, about 50 s)")
    ap.add_argument("--c2", action="store_true",
                    help="also run the L=2048 configuration from t=0 to t_max=1e4 (about 40,000 steps, 75 s)")
    ap.add_argument("--serving", type=int, default=24, help="requests in the serving sweep (0: skip)")
    ap.add_argument("--kernel", action="store_true",
                    help="time the history-integral kernel alone on a synthetic full-size history")
    ap.add_argument("--aging-t-end", type=float, default=1e4, help="end time of --aging")
    ap.add_argument("--aging-eps", type=float, default=1e-10, help="tolerance of --aging")
    ap.add_argument("--c5", action="store_true",
                    help="only the large-grid configuration: 16 solves at L=8192 in one pool")
    ap.add_argument("--stencils", action="store_true",
                    help="only the cost and accuracy of the theta-stencil schemes and the log-R option")
    ap.add_argument("--c4", type=int, default=0,
                    help="only the serving sweep with this many requests (pooled and one-by-one, both precisions)")
    ap.add_argument("--c4-tmax", type=float, nargs=2, default=(1e2, 1e3), help="t_max range of --c4")
    ap.add_argument("--c4-part", choices=["all", "fp32", "fp64"], default="all",
                    help="--c4: fp32 = FP32-comp closed batch and Poisson arrivals; fp64 = FP64 closed batch and "
                         "the pooled-against-sequential comparison on L in {512, 1024}")
    ap.add_argument("--c3-error", type=float, default=0.0,
                    help="only the FP32-comp error against FP64 on the L=4096 workload, both solved to this t")
    ap.add_argument("--fdt", action="store_true",
                    help="only the fluctuation-dissipation plot of pure p=3 at T=1/2 (chi against C) to t=1e4")
    ap.add_argument("--no-sparsify", action="store_true", help="skip the sparsification kernel's roofline line")
    ap.add_argument("--pool-ticks", action="store_true",
                    help="serving tick cost against the number of admitted solves (FP64, L=512 and 1024)")
    ap.add_argument("--pool-L", type=int, default=0, help="restrict --pool-ticks to one grid length")
    ap.add_argument("--pool-n", type=int, default=0, help="restrict --pool-ticks to one number of solves")
    ap.add_argument("--no-ssprk-window", action="store_true",
                    help="skip the SSPRK(10,4) window at the value window's end state")
    ap.add_argument("--no-long-window", action="store_true",
                    help="skip the long window and the SSPRK(10,4) window (for profiled runs: the value "
                         "window is then the last "
                         "launches of the history-integral kernel)")
    ap.add_argument("--sparsify", action="store_true",
                    help="only the sparsification residual kernel at L=4096, M=4096 (one pass, nothing removed)")
    ap.add_argument("--kernel-slices", type=int, default=2500,
                    help="history slices of --kernel (the solver's steady state holds about 2500)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver has no multi-GPU path; "
              f"independent solves shard trivially across GPUs and are not benchmarked here.", file=sys.stderr)
        return 2

    import torch

    import paper_2604_06309_amd as pk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.kernel:
        print(json.dumps(kernel_bench(pk, args)), flush=True)
        return 0
    if args.stencils:
        print(json.dumps(stencil_sweep(pk, torch, args)), flush=True)
        return 0
    if args.c5:
        print(json.dumps(large_grid_c5(pk, torch)), flush=True)
        return 0
    if args.sparsify:
        print(json.dumps(sparsify_bench(pk, torch)), flush=True)
        return 0
    if args.fdt:
        print(json.dumps(fdt_run(pk, torch)), flush=True)
        return 0
    if args.pool_ticks:
        Ls = (args.pool_L,) if args.pool_L else (512, 1024)
        ns = (args.pool_n,) if args.pool_n else (1, 4, 16, 64, 128)
        print(json.dumps(pool_ticks(pk, torch, Ls, ns, solo=not args.pool_n)), flush=True)
        return 0
    if args.c4 > 0:
        print(json.dumps(c4_sweep(pk, torch, args.c4, tuple(args.c4_tmax), part=args.c4_part)), flush=True)
        return 0
    if args.c3_error > 0:
        print(json.dumps(c3_fp32_error(pk, torch, args.c3_error)), flush=True)
        return 0
    prec_name = args.precision
    other = "fp32c" if prec_name == "fp64" else "fp64"
    w = timed_window(pk, torch, prec_name, args)
    L = w["L"]
    out = {
        "metric": METRIC,
        "value": w["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": w["steps"],
        "warmup": args.warmup,
        "ms_per_step": w["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec_name == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": w["config"],
        "roofline": w["roofline"],
        "long_window": w["long_window"],
        "ssprk_window": w["ssprk_window"],
        "rhs_evals_per_s": w["steps_per_s"] * w["config"]["rhs_evals_per_step"],
    }
    calibration_copies(torch)
    if not args.no_compare:
        o = timed_window(pk, torch, other, args)
        out[other] = {"value": o["steps_per_s"], "unit": "steps/s", "ms_per_step": o["ms_per_step"],
                      "speedup_vs_" + prec_name: o["steps_per_s"] / w["steps_per_s"],
                      "M_window": o["config"]["M_window"], "t_window": o["config"]["t_window"],
                      "rhs_evals_per_step": o["config"]["rhs_evals_per_step"],
                      "hist_integral_avg_launch_us": o["roofline"]["avg_launch_us"],
                      "roofline": o["roofline"], "long_window": o["long_window"], "ssprk_window": o["ssprk_window"]}
        if w["long_window"] and o["long_window"]:
            out[other]["long_window_speedup_vs_" + prec_name] = (o["long_window"]["stage_evals_per_s"] /
                                                                w["long_window"]["stage_evals_per_s"])
    if not args.no_sparsify:
        out["sparsify_roofline"] = sparsify_bench(pk, torch)
    if not args.no_configs:
        out["c1_uniform"] = uniform_c1(pk, torch, with_oracle=not args.no_cpu_baseline)
    if args.c2:
        out["c2_adaptive"] = adaptive_c2(pk, torch)
    if args.aging:
        out["aging_p3"] = aging_p3(pk, torch, args.aging_t_end, args.aging_eps)
    if args.serving > 0:
        out["serving"] = serving_sweep(pk, args.serving)
    if not args.no_cpu_baseline:
        sl = w["config"]["mean_slices_per_stage"]
        out["cpu_baseline"] = cpu_baseline(L, int(round(sl)) if sl > 16 else L,
                                           w["config"]["rhs_evals_per_step"])
    print(json.dumps(out), flush=True)
    return 0


def _kernel_window(pk, torch, s, steps: int = 0, passes: int = 0, max_steps: int = 0, max_s: float = 0.0,
                   kernels=None):
    """Time `steps` RK steps (or, with passes > 0, steps until `passes` more automatic
    sparsification passes have run, within max_steps / max_s) between device
    synchronisations, with the library's per-launch HIP events on the given kernels
    (default: the history-integral kernel alone; each timed launch adds two event
    records to the stream)."""
    i0 = s.info()
    s.timing(True, [pk.K_HIST_INTEGRAL] if kernels is None else kernels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if passes <= 0:
        _, i1 = s.step(float("inf"), steps)
    else:
        i1 = i0
        while (i1.sparsify_calls - i0.sparsify_calls < passes and
               (i1.accepted + i1.rejected) - (i0.accepted + i0.rejected) < max_steps and
               time.perf_counter() - t0 < max_s):
            _, i1 = s.step(float("inf"), 100)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k = {name: s.timing_read(kid) for name, kid in (("hist_integral", pk.K_HIST_INTEGRAL),
                                                   ("sparsify_residual", pk.K_SPARSIFY),
                                                   ("stage_prep", pk.K_STAGE_PREP), ("rk", pk.K_RK))}
    s.timing(False)
    nsteps = (i1.accepted + i1.rejected) - (i0.accepted + i0.rejected)
    return i0, i1, nsteps, elapsed, k


def timed_window(pk, torch, prec_name: str, args) -> dict:
    """Fill, warm up and time one solve of the workload at the given precision.

    (1) Untimed fill from t = 0 until the history has first reached its capacity
    and an automatic sparsification pass has run.  (2) args.warmup steps.
    (3) The value window: exactly args.steps steps.  (4) The long window: the
    steps that follow until three more automatic sparsification passes have run
    (the solver's cycle at its capacity), sparsification time included.  The
    scheme is whatever the controller uses there: Dormand-Prince 5(4) on this
    workload (SSPRK(10,4) takes over only once dt * 4 sqrt(f''(1)) reaches 3.3065,
    dt ~ 0.39, which the history at a 4096-slice capacity does not reach; see the
    design notes)."""
    import numpy as np
    prec = pk.FP64 if prec_name == "fp64" else pk.FP32_COMP
    params = workload_params(pk, prec)
    L = params.L
    s = pk.Solver(params)
    th, thc = s.read(pk.F_THETA), s.read(pk.F_THETA_C)

    t_fill = time.perf_counter()
    filled = False
    while time.perf_counter() - t_fill < args.fill_seconds:
        _, info = s.step(float("inf"), 250)
        log(f"fill ({prec_name}): steps={info.accepted + info.rejected} M={info.M} t={info.t:.5g} "
            f"dt={info.dt:.3g} scheme={info.scheme} sparsify={info.sparsify_calls} "
            f"({time.perf_counter() - t_fill:.1f} s)")
        if info.sparsify_calls >= 1:
            filled = True
            break
    s.step(float("inf"), args.warmup)
    # algorithmic bytes: the history points one launch at the window's start touches
    iw = s.info()
    tgrid = s.read(pk.F_T_GRID)
    gamma = _gamma_of(params.t_max)
    touched = touched_points(th, thc, tgrid, iw.t, gamma)
    i0, i1, steps, elapsed, k = _kernel_window(pk, torch, s, steps=args.steps)
    assert steps == args.steps, (steps, args.steps)
    n_hi, ms_hi, slices_hi = k["hist_integral"]
    evals = i1.rhs_evals - i0.rhs_evals
    avg_ms = ms_hi / n_hi
    avg_slices = slices_hi / n_hi
    fp32 = prec == pk.FP32_COMP
    pb = 16.0 if fp32 else 32.0
    alg_bytes = touched * pb + L * (16.0 + 16.0 + 24.0)
    upper_bytes = hist_integral_bytes(L, avg_slices, fp32=fp32)
    gbps = alg_bytes / (avg_ms * 1e-3) / 1e9
    flops = hist_integral_flops(L)
    tflops = flops / (avg_ms * 1e-3) / 1e12
    # which roof is nearer: the byte floor or the FP64-arithmetic floor of one launch
    t_bytes = alg_bytes / (PEAK_HBM_GBS * 1e9)
    t_flops = flops / (PEAK_FP64_TFLOPS * 1e12)
    alu = t_flops >= t_bytes
    log(f"window ({prec_name}): {steps} steps in {elapsed:.3f} s, hist_integral {avg_ms * 1e3:.1f} us/launch")
    scheme = lambda i: "SSPRK(10,4)" if i.scheme == pk.SCHEME_SSPRK104 else "DP5"
    ssprk = None if (args.no_ssprk_window or args.no_long_window) else _ssprk_window(pk, torch, s, params, prec_name)
    long_window = None
    if not args.no_long_window:
        # the long window: three more sparsification passes
        j0, j1, lsteps, lelapsed, lk = _kernel_window(pk, torch, s, passes=3, max_steps=12000, max_s=90.0,
                                                      kernels=[pk.K_HIST_INTEGRAL, pk.K_SPARSIFY])
        lev = j1.rhs_evals - j0.rhs_evals
        log(f"long window ({prec_name}): {lsteps} steps in {lelapsed:.2f} s, "
            f"{j1.sparsify_calls - j0.sparsify_calls} sparsification passes, t {j0.t:.5g} -> {j1.t:.5g}, "
            f"M {j0.M} -> {j1.M}")
        long_window = {
            "what": "the steps after the value window until three more automatic sparsification passes, "
                    "sparsification included",
            "steps": int(lsteps), "seconds": lelapsed, "steps_per_s": lsteps / lelapsed,
            "stage_evals_per_s": lev / lelapsed, "rhs_evals_per_step": lev / max(lsteps, 1),
            "sparsify_passes": int(j1.sparsify_calls - j0.sparsify_calls),
            "t_window": [j0.t, j1.t], "M_window": [int(j0.M), int(j1.M)], "scheme": scheme(j1),
            "hist_integral_avg_launch_us": lk["hist_integral"][1] / max(lk["hist_integral"][0], 1) * 1e3,
            "sparsify_avg_pass_us": lk["sparsify_residual"][1] / max(lk["sparsify_residual"][0], 1) * 1e3,
            "kernel_s": {name: lk[name][1] * 1e-3 for name in ("hist_integral", "sparsify_residual")},
            "ssprk_regime": "not reached: at this capacity the run stays under DP5 (dt ~ 0.31 at t ~ 8000, "
                            "where the 4096-slice history fills up and a pass frees nothing)",
        }
    s.close()
    return {
        "L": L,
        "steps": steps,
        "steps_per_s": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "config": {
            "workload": "mixed spherical 3+4 (a3^2=a4^2=1/2), T=0.55, t_max=1e7, theta grid L=4096, "
                        "history cap 4096, eps=1e-8, DP5 then SSPRK(10,4), automatic sparsification",
            "precision": prec_name,
            "L": L,
            "M_cap": params.M_cap,
            "regime": (f"{scheme(i1)} steps with the history at its capacity (filled from t=0 until the first "
                       f"sparsification pass)" if filled else "fill budget ran out before the first sparsification"),
            "M_window": [int(i0.M), int(i1.M)],
            "mean_slices_per_stage": avg_slices,
            "t_window": [i0.t, i1.t],
            "dt_end": i1.dt,
            "scheme_end": scheme(i1),
            "rhs_evals_per_step": evals / steps,
            "sparsify_passes_in_window": int(i1.sparsify_calls - i0.sparsify_calls),
            "hist_integral_ms_per_step": k["hist_integral"][1] / steps,
            "timed_kernels": "HIP events on the history-integral kernel only (events on every kernel cost ~5% of a step)",
        },
        "long_window": long_window,
        "ssprk_window": ssprk,
        "roofline": {
            "kernel": "hist_integral",
            "bound": "alu" if alu else "hbm",
            "achieved": tflops if alu else gbps,
            "peak": PEAK_FP64_TFLOPS if alu else PEAK_HBM_GBS,
            "unit": "TFLOP/s" if alu else "GB/s",
            "frac": tflops / PEAK_FP64_TFLOPS if alu else gbps / PEAK_HBM_GBS,
            "traffic": traffic_record(L, prec_name),
            "avg_launch_us": avg_ms * 1e3,
            "launches": n_hi,
            "algorithmic_bytes_per_launch": alg_bytes,
            "touched_points_per_launch": touched,
            "stored_points": int(iw.M) * L,
            "hbm": {"achieved_GBps": gbps, "peak": PEAK_HBM_GBS, "frac": gbps / PEAK_HBM_GBS,
                    "floor_us": t_bytes * 1e6,
                    "upper_bound_bytes_all_stored_points": upper_bytes},
            "fp64_alu": {"flops_per_launch": flops, "achieved_TFLOPs": tflops, "peak": PEAK_FP64_TFLOPS,
                         "frac": tflops / PEAK_FP64_TFLOPS, "floor_us": t_flops * 1e6},
        },
    }


def _ssprk_window(pk, torch, s, params, prec_name: str, steps: int = 100, warm: int = 10) -> dict:
    """SSPRK(10,4) steps at the workload's own state: the history, state and step of the
    solve just timed are loaded into a second solve of the same parameters with the
    scheme set to SSPRK(10,4) (the scheme of the long-time regime, which the run
    switches to once dt reaches DP5's stability boundary; a 4096-slice history does not
    get there), which then takes `warm` untimed and `steps` timed steps: the same
    kernels at ten stages per step instead of six."""
    info = s.info()
    nb = int(info.nb_valid)
    t, C, R, dC, dR = (s.read(f) for f in (pk.F_T_GRID, pk.F_C, pk.F_R, pk.F_DC, pk.F_DR))
    s2 = pk.Solver(params)
    s2.set_history(t, C, R, dC, dR, nb=nb, dt=info.dt, scheme=pk.SCHEME_SSPRK104)
    del C, R, dC, dR
    s2.step(float("inf"), warm)
    i0, i1, n, elapsed, k = _kernel_window(pk, torch, s2, steps=steps)
    s2.close()
    ev = i1.rhs_evals - i0.rhs_evals
    assert i1.scheme == pk.SCHEME_SSPRK104
    log(f"SSPRK window ({prec_name}): {n} steps in {elapsed:.3f} s, {ev / max(n, 1):.2f} evaluations per step, "
        f"t {i0.t:.5g} -> {i1.t:.5g}, dt {i1.dt:.3g}")
    return {"what": "SSPRK(10,4) steps from the value window's end state (history, state and dt loaded into a "
                    "second solve with the scheme set to SSPRK(10,4))",
            "steps": int(n), "seconds": elapsed, "steps_per_s": n / elapsed, "stage_evals_per_s": ev / elapsed,
            "rhs_evals_per_step": ev / max(n, 1), "t_window": [i0.t, i1.t], "M_window": [int(i0.M), int(i1.M)],
            "dt_end": i1.dt, "accepted": int(i1.accepted - i0.accepted), "rejected": int(i1.rejected - i0.rejected),
            "hist_integral_avg_launch_us": k["hist_integral"][1] / max(k["hist_integral"][0], 1) * 1e3}


def _gamma_of(tmax: float) -> float:
    """gamma = -W_{-1}(-1/t_max) of eq. (theta) (Newton on g - log g = log t_max)."""
    import math
    g = math.log(tmax) + math.log(math.log(tmax))
    for _ in range(50):
        g -= (g - math.log(g) - math.log(tmax)) / (1.0 - 1.0 / g)
    return g


if __name__ == "__main__":
    sys.exit(main())
