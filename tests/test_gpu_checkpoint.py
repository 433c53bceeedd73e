"""Checkpoint and resume: a solve saved to a file and restored into a new handle
continues bitwise as the uninterrupted solve (same accepted/rejected counts, time
grid and history), through sparsification, the DP5 -> SSPRK(10,4) switch, FP32
histories and asynchronous writes; a checkpoint whose payload is altered is
refused."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2604_06309_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _state(s):
    info = s.info()
    return (info.accepted, info.rejected, info.M, info.scheme, info.sparsify_calls, info.removed,
            s.read(pk.F_T_GRID), s.read(pk.F_C), s.read(pk.F_R), s.read(pk.F_DC), s.read(pk.F_DR))


def _same(a, b):
    assert a[:6] == b[:6], (a[:6], b[:6])
    for x, y in zip(a[6:], b[6:]):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("precision,policy,async_write,n1,n2,extra", [
    (pk.FP64, 0, False, 300, 560, {}),       # DP5, sparsification at a 400-slice cap before and after the save
    (pk.FP32_COMP, 0, True, 300, 560, {}),   # FP32 history, asynchronous write
    (pk.FP64, 1, True, 200, 450, {}),        # SSPRK(10,4) from the start
    # log-R option on a theta Floater-Hormann stencil: the log mirror is rebuilt from the stored slices
    (pk.FP64, 0, False, 300, 560, dict(theta_interp=pk.INTERP_THETA_FH, fh_d=5, log_r=True)),
    (pk.FP32_COMP, 1, True, 200, 450, dict(log_r=True)),
])
def test_resume_is_bitwise(tmp_path, precision, policy, async_write, n1, n2, extra):
    say(f"checkpoint precision={precision} policy={policy} async={async_write} {extra}")
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=64, M_cap=400, eps=1e-8, dt0=1e-3, dt_min=1e-12,
                       precision=precision, scheme_policy=policy, **extra)
    path = str(tmp_path / "solve.ckpt")
    ref = pk.Solver(p)
    ref.step(float("inf"), n1)
    ref.checkpoint(path, async_write=async_write)
    ref.step(float("inf"), n2 - n1)  # steps on while the file is written
    ref.checkpoint_wait()
    want = _state(ref)
    ref.close()
    s = pk.Solver.load(path, p)
    s.step(float("inf"), n2 - n1)
    got = _state(s)
    s.close()
    _same(got, want)
    say(f"  resumed solve equals the uninterrupted one after {want[0] + want[1]} steps, M={want[2]}, "
        f"sparsify passes={want[4]}")


def test_corrupted_checkpoint_is_refused(tmp_path):
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=64, M_cap=100, eps=1e-8, dt0=1e-3, dt_min=1e-12)
    path = tmp_path / "solve.ckpt"
    s = pk.Solver(p)
    s.step(float("inf"), 40)
    s.checkpoint(str(path))
    s.close()
    good = path.read_bytes()
    # one bit of the stored history; one bit of the temperature in the header's parameters
    # (the header starts with an 8-byte magic and two 32-bit words, then the dmfe_params)
    for at in (len(good) - 9, 16 + pk.dmfe_params.T.offset + 3):
        raw = bytearray(good)
        raw[at] ^= 0x40
        path.write_bytes(bytes(raw))
        with pytest.raises(pk.DmfeError) as e:
            pk.Solver.load(str(path), p)
        assert e.value.status == pk.ERR_INVALID
    path.write_bytes(good)
    pk.Solver.load(str(path), p).close()


def test_sparsify_keeps_the_newest_slice_without_derivative():
    """A history whose newest slice has no stored d/dt yet (nb = M-1): a
    sparsification pass removes older slices only (candidates 1..M-12), so the
    newest slice is still the one without a derivative afterwards."""
    L, M = 64, 60
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=L, M_cap=100, eps=1e-8)
    s = pk.Solver(p)
    th = s.read(pk.F_THETA)
    times = 0.1 * np.arange(M)
    # linear in t along fixed theta, with its exact derivative: every residual vanishes
    C = np.array([1.0 - 0.01 * (1 - th) * t for t in times])
    dC = np.array([-0.01 * (1 - th) for _ in times])
    s.set_history(times, C, C, dC, dC, nb=M - 1)
    assert s.info().nb_valid == M - 1
    removed = s.sparsify(1)
    info = s.info()
    s.close()
    assert removed > 0 and info.M == M - removed
    assert info.nb_valid == info.M - 1


def test_parameter_record(tmp_path):
    """The human-readable record of a solve: library build, device, every parameter
    (round-trip exact), the grid and the state; a resumed solve records the same
    parameters and state as the one it was saved from."""
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=64, M_cap=200, eps=1e-8, dt0=1e-3, dt_min=1e-12,
                       theta_interp=pk.INTERP_THETA_FH, fh_d=5, log_r=True)
    s = pk.Solver(p)
    s.step(float("inf"), 40)
    rec = s.param_record()
    say(rec)
    kv = dict(line.split(" = ", 1) for line in rec.splitlines() if " = " in line and not line.startswith("#"))
    info = s.info()
    assert kv["library_revision"] and kv["compiler"] and "gfx950" in kv["device"]
    assert float(kv["T"]) == 0.6 and float(kv["eps"]) == 1e-8 and float(kv["t_max"]) == 1e4
    assert int(kv["L"]) == 64 and int(kv["M_cap"]) == 200 and int(kv["s"]) == 10
    assert kv["theta_interp"] == "theta-floater-hormann" and int(kv["fh_d"]) == 5 and int(kv["log_r"]) == 1
    assert kv["f(q)"] == "0.5 q^3/2 + 0.5 q^4/2"
    assert int(kv["accepted"]) == info.accepted and float(kv["state_t"]) == info.t and int(kv["state_M"]) == info.M
    assert float(kv["grid_gamma"]) > 1.0
    path = str(tmp_path / "rec.ckpt")
    s.checkpoint(path)
    s.close()
    r = pk.Solver.load(path, p)
    kv2 = dict(line.split(" = ", 1) for line in r.param_record().splitlines() if " = " in line)
    r.close()
    for k, v in kv.items():
        if k not in ("command_line",):
            assert kv2[k] == v, k


def test_compressed_snapshot(tmp_path):
    """The post-processing snapshot holds every theta_stride-th node (and theta = 1),
    every slice_stride-th slice (and the newest), E and mu of those slices exactly,
    C and R rounded to FP32, and the parameter record."""
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=64, M_cap=200, eps=1e-8, dt0=1e-3, dt_min=1e-12)
    s = pk.Solver(p)
    s.step(float("inf"), 60)
    path = str(tmp_path / "run.snap")
    s.snapshot(path, theta_stride=3, slice_stride=4)
    snap = pk.load_snapshot(path)
    M = s.info().M
    nodes = np.unique(np.r_[np.arange(0, 64, 3), 63])
    slices = np.unique(np.r_[np.arange(0, M, 4), M - 1])
    np.testing.assert_array_equal(snap["theta"], s.read(pk.F_THETA)[nodes])
    np.testing.assert_array_equal(snap["t"], s.read(pk.F_T_GRID)[slices])
    np.testing.assert_array_equal(snap["E"], s.read(pk.F_ENERGY)[slices])
    np.testing.assert_array_equal(snap["mu"], s.read(pk.F_MU)[slices])
    np.testing.assert_array_equal(snap["C"], s.read(pk.F_C)[np.ix_(slices, nodes)].astype(np.float32))
    np.testing.assert_array_equal(snap["R"], s.read(pk.F_R)[np.ix_(slices, nodes)].astype(np.float32))
    assert (snap["L"], snap["M"], snap["theta_stride"], snap["slice_stride"]) == (64, M, 3, 4)
    assert "L = 64" in snap["record"] and "state_M = %d" % M in snap["record"]
    with pytest.raises(pk.DmfeError):
        s.snapshot(path, theta_stride=0)
    s.close()
