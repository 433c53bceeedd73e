"""Host-side checks of libdmfe: exported symbols, struct layout, and the pure host
logic (grid precompute, step-size controller, greedy sparsification) against
the oracle.  No device call is made here."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_2604_06309_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmfe.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("libdmfe.so not built")
    return pk.lib()


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dmfe_[a-z_]+)\s*\(", src)))


def test_every_declared_function_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
        assert n in pk.SIGNATURES, n


def test_struct_layout_matches_header(tmp_path):
    """sizeof/offsetof from the C compiler against the ctypes mirrors."""
    prog = tmp_path / "layout.c"
    structs = {"dmfe_params": pk.dmfe_params, "dmfe_resources": pk.dmfe_resources,
               "dmfe_step_info": pk.dmfe_step_info, "dmfe_control": pk.dmfe_control}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0;}")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.split() for line in out if line)
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)


@pytest.mark.parametrize("L,tmax", [(64, 1e4), (512, 1e2), (4096, 1e7), (2049, 1e4)])
def test_grid_precompute_matches_oracle(lib, L, tmax):
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=tmax, L=L)
    th, thc, nu, g = pk.dmfe_grid(p)
    oth, othc = oracle.theta_grid(L, tmax)
    onu = oracle.quad_weights(oth)
    assert abs(g - oracle.gamma_of(tmax)) <= 4e-16 * g
    # both evaluate eq. (theta) without cancellation; theta is conditioned like
    # 2 gamma ulps in y, so the two evaluations agree to ~2 gamma * 1.1e-16 relative
    small = np.minimum(th, thc)
    osmall = np.minimum(oth, othc)
    assert np.all(np.abs(small - osmall) <= 6e-15 * osmall)
    # the quadrature weights come from two different banded solvers
    assert np.max(np.abs(nu - onu)) <= 1e-12 * np.max(np.abs(onu))
    assert abs(nu.sum() - 1) < 1e-13
    for k in range(1, 6):
        assert abs(nu @ th ** k - 1 / (k + 1)) < 1e-13


def test_grid_rejects_bad_params(lib):
    p = pk.make_params({3: 1.0}, 0.5, t_max=2.0, L=64)  # t_max <= e: Lambert branch undefined
    with pytest.raises(pk.DmfeError):
        pk.dmfe_grid(p)
    p = pk.make_params({3: 1.0}, 0.5, L=64, grid_alpha=0.5)
    with pytest.raises(pk.DmfeError) as e:
        pk.dmfe_grid(p)
    assert e.value.status == pk.ERR_UNSUPPORTED
    p = pk.make_params({1: 1.0}, 0.5, L=64)
    with pytest.raises(pk.DmfeError):
        pk.dmfe_grid(p)
    p = pk.make_params({3: 1.0}, 0.5, L=64, s=7)
    with pytest.raises(pk.DmfeError):
        pk.dmfe_grid(p)
    # theta-stencil options: scheme, Floater-Hormann degree, log flag, stencil size
    for kw in (dict(theta_interp=4), dict(theta_interp=-1), dict(theta_interp=pk.INTERP_INDEX_FH, fh_d=10),
               dict(theta_interp=pk.INTERP_THETA_FH, fh_d=-1), dict(s=18), dict(s=2)):
        with pytest.raises(pk.DmfeError) as e:
            pk.dmfe_grid(pk.make_params({3: 1.0}, 0.5, L=64, **kw))
        assert e.value.status == pk.ERR_INVALID, kw
    p = pk.make_params({3: 1.0}, 0.5, L=64)
    p.log_r = 2
    with pytest.raises(pk.DmfeError):
        pk.dmfe_grid(p)
    # history capacity: up to 65536 slices with every scheme
    for kw in (dict(), dict(theta_interp=pk.INTERP_INDEX_FH), dict(theta_interp=pk.INTERP_THETA_LAGRANGE),
               dict(log_r=True)):
        pk.dmfe_grid(pk.make_params({3: 1.0}, 0.5, L=64, M_cap=65536, **kw))
    for kw in (dict(M_cap=65537), dict(M_cap=65537, theta_interp=pk.INTERP_INDEX_FH), dict(M_cap=15)):
        with pytest.raises(pk.DmfeError) as e:
            pk.dmfe_grid(pk.make_params({3: 1.0}, 0.5, L=64, **kw))
        assert e.value.status == pk.ERR_INVALID, kw
    for kw in (dict(s=16), dict(theta_interp=pk.INTERP_THETA_FH, s=14, fh_d=13), dict(log_r=True),
               dict(theta_interp=pk.INTERP_INDEX_LAGRANGE, fh_d=99)):  # fh_d is read by the FH schemes only
        pk.dmfe_grid(pk.make_params({3: 1.0}, 0.5, L=64, **kw))


def _ctl(eps=1e-8, dt=0.1, rho=4.0, M=20, scheme=0, policy=0, dt_min=1e-9):
    c = pk.dmfe_control()
    c.eps, c.dt, c.rho, c.M, c.scheme, c.policy, c.dt_min = eps, dt, rho, M, scheme, policy, dt_min
    return c


def test_controller_rules_scripted(lib):
    """Sec. 3.5: accept; x0.9 above eps; x1.01 below eps/2; reject+revert 10+halve above 2 eps."""
    c = _ctl()
    st, acc, nrev = pk.dmfe_control_update(c, 0.3e-8)
    assert st == 0 and acc and nrev == 0 and c.dt == 0.1 * 1.01
    c = _ctl()
    st, acc, nrev = pk.dmfe_control_update(c, 0.7e-8)
    assert acc and c.dt == 0.1
    c = _ctl()
    st, acc, nrev = pk.dmfe_control_update(c, 1.5e-8)
    assert acc and c.dt == 0.1 * 0.9
    c = _ctl()
    st, acc, nrev = pk.dmfe_control_update(c, 2.5e-8)
    assert not acc and nrev == 10 and c.dt == 0.05
    c = _ctl(M=4)
    st, acc, nrev = pk.dmfe_control_update(c, 1.0)
    assert not acc and nrev == 3
    # DP5 -> SSPRK(10,4) at the DP5 real-axis boundary, then halve
    c = _ctl(dt=0.82, rho=4.0)
    st, acc, nrev = pk.dmfe_control_update(c, 0.1e-8)
    assert acc and c.scheme == 1 and c.dt == 0.5 * (0.82 * 1.01)
    c = _ctl(dt=0.82, rho=4.0, policy=2)
    pk.dmfe_control_update(c, 0.1e-8)
    assert c.scheme == 0
    # SSPRK(10,4) cap at its real-axis limit
    c = _ctl(dt=3.47, rho=4.0, scheme=1)
    pk.dmfe_control_update(c, 0.1e-8)
    assert c.dt == 13.917 / 4.0
    # underflow and non-finite
    c = _ctl(dt=1.5e-9)
    st, acc, nrev = pk.dmfe_control_update(c, 1.0)
    assert st == pk.ERR_STEP_UNDERFLOW
    st, acc, nrev = pk.dmfe_control_update(_ctl(), float("nan"))
    assert st == pk.ERR_NONFINITE


def test_controller_matches_oracle_constants(lib):
    assert oracle.DP5_LIMIT == 3.3065 and oracle.SSP_LIMIT == 13.917
    A, b, _, _ = oracle.dp5_tableau()
    assert oracle.stability_limit(A, b) >= 3.3065


def test_sparsify_select_matches_oracle(lib):
    rng = np.random.default_rng(11)
    for trial in range(200):
        M = int(rng.integers(3, 60))
        eps = rng.uniform(0, 2, M)
        eps[0] = eps[-1] = -1
        last = int(rng.integers(0, M - 1))
        n1, d1 = pk.dmfe_sparsify_select(eps, last, 1.0)
        n2, d2 = oracle.sparsify_select(eps, last, 1.0)
        assert n1 == n2 and np.array_equal(d1, d2)


def test_timing_calls_need_a_handle(lib):
    """The timing entry points refuse a null handle (host checks, no device call)."""
    assert lib.dmfe_timing(None, 1) == pk.ERR_INVALID
    assert lib.dmfe_timing_select(None, 1) == pk.ERR_INVALID
    n, ms, sl = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    assert lib.dmfe_timing_read(None, 0, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(sl)) == pk.ERR_INVALID


def test_param_record_needs_a_handle(lib):
    need = ctypes.c_size_t(7)
    assert lib.dmfe_param_record(None, None, 0, ctypes.byref(need)) == pk.ERR_INVALID


def test_footprint(lib):
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.55, t_max=1e7, L=4096)
    fp = pk.dmfe_footprint(p)
    # history slots (M_cap = L, plus the stage slot) and the two coordinate tables
    hist, coords = (4096 + 1) * 4096 * 32, 2 * 4096 * 4096 * 8
    assert hist + coords <= fp < (hist + coords) * 1.01
    p32 = pk.make_params({3: 0.5, 4: 0.5}, 0.55, t_max=1e7, L=4096, precision=pk.FP32_COMP)
    assert fp - pk.dmfe_footprint(p32) == hist // 2
    # the barycentric coefficient table of the other theta schemes: (L-s+1) rows of s+1
    for interp in (pk.INTERP_THETA_LAGRANGE, pk.INTERP_INDEX_FH, pk.INTERP_THETA_FH):
        pt = pk.make_params({3: 0.5, 4: 0.5}, 0.55, t_max=1e7, L=4096, theta_interp=interp, s=12)
        extra = pk.dmfe_footprint(pt) - pk.dmfe_footprint(pk.make_params({3: 0.5, 4: 0.5}, 0.55, t_max=1e7, L=4096,
                                                                          s=12))
        assert (4096 - 12 + 1) * 13 * 8 <= extra < (4096 - 12 + 1) * 13 * 8 + 512
    pu = pk.make_params({3: 1.0}, 0.5, mode=pk.UNIFORM, h=0.05, N=1000)
    assert pk.dmfe_footprint(pu) >= 2 * 1001 * 1002 // 2 * 8


def test_checkpoint_load_rejects_bad_files(lib, tmp_path):
    """Loading fails cleanly, before any device work, on a missing file, a file of
    another kind, and a checkpoint whose payload was altered."""
    missing = tmp_path / "none.ckpt"
    with pytest.raises(pk.DmfeError) as e:
        pk.dmfe_checkpoint_load(str(missing))
    assert e.value.status == pk.ERR_INVALID
    junk = tmp_path / "junk.ckpt"
    junk.write_bytes(b"not a checkpoint" * 64)
    with pytest.raises(pk.DmfeError) as e:
        pk.dmfe_checkpoint_load(str(junk))
    assert e.value.status == pk.ERR_INVALID
    assert "checkpoint" in pk.dmfe_last_error()


class _CkptHeader(ctypes.Structure):
    """The checkpoint file header (version 2) as the library writes it."""
    _fields_ = [("magic", ctypes.c_char * 8), ("version", ctypes.c_uint32), ("header_bytes", ctypes.c_uint32),
                ("params", pk.dmfe_params), ("M", ctypes.c_int64), ("nb_valid", ctypes.c_int64),
                ("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64), ("reverts", ctypes.c_int64),
                ("n_sparsify", ctypes.c_int64), ("removed", ctypes.c_int64), ("rhs_evals", ctypes.c_int64),
                ("t", ctypes.c_double), ("dt", ctypes.c_double), ("eps_rk", ctypes.c_double),
                ("scheme", ctypes.c_int32), ("fsal_valid", ctypes.c_int32), ("point_bytes", ctypes.c_int32),
                ("L", ctypes.c_int32), ("payload_bytes", ctypes.c_uint64), ("checksum", ctypes.c_uint64)]


def _fnv1a64_words(data: bytes, h: int = 1469598103934665603) -> int:
    """FNV-1a over little-endian 64-bit words, then the trailing bytes."""
    mask = (1 << 64) - 1
    n8 = len(data) // 8 * 8
    for w in np.frombuffer(data[:n8], dtype="<u8").tolist():
        h = ((h ^ w) * 1099511628211) & mask
    for b in data[n8:]:
        h = ((h ^ b) * 1099511628211) & mask
    return h


def test_checkpoint_header_is_covered_by_the_checksum(lib, tmp_path):
    """A checkpoint file written here in the library's format (one slice, L = 32,
    FP64) passes the load's checks and only then needs a device; the same file
    with one bit of the temperature, of the payload or of the version changed is
    refused with DMFE_ERR_INVALID before any device call."""
    L, M = 32, 1
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=L, M_cap=64, eps=1e-8, dt0=1e-3, dt_min=1e-12)
    payload = np.concatenate([np.zeros(M), np.ones(2 * L), np.zeros(2 * L), np.tile([1.0, 1.0, 0.0, 0.0], L)])
    payload = payload.tobytes()
    hdr = _CkptHeader()
    hdr.magic = b"DMFECKP1"
    hdr.version, hdr.header_bytes = 2, ctypes.sizeof(_CkptHeader)
    hdr.params = p
    hdr.M, hdr.nb_valid, hdr.dt, hdr.point_bytes, hdr.L = M, 0, 1e-3, 32, L
    hdr.payload_bytes = len(payload)
    hdr.checksum = _fnv1a64_words(payload, _fnv1a64_words(bytes(hdr)))
    good = bytes(hdr) + payload

    def load(raw: bytes) -> int:
        path = tmp_path / "c.ckpt"
        path.write_bytes(raw)
        out = ctypes.c_void_p()
        res = pk.dmfe_resources()
        st = lib.dmfe_checkpoint_load(os.fsencode(str(path)), ctypes.byref(res), ctypes.byref(out))
        if out.value:
            lib.dmfe_destroy(out)
        return st

    # valid: the checks pass and loading proceeds to the device (absent on a CPU-only host)
    assert load(good) in (pk.OK, pk.ERR_DEVICE)
    t_at = _CkptHeader.params.offset + pk.dmfe_params.T.offset
    for at in (t_at + 2, t_at + 7, len(good) - 3, _CkptHeader.version.offset):
        raw = bytearray(good)
        raw[at] ^= 0x10
        assert load(bytes(raw)) == pk.ERR_INVALID, at
    assert load(good[:-1]) == pk.ERR_INVALID
