"""Host-side checks of the C ABI (no GPU needed, no compute calls).

The library must load, export every function include/nbody.h declares, size
workspaces and checkpoints as documented, and reject invalid arguments on the
host before anything is enqueued.  Calls here fail validation before they
touch the HIP runtime, so they are safe without a device; the fake pointers
passed are never dereferenced.
"""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")

pytestmark = pytest.mark.skipif(
    not os.path.exists(os.path.join(ROOT, "paper_2203_08263_amd", "libnbody_hip.so")),
    reason="libnbody_hip.so not built (run __graft_entry__.build())")


@pytest.fixture(scope="module")
def B():
    from paper_2203_08263_amd import binding
    binding.load_library()
    return binding


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(nbody_\w+)\s*\(",
                                 txt, flags=re.M)))


def test_header_declares_the_four_entry_points():
    names = _declared_functions()
    for f in ("nbody_accel", "nbody_step", "nbody_accel_vjp", "nbody_step_adjoint"):
        assert f in names


def test_library_exports_every_declared_symbol(B):
    lib = ctypes.CDLL(B.library_path())
    names = _declared_functions()
    assert set(names) == set(B.SYMBOLS)
    for name in names:
        assert hasattr(lib, name), name


def test_header_enums_match_binding(B):
    txt = open(HEADER).read()
    for name, val in [("NBODY_FP64", B.NBODY_FP64), ("NBODY_MIXED", B.NBODY_MIXED),
                      ("NBODY_MIXED_D64", B.NBODY_MIXED_D64),
                      ("NBODY_MIXED_NF", B.NBODY_MIXED_NF),
                      ("NBODY_MIXED_NF64", B.NBODY_MIXED_NF64),
                      ("NBODY_MIXED_DS", B.NBODY_MIXED_DS),
                      ("NBODY_OP_MORTON_SORT", B.NBODY_OP_MORTON_SORT),
                      ("NBODY_OP_STEP_ADJOINT", B.NBODY_OP_STEP_ADJOINT)]:
        m = re.search(r"\b%s\s*=\s*(\d+)" % name, txt)
        assert m and int(m.group(1)) == val
    assert "#define NBODY_ACC_VALID 1u" in txt
    assert "#define NBODY_HALF_KICK_DRIFT 2u" in txt
    assert B.NBODY_HALF_KICK_DRIFT == 2
    assert "#define NBODY_MAX_N ((int64_t)1 << 28)" in txt


def test_error_strings(B):
    lib = B.load_library()
    for code in range(5):
        assert lib.nbody_error_string(code)
    assert lib.nbody_error_string(99) == b"unknown status code"


def test_checkpoint_bytes(B):
    assert B.nbody_checkpoint_bytes(100, 50, 10) == 5 * 9 * 100 * 8
    assert B.nbody_checkpoint_bytes(100, 51, 10) == 6 * 9 * 100 * 8
    assert B.nbody_checkpoint_bytes(100, 0, 10) == 9 * 100 * 8
    assert B.nbody_checkpoint_bytes(100, 5, 10) == 9 * 100 * 8
    inv = ctypes.c_size_t(-1).value
    assert B.nbody_checkpoint_bytes(0, 5, 1) == inv
    assert B.nbody_checkpoint_bytes(100, -1, 1) == inv
    assert B.nbody_checkpoint_bytes(100, 5, 0) == inv


def test_workspace_bytes(B):
    inv = ctypes.c_size_t(-1).value
    for prec in (0, 1, 2, 5):
        for n in (1, 255, 256, 1000, 16384, 65536, 262144):
            step = B.nbody_workspace_bytes(B.NBODY_OP_STEP, n, 10, 1, prec)
            acc = B.nbody_workspace_bytes(B.NBODY_OP_ACCEL, n, 0, 1, prec)
            vjp = B.nbody_workspace_bytes(B.NBODY_OP_VJP, n, 0, 1, prec)
            adj = B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, n, 50, 10, prec)
            # partial sums of at least one split, 256-byte rounded
            assert step >= 3 * n * 8 and step % 256 == 0
            assert acc in (0,) or (acc >= 6 * n * 8 and acc % 256 == 0)
            assert vjp in (0,) or (vjp >= 8 * n * 8 and vjp % 256 == 0)
            # v, a, abar, 10 segment positions, partials
            assert adj >= (3 * 3 + 10 * 3 + 4) * n * 8
            # small systems step in one launch per step, drifting the
            # positions into a second array in the workspace (FP64 up to
            # n = 2048, D64 and DS up to 1024, mixed up to 512)
            if n <= {0: 2048, 1: 512, 2: 1024, 5: 1024}[prec]:
                assert step >= acc + 3 * n * 8
        assert B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, 100, 50, 0, prec) == inv
    assert B.nbody_workspace_bytes(7, 100, 0, 1, 0) == inv
    assert B.nbody_workspace_bytes(0, 0, 0, 1, 0) == inv
    assert B.nbody_workspace_bytes(0, 100, 0, 1, 6) == inv
    assert B.nbody_workspace_bytes(0, B.NBODY_MAX_N + 1, 0, 1, 0) == inv
    # fewer segment positions are needed when steps < ckpt_every
    a = B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, 1000, 3, 10, 0)
    b = B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, 1000, 30, 10, 0)
    assert a < b


# ------------------------------------------- argument errors, no launches --

FAKE = 0x10000  # aligned, never dereferenced: validation fails first


def _p(v):
    return ctypes.c_void_p(v)


def _params(B, G=1.0, eps=1e-3, dt=1e-3):
    return ctypes.byref(B._Params(G, eps, dt))


def _accel(B, n=64, pos=FAKE, mass=FAKE, acc=FAKE, prec=0, ws=None, wsb=0, **kw):
    lib = B.load_library()
    return lib.nbody_accel(n, _p(pos), _p(mass), _p(acc), _params(B, **kw), prec,
                           _p(ws), wsb, None)


@pytest.mark.parametrize("kw,msg", [
    (dict(n=0), "outside"), (dict(n=-5), "outside"),
    (dict(n=(1 << 28) + 1), "outside"),
    (dict(pos=0), "pos is NULL"), (dict(mass=0), "mass is NULL"),
    (dict(acc=0), "acc is NULL"), (dict(pos=FAKE + 4), "aligned"),
    (dict(eps=0.0), "eps"), (dict(eps=-1.0), "eps"), (dict(eps=math.nan), "eps"),
    (dict(eps=1e-200), "eps^2"), (dict(G=math.inf), "G is not finite"),
    (dict(prec=6), "precision"), (dict(prec=-1), "precision"),
])
def test_accel_rejects_invalid_arguments(B, kw, msg):
    rc = _accel(B, **kw)
    assert rc == 1
    assert msg in B.load_library().nbody_last_error().decode()


def test_accel_workspace_too_small(B):
    n = 65536
    need = B.nbody_workspace_bytes(B.NBODY_OP_ACCEL, n, 0, 1, 0)
    assert need > 0
    assert _accel(B, n=n, ws=FAKE, wsb=need - 8) == 2
    assert _accel(B, n=n, ws=None, wsb=0) == 2
    assert _accel(B, n=n, ws=0, wsb=need) == 1  # NULL workspace


def _accel_noalloc(B, n=64, pos=FAKE, mass=FAKE, acc=FAKE, prec=0, **kw):
    lib = B.load_library()
    return lib.nbody_accel_noalloc(n, _p(pos), _p(mass), _p(acc), _params(B, **kw),
                                   prec, None)


@pytest.mark.parametrize("kw,msg", [
    (dict(n=0), "outside"), (dict(pos=0), "pos is NULL"), (dict(acc=0), "acc is NULL"),
    (dict(mass=FAKE + 4), "aligned"), (dict(eps=0.0), "eps"),
    (dict(prec=1, eps=1e-14), "FP32 pair range"), (dict(prec=7), "precision"),
])
def test_accel_noalloc_rejects_invalid_arguments(B, kw, msg):
    assert _accel_noalloc(B, **kw) == 1
    assert msg in B.load_library().nbody_last_error().decode()


# (n, precision) whose nbody_accel workspace exceeds the static scratch: the
# first size over it for each precision, and the largest workspaces of the
# FP32-pair modes (2 source splits of just under 2^21 bodies).
@pytest.mark.parametrize("n,prec", [(65025, 0), (262144, 0), (932068, 1), (2096891, 1),
                                    (932068, 2), (681198, 3), (14658561, 4),
                                    (932068, 5)])
def test_accel_noalloc_rejects_sizes_beyond_its_scratch(B, n, prec):
    need = B.nbody_workspace_bytes(B.NBODY_OP_ACCEL, n, 0, 1, prec)
    assert need > B.NBODY_NOALLOC_SCRATCH_BYTES
    assert _accel_noalloc(B, n=n, prec=prec) == 2
    assert "static scratch" in B.load_library().nbody_last_error().decode()


def test_accel_noalloc_limits_match_the_header(B):
    """The sizes the header says fit: every n below the stated first
    failures (checked on a grid of n plus the neighbours of each limit)."""
    lim = B.NBODY_NOALLOC_SCRATCH_BYTES
    txt = open(HEADER).read()
    assert re.search(r"NBODY_NOALLOC_SCRATCH_BYTES \(\(size_t\)64 << 20\)", txt)
    assert lim == 64 << 20
    first = {0: 65025, 1: 932068, 2: 932068, 3: 681198, 4: 14658561, 5: 932068}
    for prec, nf in first.items():
        assert B.nbody_workspace_bytes(B.NBODY_OP_ACCEL, nf, 0, 1, prec) > lim
        grid = sorted(set(list(range(1, min(nf, 70000), 97)) + [nf - 1, nf - 2, nf - 255]
                          + list(range(1, nf, max(1, nf // 3000)))))
        for n in grid:
            assert B.nbody_workspace_bytes(B.NBODY_OP_ACCEL, n, 0, 1, prec) <= lim, (prec, n)


def test_step_rejects_invalid_arguments(B):
    lib = B.load_library()
    pr = _params(B)
    n = 1000
    ws = B.nbody_workspace_bytes(B.NBODY_OP_STEP, n, 1, 1, 0)

    def step(steps=1, flags=0, ckpt=None, K=1, dt=1e-3, vel=FAKE, wsb=ws):
        return lib.nbody_step(n, steps, _p(FAKE), _p(vel), _p(FAKE), _p(FAKE),
                              _params(B, dt=dt), 0, flags, _p(ckpt), K, _p(FAKE),
                              wsb, None)
    assert step(steps=-1) == 1
    assert step(flags=4) == 1
    assert step(flags=8 | 1) == 1
    assert step(ckpt=FAKE, K=0) == 1
    assert step(dt=math.nan) == 1
    assert step(vel=0) == 1
    assert step(wsb=ws - 1) == 2
    assert pr is not None


def test_vjp_and_adjoint_reject_invalid_arguments(B):
    lib = B.load_library()
    n = 1000
    assert lib.nbody_accel_vjp(n, _p(FAKE), _p(FAKE), _p(0), _p(FAKE), _p(FAKE),
                               _params(B), 0, _p(FAKE), 1 << 30, None) == 1
    ws = B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, n, 10, 5, 1)

    def adj(steps=10, K=5, ckpt=FAKE, gacc=None, wsb=ws, prec=1, flags=0):
        return lib.nbody_step_adjoint(n, steps, K, _p(ckpt), _p(FAKE), _params(B),
                                      prec, flags, _p(FAKE), _p(FAKE), _p(gacc),
                                      _p(FAKE), _p(FAKE), wsb, None)
    assert adj(K=0) == 1
    assert adj(steps=-2) == 1
    assert adj(ckpt=0) == 1
    assert adj(gacc=FAKE + 2) == 1
    assert adj(prec=6) == 1
    assert adj(flags=1) == 1   # NBODY_ACC_VALID is not an adjoint flag
    assert adj(wsb=ws - 256) == 2


@pytest.mark.parametrize("prec", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("eps", [1e-14, 2.0 ** -42 * 0.999, 1e-30, 1e20])
def test_fp32_pair_modes_reject_eps_outside_fp32_range(B, prec, eps):
    """Every precision but FP64 evaluates the self pair in FP32 with weight
    m eps^-3: an eps whose FP32 eps^2 flushes to 0 or whose eps^-3 overflows
    would make every output NaN, so the host rejects it before any launch
    (accel, VJP, step and adjoint alike); FP64 accepts the same eps."""
    lib = B.load_library()
    n = 1000
    assert _accel(B, n=n, prec=prec, eps=eps, ws=FAKE, wsb=1 << 30) == 1
    assert "FP32 pair range" in lib.nbody_last_error().decode()
    assert lib.nbody_accel_vjp(n, _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE),
                               _params(B, eps=eps), prec, _p(FAKE), 1 << 30, None) == 1
    assert lib.nbody_step(n, 1, _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE),
                          _params(B, eps=eps), prec, 0, None, 1, _p(FAKE), 1 << 30,
                          None) == 1
    assert lib.nbody_step_adjoint(n, 10, 5, _p(FAKE), _p(FAKE), _params(B, eps=eps),
                                  prec, 0, _p(FAKE), _p(FAKE), None, _p(FAKE),
                                  _p(FAKE), 1 << 30, None) == 1
    assert lib.nbody_accel_rows(n, 0, 10, _p(FAKE), _p(FAKE), _p(FAKE),
                                _params(B, eps=eps), prec, _p(FAKE), 1 << 30,
                                None) == 1
    assert "FP32 pair range" in lib.nbody_last_error().decode()
    if eps < 1e19:
        # FP64 accepts this eps and fails only later, on the missing workspace
        # (n = 65536 needs one, so nothing is launched)
        assert _accel(B, n=65536, prec=0, eps=eps, ws=None, wsb=0) == 2


def test_fp32_pair_modes_accept_the_smallest_eps(B):
    lib = B.load_library()
    txt = open(HEADER).read()
    assert "#define NBODY_MIN_EPS_FP32 (0x1p-42)" in txt
    # passes the eps check, then fails on the missing workspace
    for prec in (1, 2, 3, 4, 5):
        rc = _accel(B, n=65536, prec=prec, eps=2.0 ** -42, ws=None, wsb=0)
        assert rc == 2, lib.nbody_last_error().decode()


@pytest.mark.parametrize("prec", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("eps", [2.0 ** -42, 1e-11, 2.0 ** -32 * 0.999])
def test_fp32_vjp_rejects_eps_below_its_range(B, prec, eps):
    """The FP32 VJP pair forms s^-5/2 (e.h) before it multiplies by e; over
    all pair distances that reaches 0.29 eps^-4 H, so the VJP calls take
    eps >= 2^-32 in the FP32 pair modes, while the forward calls still take
    eps down to 2^-42."""
    lib = B.load_library()
    n = 1000
    assert lib.nbody_accel_vjp(n, _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE),
                               _params(B, eps=eps), prec, _p(FAKE), 1 << 30, None) == 1
    assert "(VJP)" in lib.nbody_last_error().decode()
    assert lib.nbody_accel_vjp_rows(n, 0, 10, _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE),
                                    _p(FAKE), _params(B, eps=eps), prec, _p(FAKE),
                                    1 << 30, None) == 1
    assert "(VJP)" in lib.nbody_last_error().decode()
    assert lib.nbody_step_adjoint(n, 10, 5, _p(FAKE), _p(FAKE), _params(B, eps=eps),
                                  prec, 0, _p(FAKE), _p(FAKE), None, _p(FAKE),
                                  _p(FAKE), 1 << 30, None) == 1
    assert "(VJP)" in lib.nbody_last_error().decode()
    # the forward call passes the eps check and fails on the missing workspace
    assert _accel(B, n=65536, prec=prec, eps=eps, ws=None, wsb=0) == 2
    # FP64 VJP: past the eps check, fails on the missing workspace
    assert lib.nbody_accel_vjp(65536, _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE),
                               _params(B, eps=eps), 0, None, 0, None) == 2


def test_fp32_vjp_accepts_the_smallest_eps(B):
    lib = B.load_library()
    txt = open(HEADER).read()
    assert "#define NBODY_MIN_EPS_FP32_VJP (0x1p-32)" in txt
    assert B.NBODY_MIN_EPS_FP32_VJP == 2.0 ** -32 and B.NBODY_MIN_EPS_FP32 == 2.0 ** -42
    for prec in (1, 2, 3, 4, 5):
        rc = lib.nbody_accel_vjp(65536, _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE),
                                 _p(FAKE), _params(B, eps=2.0 ** -32), prec, None, 0,
                                 None)
        assert rc == 2, lib.nbody_last_error().decode()


def test_auto_checkpoint_interval_fits_the_budget(B):
    from paper_2203_08263_amd import auto_ckpt_every
    assert auto_ckpt_every(8192, 50) == 1               # every state fits in 1 GiB
    for n, S, budget in ((8192, 50, 10 << 20), (262144, 1000, 1 << 30),
                         (1 << 20, 200, 4 << 30), (200, 12, 120000)):
        K = auto_ckpt_every(n, S, "mixed", budget)
        need = (B.nbody_checkpoint_bytes(n, S, K)
                + B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, n, S, K, 1))
        assert 1 <= K <= S and need <= budget, (n, S, K, need)
        if K > 1:                                       # and it is the smallest
            prev = (B.nbody_checkpoint_bytes(n, S, K - 1)
                    + B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, n, S, K - 1, 1))
            assert prev > budget
    # nothing fits: the interval with the smallest footprint
    need = {K: B.nbody_checkpoint_bytes(200, 12, K)
            + B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, 200, 12, K, 1)
            for K in range(1, 13)}
    assert auto_ckpt_every(200, 12, "mixed", 20000) == min(need, key=need.get)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2203_08263_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        binding.load_library()


# ------------------------------------------------------------- row ranges --

def test_rows_workspace_matches_full_call(B):
    # the plan for all n rows is the whole-system plan (same split count, so
    # the same workspace and, on the GPU, bitwise the same result)
    for prec in (0, 1, 2, 3, 4, 5):
        for n in (1, 255, 256, 1000, 3001, 16384, 65536, 262144, 1 << 20):
            for op in (B.NBODY_OP_ACCEL, B.NBODY_OP_VJP):
                assert (B.nbody_rows_workspace_bytes(op, n, n, prec)
                        == B.nbody_workspace_bytes(op, n, 0, 1, prec)), (op, n, prec)


def test_rows_workspace_bytes(B):
    inv = ctypes.c_size_t(-1).value
    for prec in (0, 1, 2, 3, 4, 5):
        assert B.nbody_rows_workspace_bytes(B.NBODY_OP_ACCEL, 1000, 0, prec) == 0
        for n, rows in ((262144, 32768), (262144, 1), (1 << 28, 1), (5000, 77)):
            a = B.nbody_rows_workspace_bytes(B.NBODY_OP_ACCEL, n, rows, prec)
            v = B.nbody_rows_workspace_bytes(B.NBODY_OP_VJP, n, rows, prec)
            # at most 64 source splits of FP64 partials (plus the bounding
            # boxes of the near / far mode)
            boxes = ((-(-n // 16) + 2 * -(-rows // 4)) * 48 + 255) // 256 * 256 \
                if prec in (3, 4) else 0
            assert a % 256 == 0 and a <= 64 * 3 * rows * 8 + 256 + boxes
            assert v % 256 == 0 and v <= 64 * 4 * rows * 8 + 256 + boxes
        assert B.nbody_rows_workspace_bytes(B.NBODY_OP_STEP, 1000, 10, prec) == inv
        assert B.nbody_rows_workspace_bytes(B.NBODY_OP_ACCEL, 1000, 1001, prec) == inv
        assert B.nbody_rows_workspace_bytes(B.NBODY_OP_ACCEL, 1000, -1, prec) == inv
    assert B.nbody_rows_workspace_bytes(B.NBODY_OP_ACCEL, 1000, 10, 6) == inv


def test_rows_reject_invalid_ranges(B):
    lib = B.load_library()

    def acc_rows(n=1000, r0=0, rc=10, pos=FAKE, prec=0):
        return lib.nbody_accel_rows(n, r0, rc, _p(pos), _p(FAKE), _p(FAKE),
                                    _params(B), prec, _p(FAKE), 1 << 30, None)

    def vjp_rows(n=1000, r0=0, rc=10, gacc=FAKE):
        return lib.nbody_accel_vjp_rows(n, r0, rc, _p(FAKE), _p(FAKE), _p(gacc),
                                        _p(FAKE), _p(FAKE), _params(B), 0,
                                        _p(FAKE), 1 << 30, None)
    for f in (acc_rows, vjp_rows):
        assert f(r0=-1) == 1
        assert f(rc=-1) == 1
        assert f(r0=995, rc=6) == 1
        assert "outside [0, n" in lib.nbody_last_error().decode()
        assert f(r0=1001, rc=0) == 1
        assert f(n=0) == 1
        # an empty range is a valid no-op: pointers are not examined
        assert f(r0=1000, rc=0) == 0
    assert acc_rows(rc=0, pos=0) == 0
    assert acc_rows(pos=0) == 1
    assert acc_rows(prec=7) == 1
    assert vjp_rows(gacc=0) == 1
    # too small a workspace
    need = B.nbody_rows_workspace_bytes(B.NBODY_OP_ACCEL, 262144, 32768, 1)
    assert need > 0
    assert lib.nbody_accel_rows(262144, 0, 32768, _p(FAKE), _p(FAKE), _p(FAKE),
                                _params(B), 1, _p(FAKE), need - 8, None) == 2


# -------------------------------------------------------- near / far, sort --

def _tile_boxes(n):
    return (6 * ((n + 255) // 256) * 8 + 255) // 256 * 256


def test_near_far_workspace_adds_box_scratch(B):
    # the near / far mode has the launch plan of the mixed mode plus bounding
    # boxes at the front of the workspace: one per run of >= 16 sources, per
    # wave of >= 4 targets and per workgroup of >= 16 targets
    def most(n):
        boxes = -(-n // 16) + -(-n // 4) + -(-n // 16)
        return (boxes * 48 + 255) // 256 * 256
    ops = (B.NBODY_OP_ACCEL, B.NBODY_OP_VJP, B.NBODY_OP_STEP)
    for n in (16384, 262144):
        for op in ops:
            nf = B.nbody_workspace_bytes(op, n, 10, 1, B.NBODY_MIXED_NF)
            mx = B.nbody_workspace_bytes(op, n, 10, 1, B.NBODY_MIXED)
            assert 0 < nf - mx <= most(n) and (nf - mx) % 256 == 0, (op, n)
        adj_nf = B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, n, 50, 10, 3)
        adj_mx = B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, n, 50, 10, 1)
        assert 0 < adj_nf - adj_mx <= most(n)
        # rows: boxes over all n sources plus the target rows' own
        r = B.nbody_rows_workspace_bytes(B.NBODY_OP_ACCEL, n, n // 8, 3)
        assert r > B.nbody_rows_workspace_bytes(B.NBODY_OP_ACCEL, n, n // 8, 1)
        # the FP64-near variant has boxes too (its plan may use more lanes
        # per target, hence fewer splits and a different size)
        for op in ops:
            nf64 = B.nbody_workspace_bytes(op, n, 10, 1, B.NBODY_MIXED_NF64)
            assert 0 < nf64 and nf64 % 256 == 0
            assert nf64 <= B.nbody_workspace_bytes(op, n, 10, 1, B.NBODY_MIXED) + most(n)
        # the potential of the diagnostics uses the D64 arithmetic, no boxes
        assert (B.nbody_workspace_bytes(B.NBODY_OP_DIAGNOSTICS, n, 0, 1, 3)
                == B.nbody_workspace_bytes(B.NBODY_OP_DIAGNOSTICS, n, 0, 1, 2))


def test_small_systems_evaluate_near_far_as_all_near(B):
    # up to 1024 bodies NBODY_MIXED_NF is NBODY_MIXED_D64 (every run near),
    # up to 2048 NBODY_MIXED_NF64 is NBODY_FP64: same workspaces for every
    # operation; above those sizes the near / far modes keep their boxes
    ops = (B.NBODY_OP_ACCEL, B.NBODY_OP_VJP, B.NBODY_OP_STEP,
           B.NBODY_OP_STEP_ADJOINT, B.NBODY_OP_DIAGNOSTICS)
    for n in (1, 300, 1024, 2048):
        for op in ops:
            nf64 = B.nbody_workspace_bytes(op, n, 10, 3, B.NBODY_MIXED_NF64)
            assert nf64 == B.nbody_workspace_bytes(op, n, 10, 3, B.NBODY_FP64), (op, n)
            nf = B.nbody_workspace_bytes(op, n, 10, 3, B.NBODY_MIXED_NF)
            d64 = B.nbody_workspace_bytes(op, n, 10, 3, B.NBODY_MIXED_D64)
            if op == B.NBODY_OP_DIAGNOSTICS:   # the potential is D64 anyway
                assert nf == d64
            else:
                assert (nf == d64) == (n <= 1024), (op, n)
        for op in (B.NBODY_OP_ACCEL, B.NBODY_OP_VJP):
            r64 = B.nbody_rows_workspace_bytes(op, n, max(1, n // 3), B.NBODY_MIXED_NF64)
            assert r64 == B.nbody_rows_workspace_bytes(op, n, max(1, n // 3), B.NBODY_FP64)


def test_morton_workspace_bytes(B):
    for n, npad in ((1, 1), (2, 2), (1000, 1024), (1024, 1024), (1025, 2048),
                    (262144, 262144)):
        want = _tile_boxes(n) + 256 + (npad * 8 + 255) // 256 * 256
        for prec in (0, 1, 2, 3, 4, 5):
            assert B.nbody_workspace_bytes(B.NBODY_OP_MORTON_SORT, n, 0, 1, prec) == want


def test_morton_sort_rejects_invalid_arguments(B):
    lib = B.load_library()
    ws = B.nbody_workspace_bytes(B.NBODY_OP_MORTON_SORT, 1000, 0, 1, 0)

    def sort(n=1000, pos=FAKE, vel=None, vel_out=None, perm=FAKE, wsb=ws):
        return lib.nbody_morton_sort(n, _p(pos), _p(vel), _p(FAKE), _p(perm),
                                     _p(FAKE), _p(vel_out), _p(FAKE), _p(FAKE),
                                     wsb, None)
    assert sort(n=0) == 1
    assert sort(n=(1 << 28) + 1) == 1
    assert sort(pos=0) == 1
    assert sort(perm=0) == 1
    assert sort(perm=FAKE + 4) == 1
    assert sort(vel=FAKE) == 1
    assert "both NULL" in lib.nbody_last_error().decode()
    assert sort(vel_out=FAKE) == 1
    assert sort(wsb=ws - 8) == 2


# ------------------------------------------------------------- FP32 state --

def test_f32_workspace_bytes(B):
    inv = ctypes.c_size_t(-1).value
    for n in (1, 255, 1000, 16384, 262144):
        # the mixed mode's plan with FP32 partials: half its bytes (rounded)
        step = B.nbody_f32_workspace_bytes(B.NBODY_OP_STEP, n)
        step64 = B.nbody_workspace_bytes(B.NBODY_OP_STEP, n, 1, 1, B.NBODY_MIXED)
        if n <= 512:    # minus the mixed loop's second position array
            step64 -= (3 * n * 8 + 255) // 256 * 256
        assert step % 256 == 0 and step >= 12 * n and abs(2 * step - step64) <= 512
        acc = B.nbody_f32_workspace_bytes(B.NBODY_OP_ACCEL, n)
        assert acc == 0 or abs(2 * acc - B.nbody_workspace_bytes(
            B.NBODY_OP_ACCEL, n, 0, 1, B.NBODY_MIXED)) <= 512
    assert B.nbody_f32_workspace_bytes(B.NBODY_OP_VJP, 100) == inv
    assert B.nbody_f32_workspace_bytes(B.NBODY_OP_ACCEL, 0) == inv


def test_f32_rejects_invalid_arguments(B):
    lib = B.load_library()
    ws = B.nbody_f32_workspace_bytes(B.NBODY_OP_STEP, 1000)

    def acc(n=1000, pos=FAKE, **kw):
        return lib.nbody_accel_f32(n, _p(pos), _p(FAKE), _p(FAKE), _params(B, **kw),
                                   _p(FAKE), 1 << 30, None)

    def step(steps=1, flags=0, vel=FAKE, wsb=ws, **kw):
        return lib.nbody_step_f32(1000, steps, _p(FAKE), _p(vel), _p(FAKE), _p(FAKE),
                                  _params(B, **kw), flags, _p(FAKE), wsb, None)
    assert acc(n=0) == 1
    assert acc(pos=0) == 1
    assert acc(pos=FAKE + 2) == 1
    assert acc(eps=0.0) == 1
    assert acc(eps=1e-30) == 1          # eps^2 underflows FP32
    assert "FP32" in lib.nbody_last_error().decode()
    assert acc(G=1e300) == 1
    assert step(steps=-1) == 1
    assert step(flags=4) == 1
    assert step(vel=0) == 1
    assert step(dt=1e300) == 1
    assert step(wsb=ws - 4) == 2


# ------------------------------------------------------ size overflow guards --

def test_step_counts_and_sizes_cannot_overflow(B):
    inv = ctypes.c_size_t(-1).value
    big_n, max_steps = 1 << 28, 1 << 40
    assert "#define NBODY_MAX_STEPS ((int64_t)1 << 40)" in open(HEADER).read()
    # 2^40 records of 9 * 2^28 doubles is far beyond 2^62 bytes
    assert B.nbody_checkpoint_bytes(big_n, max_steps, 1) == inv
    assert B.nbody_checkpoint_bytes(100, max_steps + 1, 1) == inv
    assert B.nbody_checkpoint_bytes(100, max_steps, max_steps) == 9 * 100 * 8
    assert B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, big_n, max_steps,
                                   max_steps, 0) == inv
    assert B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, 100, max_steps + 1,
                                   1, 0) == inv
    lib = B.load_library()
    # rejected on the host before anything is enqueued
    rc = lib.nbody_step(100, max_steps + 1, _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE),
                        _params(B), 0, 0, None, 0, _p(FAKE), 1 << 40, None)
    assert rc == 1 and "steps" in lib.nbody_last_error().decode()
    rc = lib.nbody_step(big_n, max_steps, _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE),
                        _params(B), 0, 0, _p(FAKE), 1, _p(FAKE), 1 << 62, None)
    assert rc == 1 and "overflows" in lib.nbody_last_error().decode()
    rc = lib.nbody_step_adjoint(big_n, max_steps, max_steps, _p(FAKE), _p(FAKE),
                                _params(B), 0, 0, _p(FAKE), _p(FAKE), None, _p(FAKE),
                                _p(FAKE), 1 << 62, None)
    assert rc == 1 and "overflows" in lib.nbody_last_error().decode()
    rc = lib.nbody_step_f32(100, max_steps + 1, _p(FAKE), _p(FAKE), _p(FAKE), _p(FAKE),
                            _params(B), 0, _p(FAKE), 1 << 40, None)
    assert rc == 1


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: bench.py --gpus 2 exits with a message, before touching
    # torch or the GPU
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
