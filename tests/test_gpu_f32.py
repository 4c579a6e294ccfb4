"""GPU parity of the FP32-state path (nbody_accel_f32, nbody_step_f32), the
paper's single-precision variant: FP32 arrays and FP32 arithmetic throughout,
including the sum over sources.

The oracle gets the FP32 input values exactly (upcast), and G = 1,
eps = 2^-10 (eps^2 = 2^-20) and dt = 2^-10 are exact in FP32, so the only
differences are the FP32 roundings the bounds of _tol.accel_bound_f32 count.
"""
import sys

import numpy as np
import pytest

import _tol
from paper_2203_08263_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = 2.0 ** -10
DT = 2.0 ** -10
U32 = 2.0 ** -24


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_08263_amd import binding
    binding.load_library()
    return binding


@pytest.fixture(scope="module")
def dev(B):
    return torch.device("cuda:0")


def F(a, dev):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _state32(n, seed):
    pos, vel, mass = inputs.uniform_cube(n, seed)
    return (pos.astype(np.float32).astype(np.float64),
            vel.astype(np.float32).astype(np.float64),
            mass.astype(np.float32).astype(np.float64))


def _check(got, ref, bound, what):
    err = np.sqrt(((got - ref) ** 2).sum(axis=0))
    worst = int(np.argmax(err / np.maximum(bound, 1e-300)))
    assert np.all(err <= bound), "%s: row %d err %.3e bound %.3e" % (
        what, worst, err[worst], bound[worst])


@pytest.mark.parametrize("n", [1, 2, 257, 3001])
def test_accel_f32_vs_oracle(B, dev, oracle, n):
    say("accel f32", n)
    pos, _, mass = _state32(n, 2000 + n)
    a = N(B.nbody_accel_f32(F(pos, dev), F(mass, dev), 1.0, EPS))
    ref = oracle.accel(pos, mass, 1.0, EPS)
    _check(a, ref, _tol.accel_bound_f32(pos, mass, 1.0, EPS), "accel f32")
    if n == 1:
        assert np.all(a == 0.0)


def test_accel_f32_golden_two_body(B, dev):
    # x1 = 0, x2 = (3, 4, 0), eps^2 = 2^-20, m = (2, 3): |d|^2 + eps^2 = 25 + 2^-20
    pos = np.array([[0.0, 3.0], [0.0, 4.0], [0.0, 0.0]])
    mass = np.array([2.0, 3.0])
    a = N(B.nbody_accel_f32(F(pos, dev), F(mass, dev), 1.0, EPS))
    s = (25.0 + EPS ** 2) ** -1.5
    np.testing.assert_allclose(a[:, 0], 3.0 * s * np.array([3.0, 4.0, 0.0]), rtol=1e-6)
    np.testing.assert_allclose(a[:, 1], -2.0 * s * np.array([3.0, 4.0, 0.0]), rtol=1e-6)


@pytest.mark.parametrize("integrator", ["kdk", "half_kick_drift"])
def test_step_f32_chaining_bitwise(B, dev, integrator):
    pos, vel, mass = _state32(1500, 2100)
    P1, V1, M = F(pos, dev), F(vel, dev), F(mass, dev)
    A1 = torch.empty_like(P1)
    B.nbody_step_f32(P1, V1, A1, M, 1.0, EPS, DT, 5, integrator=integrator)
    P2, V2 = F(pos, dev), F(vel, dev)
    A2 = torch.empty_like(P2)
    B.nbody_step_f32(P2, V2, A2, M, 1.0, EPS, DT, 2, integrator=integrator)
    B.nbody_step_f32(P2, V2, A2, M, 1.0, EPS, DT, 3, acc_valid=True,
                     integrator=integrator)
    for x, y in ((P1, P2), (V1, V2), (A1, A2)):
        assert torch.equal(x, y)
    # zero steps still fill acc
    P3, V3 = F(pos, dev), F(vel, dev)
    A3 = torch.full_like(P3, 7.0)
    B.nbody_step_f32(P3, V3, A3, M, 1.0, EPS, DT, 0)
    assert torch.equal(A3, B.nbody_accel_f32(P3, M, 1.0, EPS))
    assert torch.equal(P3, F(pos, dev)) and torch.equal(V3, F(vel, dev))


def test_step_f32_one_kdk_step_vs_oracle(B, dev, oracle):
    # error propagation through one KDK step, every FP32 rounding counted:
    # a0 (accel bound), v_half = v0 + h a0, x1 = x0 + dt v_half, a1 = A(x1)
    # (accel bound + Lipschitz term of the x1 error), v1 = v_half + h a1
    n = 2000
    pos, vel, mass = _state32(n, 2200)
    P, V, M = F(pos, dev), F(vel, dev), F(mass, dev)
    A = torch.empty_like(P)
    B.nbody_step_f32(P, V, A, M, 1.0, EPS, DT, 1)
    x1, v1, a1 = oracle.step(pos, vel, mass, 1.0, EPS, DT, 1)
    h = 0.5 * DT
    nrm = lambda v: np.sqrt((v * v).sum(axis=0))  # noqa
    a0 = oracle.accel(pos, mass, 1.0, EPS)
    vh = vel + h * a0
    da0 = _tol.accel_bound_f32(pos, mass, 1.0, EPS)
    dvh = h * da0 + 2 * U32 * (nrm(vel) + h * nrm(a0))
    dx1 = DT * dvh + 2 * U32 * (nrm(pos) + DT * nrm(vh))
    da1 = _tol.accel_bound_f32(x1, mass, 1.0, EPS) + _tol.lipschitz_accel(x1, mass, 1.0,
                                                                          EPS, dx1)
    dv1 = dvh + h * da1 + 2 * U32 * (nrm(vh) + h * nrm(a1))
    _check(N(P), x1, 2 * dx1, "x1")
    _check(N(A), a1, 2 * da1, "a1")
    _check(N(V), v1, 2 * dv1, "v1")


def test_f32_rollout_tracks_fp64(B, dev):
    # 20 KDK steps of N = 1024: the FP32 state stays within 1e-5 (normwise)
    # of the FP64 GPU rollout of the same (FP32-representable) initial state
    # -- per step the state is rounded (u32 ~ 6e-8) and the force carries
    # the FP32 sum error; nothing here is chaotic on this time scale
    pos, vel, mass = _state32(1024, 2300)
    P, V, M = F(pos, dev), F(vel, dev), F(mass, dev)
    A = torch.empty_like(P)
    B.nbody_step_f32(P, V, A, M, 1.0, EPS, DT, 20)
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa
    P6, V6, M6 = T(pos), T(vel), T(mass)
    A6 = torch.empty_like(P6)
    B.nbody_step(P6, V6, A6, M6, 1.0, EPS, DT, 20, "fp64")
    x, x6 = N(P), N(P6)
    v, v6 = N(V), N(V6)
    ex = np.linalg.norm(x - x6) / np.linalg.norm(x6)
    ev = np.linalg.norm(v - v6) / np.linalg.norm(v6)
    say("  f32 vs fp64 rollout: x %.2e v %.2e" % (ex, ev))
    assert ex < 1e-5 and ev < 1e-5
