"""GPU FFT-diagonalized exact preconditioner (build_preconditioner_fft; the
paper's first approach, Section 4.2) against the oracle.

Tolerances: apply within 1e-12 relative (double FFTs both sides); the solve is
the same textbook PCG as the oracle's with the same exact preconditioner, so
the solutions agree within 1e-9 relative at tol 1e-12 and the iteration
counts within 3 % (plus one): over 150 iterations of CG the different rounding
of the reductions and FFTs moves the count by a few (measured 149 vs 147 on
the log-normal case).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2007_06524_amd as kp  # noqa: E402
from oracle import assembly as asm  # noqa: E402
from oracle import fourier as fo  # noqa: E402
from oracle.pcg import pcg  # noqa: E402
from workloads import cells_lognormal, cells_uniform, random_field  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kp.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("N", [8, 12, 30, 64, 256])
def test_fft_apply_parity(ctx, N):
    pc = kp.Precond(ctx, N, fft=True)
    assert pc.R == 0
    x = random_field(N, seed=N)
    xd = dev(x)
    z = host(pc.apply(xd))
    ref = fo.apply_pinv_laplacian(x)
    assert np.linalg.norm(z - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.array_equal(host(xd), x)          # the input is left intact
    assert pc.autotune(reps=1) == []            # nothing to tune
    pc.free()


def test_fft_exact_preconditioner_one_iteration(ctx):
    """Pin P1: constant coefficient c, any zero-mean f: PCG with the exact
    preconditioner converges in one iteration to the FFT closed form."""
    N, c = 24, 3.5
    co = kp.Coeff(ctx, np.full((6, 6, 6), c), 4, "fp64")
    pc = kp.Precond(ctx, N, fft=True)
    f = random_field(N, seed=3)
    f -= f.mean()
    x, st, status = kp.solve(ctx, co, pc, rhs=0, f=dev(f), tol=1e-10)
    assert status == kp.KP_OK and st["iters"] == 1, st
    u = fo.apply_pinv_laplacian(f) / c
    assert np.abs(host(x) - u).max() <= 1e-12 * np.abs(u).max()
    co.free()
    pc.free()


@pytest.mark.parametrize("L,n0,law", [(6, 4, "uniform"), (8, 4, "lognormal"), (5, 3, "uniform")])
def test_fft_solve_matches_oracle_pcg(ctx, L, n0, law):
    cells = cells_uniform(L, 1.0, 10.0, seed=L) if law == "uniform" else cells_lognormal(L, 1.0, seed=L)
    N = L * n0
    co = kp.Coeff(ctx, cells, n0, "fp64")
    pc = kp.Precond(ctx, N, fft=True)
    w = asm.edge_weights(cells, n0)
    for i in (1, 3):
        f = asm.corrector_rhs(w, i)
        ref = pcg(lambda u: asm.stiffness_apply(w, u), f, fo.apply_pinv_laplacian, tol=1e-12)
        x, st, status = kp.solve(ctx, co, pc, rhs=i, tol=1e-12)
        assert status == kp.KP_OK
        assert abs(st["iters"] - ref["iters"]) <= 1 + ref["iters"] // 33, (st["iters"], ref["iters"])
        assert np.linalg.norm(host(x) - ref["x"]) <= 1e-9 * np.linalg.norm(ref["x"])
    co.free()
    pc.free()


def test_fft_not_for_batched_or_mixed(ctx):
    co = kp.Coeff(ctx, cells_uniform(4, 1.0, 2.0, seed=1), 4, "fp64")
    pc = kp.Precond(ctx, 16, fft=True)
    with pytest.raises(kp.KronPCGError) as e:
        kp.solve_batched(ctx, [co], [pc])
    assert e.value.status == -6
    with pytest.raises(ValueError):
        kp.Precond(ctx, 16, precision="mixed_bf16", fft=True)
    co.free()
    pc.free()
