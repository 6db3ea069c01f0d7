"""Full-size GPU checks at the sizes the benchmark runs (N = 256) and the large
configuration (N = 512), where the oracle cannot solve: sampled outputs the
oracle computes one by one, the oracle's own operator on the GPU solutions,
and properties that hold at any size.

Tolerances: preconditioner samples 1e-2 relative to the sample RMS of the
exact apply (four 16-bit roundings, as in the small-size tests); true relative
residual <= 1e-8 by the oracle's operator; a_hom of the mixed solve within
1e-6 relative of the plain FP64 GPU solve, symmetric to 1e-6 and inside the
harmonic / arithmetic mean bounds.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2007_06524_amd as kp  # noqa: E402
from oracle import assembly as asm  # noqa: E402
from workloads import config_cells, even_factors, random_field  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kp.Context(0)
    yield c
    c.close()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def circulant_rows(u, js):
    """Rows js of the circulant F* diag(u) F (first column by the DFT of the even symbol)."""
    N = u.shape[0]
    c = np.real(np.fft.ifft(u))
    return np.stack([c[(j - np.arange(N)) % N] for j in js])


def sampled_apply(F, x, points):
    """z(j) = sum_k sum_i C1^k[j1,i1] C2^k[j2,i2] C3^k[j3,i3] x(i) at the given points:
    the i3 contraction of all points and terms is one matrix product, the rest is small."""
    N, R = x.shape[0], F.shape[1]
    P = len(points)
    rows3 = np.concatenate([circulant_rows(F[2, k], [p[2] for p in points]) for k in range(R)])  # (R P, N)
    y = x.reshape(N * N, N) @ rows3.T                                                           # (N^2, R P)
    y = y.reshape(N, N, R, P)
    out = np.zeros(P)
    for k in range(R):
        r1 = circulant_rows(F[0, k], [p[0] for p in points])
        r2 = circulant_rows(F[1, k], [p[1] for p in points])
        for q in range(P):
            out[q] += r1[q] @ (y[:, :, k, q] @ r2[q])
    return out


def check_sampled_apply(pc, N, R, seed):
    F, _ = kp.lowrank_factors(N, 1e-3, R)
    x = random_field(N, seed=seed)
    z = host(pc.apply(torch.from_numpy(x).cuda()))
    g = np.random.default_rng(seed)
    pts = [tuple(int(v) for v in g.integers(0, N, 3)) for _ in range(6)] + [(0, 0, 0), (N - 1, N - 1, N - 1)]
    ref = sampled_apply(F, x, pts)
    got = np.array([z[p] for p in pts])
    assert np.abs(got - ref).max() <= 1e-2 * np.sqrt(np.mean(ref ** 2))


def test_wave_kernels_n512(ctx):
    """N = 512 (16 K steps per circulant, so the wave-streamed kernels keep their
    fragment ring across two turns of their loop) with R = 2: sampled outputs of
    the apply under the circulant-operand tiles, both block orders, against the
    circulant definition."""
    N, R = 512, 2
    F = even_factors(N, R, seed=5120)
    pc = kp.Precond(ctx, N, precision="mixed_bf16", factors=F)
    x = random_field(N, seed=512)
    g = np.random.default_rng(77)
    pts = [tuple(int(v) for v in g.integers(0, N, 3)) for _ in range(6)] + [(0, 0, 0), (N - 1, N - 1, N - 1)]
    ref = sampled_apply(F, x, pts)
    xd = torch.from_numpy(x).cuda()
    ntile = 18                                       # 16-bit tile shapes (cfg = tile + ntile * order)
    for t in (7, 10, 11):
        for order in (0, 1):
            c = t + ntile * order
            pc.tiles = (c, c, c)
            z = pc.apply(xd)
            got = np.array([float(z[p]) for p in pts])
            assert np.abs(got - ref).max() <= 1e-2 * np.sqrt(np.mean(ref ** 2)), (t, order)
    pc.free()


def ahom_bounds_ok(A, cells):
    harm, arith = 1.0 / np.mean(1.0 / cells), cells.mean()
    return all(harm <= A[i, i] <= arith for i in range(3))


@pytest.mark.parametrize("prec", ["mixed_fp16", "mixed_bf16"])
def test_c3_full_size_mixed(ctx, prec):
    """64^3-cell Bernoulli{1,100} checkerboard, N = 256, mixed FP16 (the benchmark's
    precision) and BF16 with the tiles the autotuner picks (the benchmark's launch
    configuration)."""
    cells = config_cells("c3")
    N = 256
    co = kp.Coeff(ctx, cells, 4, prec)
    pc = kp.Precond(ctx, N, 1e-3, 5, prec)
    pc.autotune(reps=1)
    check_sampled_apply(pc, N, 5, seed=256)
    # solves: oracle residual, a_hom against the plain FP64 GPU solve
    phis = []
    for i in (1, 2, 3):
        xs, st, status = kp.solve(ctx, co, pc, rhs=i, tol=1e-8)
        assert status == kp.KP_OK and st["relres_true"] <= 1e-8, st
        phis.append(xs)
    w = asm.edge_weights(cells, 4)
    f1 = asm.corrector_rhs(w, 1)
    assert np.linalg.norm(f1 - asm.stiffness_apply(w, host(phis[0]))) <= 1e-8 * np.linalg.norm(f1)
    del w, f1
    A = kp.homogenized_matrix(ctx, co, phis)
    co64 = kp.Coeff(ctx, cells, 4, "fp64")
    pc64 = kp.Precond(ctx, N, 1e-3, 5, "fp64")
    phis64 = [kp.solve(ctx, co64, pc64, rhs=i, tol=1e-8)[0] for i in (1, 2, 3)]
    A64 = kp.homogenized_matrix(ctx, co64, phis64)
    assert np.abs(A - A64).max() <= 1e-6 * np.abs(A64).max()
    assert np.abs(A - A.T).max() <= 1e-6 * np.abs(A).max() and ahom_bounds_ok(A, cells)
    for o in (co, pc, co64, pc64):
        o.free()


def test_c5_large_mixed(ctx):
    """128^3-cell log-normal (sigma = 1.5) checkerboard, N = 512 (134M unknowns), mixed
    BF16, rank 5.  The largest and smallest of the 2.1M cells differ by a factor of
    about 4e6, so the solve takes thousands of iterations (the bound of Lemma
    Cond_Number grows with the contrast): corrector 1 only, checked by the oracle's
    operator, then refined in plain FP64 from the mixed solution to 5e-9; the first
    row of a_hom (which needs corrector 1 only) agrees between the two."""
    cells = config_cells("c5")
    N = 512
    co = kp.Coeff(ctx, cells, 4, "mixed_bf16")
    pc = kp.Precond(ctx, N, 1e-3, 5, "mixed_bf16")
    assert pc.info["rho_min"] > 0
    pc.autotune(reps=1)
    check_sampled_apply(pc, N, 5, seed=512)
    x, st, status = kp.solve(ctx, co, pc, rhs=1, tol=1e-8, maxit=20000)
    assert status == kp.KP_OK and st["relres_true"] <= 1e-8, st
    A = kp.homogenized_matrix(ctx, co, [x, x, x])
    x1 = host(x)
    co.free()
    pc.free()
    co64 = kp.Coeff(ctx, cells, 4, "fp64")
    pc64 = kp.Precond(ctx, N, 1e-3, 5, "fp64")
    pc64.autotune(reps=1)
    x64, st64, status = kp.solve(ctx, co64, pc64, rhs=1, x=x.clone(), use_x0=True, tol=5e-9, maxit=20000)
    assert status == kp.KP_OK, st64
    A64 = kp.homogenized_matrix(ctx, co64, [x64, x64, x64])
    assert np.abs(A[0] - A64[0]).max() <= 1e-6 * np.abs(A64[0]).max()
    assert ahom_bounds_ok(np.diag([A64[0, 0]] * 3), cells)
    co64.free()
    pc64.free()
    # the oracle's operator on the mixed solution
    w = asm.edge_weights(cells, 4)
    f1 = asm.corrector_rhs(w, 1)
    assert np.linalg.norm(f1 - asm.stiffness_apply(w, x1)) <= 1e-8 * np.linalg.norm(f1)
