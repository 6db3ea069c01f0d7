"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Tolerances
  assembly (w, f):     1e-15 relative (same additions in double)
  stencil FP64:        1e-13 relative to max |w| max |p|
  stencil FP32:        4e-6 relative to max |w| max |p| (float inputs, ~7 ops)
  preconditioner FP64: 1e-12 norm-wise (three double GEMMs)
  preconditioner BF16: 1e-2 norm-wise; FP16: 2e-3 norm-wise.  Four roundings to
                       the 16-bit type (input, circulant entries, two
                       intermediates) with unit roundoff u = 2^-9 (BF16) or
                       2^-12 (FP16) bound the error by about 4u.
  solve:               true relative residual <= tol (1e-8) measured by the
                       oracle's own operator; a_hom within 1e-6 relative.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2007_06524_amd as kp  # noqa: E402
from oracle import assembly as asm  # noqa: E402
from oracle import lowrank as lr  # noqa: E402
from oracle.homogenize import homogenized_matrix, solve_correctors  # noqa: E402
from workloads import (cells_bernoulli, cells_lognormal, cells_uniform, config_cells,  # noqa: E402
                       even_factors, random_field)


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


# ----------------------------------------------------------------- assembly
@pytest.mark.parametrize("L,n0", [(2, 4), (3, 2), (4, 4), (5, 3), (12, 4), (33, 4)])
def test_assembly_parity(ctx, L, n0):
    cells = cells_uniform(L, 1.0, 10.0, seed=1000 + L)
    co = kp.Coeff(ctx, cells, n0, "fp64")
    w, f = co.fields()
    wr = asm.edge_weights(cells, n0)
    np.testing.assert_allclose(host(w), wr, rtol=1e-15, atol=0)
    fr = np.stack([asm.corrector_rhs(wr, i) for i in (1, 2, 3)])
    np.testing.assert_allclose(host(f), fr, rtol=0, atol=1e-15 * np.abs(wr).max() / (n0 * L))
    co.free()


# ------------------------------------------------------------------ stencil
@pytest.mark.parametrize("L,n0", [(4, 4), (5, 3), (12, 4), (18, 4), (65, 2), (64, 4)])
def test_stencil_fp64_parity(ctx, L, n0):
    cells = cells_lognormal(L, 1.0, seed=2000 + L)
    N = L * n0
    co = kp.Coeff(ctx, cells, n0, "fp64")
    p = random_field(N, seed=N)
    q = host(kp.stiffness_apply(ctx, co, dev(p)))
    w = asm.edge_weights(cells, n0)
    ref = asm.stiffness_apply(w, p)
    scale = np.abs(w).max() * np.abs(p).max()
    assert np.abs(q - ref).max() <= 1e-13 * scale
    co.free()


@pytest.mark.parametrize("L,n0", [(4, 4), (12, 4), (65, 2), (64, 4)])
def test_stencil_fp32_parity(ctx, L, n0):
    cells = cells_uniform(L, 1.0, 100.0, seed=3000 + L)
    N = L * n0
    co = kp.Coeff(ctx, cells, n0, "mixed_bf16")
    p = random_field(N, seed=N + 1)
    q = host(kp.stiffness_apply(ctx, co, dev(p), precision="mixed_bf16"))
    w = asm.edge_weights(cells, n0)
    ref = asm.stiffness_apply(w, p)
    scale = np.abs(w).max() * np.abs(p).max()
    assert np.abs(q - ref).max() <= 4e-6 * scale
    co.free()


# ----------------------------------------------------------- preconditioner
def _apply_err(ctx, F, prec, seed=5):
    N = F.shape[2]
    pc = kp.Precond(ctx, N, precision=prec, factors=F)
    x = random_field(N, seed=seed)
    z = host(pc.apply(dev(x)))
    ref = lr.kron_apply(F, x)
    pc.free()
    return np.linalg.norm(z - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_precond_single_mode_fp64(ctx, mode):
    """One random mode, the others the identity (u = 1): isolates each GEMM stage."""
    N, R = 16, 1
    F = np.ones((3, R, N))
    F[mode] = even_factors(N, R, seed=mode)[0]
    assert _apply_err(ctx, F, "fp64") <= 1e-13


@pytest.mark.parametrize("N,R", [(8, 1), (16, 3), (24, 2), (48, 7), (64, 5), (72, 4)])
def test_precond_apply_fp64(ctx, N, R):
    assert _apply_err(ctx, even_factors(N, R, seed=N * R), "fp64") <= 1e-12


def test_precond_apply_oracle_factors_fp64(ctx):
    F, _ = lr.canonical_preconditioner(32, 1e-3, 0)
    assert _apply_err(ctx, F, "fp64") <= 1e-12


@pytest.mark.parametrize("prec,tol", [("mixed_bf16", 1e-2), ("mixed_fp16", 2e-3)])
@pytest.mark.parametrize("N,R", [(16, 4), (48, 3), (64, 7), (136, 2)])
def test_precond_apply_16bit(ctx, prec, tol, N, R):
    assert _apply_err(ctx, even_factors(N, R, seed=N + R), prec) <= tol


# -------------------------------------------------------------------- solve
def _oracle_relres(cells, n0, i, x):
    w = asm.edge_weights(cells, n0)
    f = asm.corrector_rhs(w, i)
    return np.linalg.norm(f - asm.stiffness_apply(w, x)) / np.linalg.norm(f)


@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16", "mixed_fp16"])
def test_solve_c1_against_oracle(ctx, prec):
    """16^3 Bernoulli{1,10} checkerboard, rank-4 preconditioner, three correctors."""
    cells = config_cells("c1")
    co = kp.Coeff(ctx, cells, 4, prec)
    pc = kp.Precond(ctx, 16, 1e-3, 4, prec)
    ref = solve_correctors(cells, 4, tol=1e-13)
    phis = []
    for i in (1, 2, 3):
        x, st, status = kp.solve(ctx, co, pc, rhs=i, tol=1e-8)
        assert status == kp.KP_OK
        xh = host(x)
        assert abs(xh.mean()) < 1e-14 * np.abs(xh).max()
        rr = _oracle_relres(cells, 4, i, xh)
        assert rr <= 1e-8, (i, rr, st)
        assert abs(st["relres_true"] - rr) <= 1e-3 * rr + 1e-15
        assert np.linalg.norm(xh - ref["phis"][i - 1]) <= 1e-6 * np.linalg.norm(ref["phis"][i - 1])
        phis.append(x)
    A = kp.homogenized_matrix(ctx, co, phis)
    assert np.abs(A - ref["ahom"]).max() <= 1e-6 * np.abs(ref["ahom"]).max()
    # the library's a_hom formula on the oracle's own solutions is the oracle's
    Ao = kp.homogenized_matrix(ctx, co, [dev(p) for p in ref["phis"]])
    np.testing.assert_allclose(Ao, homogenized_matrix(cells, ref["phis"], ref["fs"]), atol=1e-13)
    co.free()
    pc.free()


@pytest.mark.parametrize("L,n0,law,prec", [(8, 4, "lognormal", "fp64"), (12, 4, "uniform", "fp64"),
                                           (12, 4, "lognormal", "mixed_bf16"),
                                           (16, 4, "bernoulli", "mixed_bf16"),
                                           (9, 3, "uniform", "mixed_fp16")])
def test_solve_against_oracle(ctx, L, n0, law, prec):
    if law == "lognormal":
        cells = cells_lognormal(L, 1.0, seed=L)
    elif law == "uniform":
        cells = cells_uniform(L, 1.0, 10.0, seed=L)
    else:
        cells = cells_bernoulli(L, 1.0, 100.0, 0.5, seed=L)
    N = L * n0
    co = kp.Coeff(ctx, cells, n0, prec)
    pc = kp.Precond(ctx, N, 1e-3, 0, prec)
    ref = solve_correctors(cells, n0, tol=1e-12)
    phis = []
    for i in (1, 2, 3):
        x, st, status = kp.solve(ctx, co, pc, rhs=i, tol=1e-8)
        assert status == kp.KP_OK, st
        rr = _oracle_relres(cells, n0, i, host(x))
        assert rr <= 1e-8, (i, rr, st)
        phis.append(x)
    A = kp.homogenized_matrix(ctx, co, phis)
    assert np.abs(A - ref["ahom"]).max() <= 1e-6 * np.abs(ref["ahom"]).max(), (A, ref["ahom"])
    co.free()
    pc.free()


def test_solve_tight_tolerance_solution(ctx):
    cells = cells_uniform(6, 1.0, 10.0, seed=66)
    co = kp.Coeff(ctx, cells, 4, "fp64")
    pc = kp.Precond(ctx, 24, 1e-3, 0, "fp64")
    ref = solve_correctors(cells, 4, tol=1e-13)
    x, st, status = kp.solve(ctx, co, pc, rhs=2, tol=1e-12)
    assert status == kp.KP_OK
    xh = host(x)
    assert np.abs(xh - ref["phis"][1]).max() <= 1e-9 * np.abs(ref["phis"][1]).max()


def test_c2_full_size_properties(ctx):
    """128^3 uniform[1,10] (FP64): residual by the oracle's operator, a_hom symmetry and bounds."""
    cells = config_cells("c2")
    co = kp.Coeff(ctx, cells, 4, "fp64")
    pc = kp.Precond(ctx, 128, 1e-3, 0, "fp64")
    phis = []
    for i in (1, 2, 3):
        x, st, status = kp.solve(ctx, co, pc, rhs=i, tol=1e-8)
        assert status == kp.KP_OK, st
        phis.append(x)
    rr = _oracle_relres(cells, 4, 1, host(phis[0]))
    assert rr <= 1e-8
    A = kp.homogenized_matrix(ctx, co, phis)
    assert np.abs(A - A.T).max() <= 1e-6 * np.abs(A).max()
    harm, arith = 1.0 / np.mean(1.0 / cells), cells.mean()
    for i in range(3):
        assert harm <= A[i, i] <= arith
    co.free()
    pc.free()


# ------------------------------------------------------- edge cases, errors
def test_errors_and_edge_cases(ctx):
    cells = config_cells("c1")
    bad = cells.copy()
    bad[1, 2, 3] = np.nan
    with pytest.raises(kp.KronPCGError) as e:
        kp.Coeff(ctx, bad, 4)
    assert e.value.status == -1
    bad[1, 2, 3] = -1.0
    with pytest.raises(kp.KronPCGError):
        kp.Coeff(ctx, bad, 4)
    co = kp.Coeff(ctx, cells, 4, "fp64")
    pc = kp.Precond(ctx, 16, 1e-3, 4, "fp64")
    pc8 = kp.Precond(ctx, 8, 1e-3, 2, "fp64")
    with pytest.raises(kp.KronPCGError) as e:
        kp.solve(ctx, co, pc8, rhs=1)
    assert e.value.status == -6
    pcm = kp.Precond(ctx, 16, 1e-3, 4, "mixed_bf16")
    with pytest.raises(kp.KronPCGError) as e:
        kp.solve(ctx, co, pcm, rhs=1)
    assert e.value.status == -6
    # maxit reached
    x, st, status = kp.solve(ctx, co, pc, rhs=1, tol=1e-12, maxit=1)
    assert status == kp.KP_NOT_CONVERGED and st["iters"] == 1
    # zero right-hand side: x = 0, no iteration
    x, st, status = kp.solve(ctx, co, pc, rhs=0, f=torch.zeros((16, 16, 16), dtype=torch.float64, device="cuda"))
    assert status == kp.KP_OK and st["iters"] == 0 and float(x.abs().max()) == 0.0
    # nonzero mean is projected and reported
    f = random_field(16, seed=9) + 3.0
    x, st, status = kp.solve(ctx, co, pc, rhs=0, f=dev(f), tol=1e-9)
    assert status == kp.KP_WARN_RHS_MEAN and abs(st["rhs_mean"] - f.mean()) < 1e-12
    w = asm.edge_weights(cells, 4)
    fz = f - f.mean()
    assert np.linalg.norm(fz - asm.stiffness_apply(w, host(x))) <= 1e-9 * np.linalg.norm(fz)
    # warm start from the solution: converges without iterating
    x1, st1, _ = kp.solve(ctx, co, pc, rhs=1, tol=1e-10)
    x2, st2, status = kp.solve(ctx, co, pc, rhs=1, x=x1.clone(), use_x0=True, tol=1e-8)
    assert status == kp.KP_OK and st2["iters"] == 0
    for o in (co, pc, pc8, pcm):
        o.free()


def test_bitwise_repeatable(ctx):
    cells = cells_lognormal(12, 1.0, seed=7)
    for prec in ("fp64", "mixed_bf16"):
        co = kp.Coeff(ctx, cells, 4, prec)
        pc = kp.Precond(ctx, 48, 1e-3, 0, prec)
        a, sa, _ = kp.solve(ctx, co, pc, rhs=3)
        b, sb, _ = kp.solve(ctx, co, pc, rhs=3)
        assert sa["iters"] == sb["iters"]
        assert torch.equal(a, b)
        co.free()
        pc.free()


def test_coeff_update_and_timing(ctx):
    a = cells_uniform(6, 1.0, 10.0, seed=1)
    b = cells_lognormal(6, 1.0, seed=2)
    co = kp.Coeff(ctx, a, 4, "mixed_bf16")
    ctx.set_timing(True)
    co.update(dev(b))
    w, f = co.fields()
    wr = asm.edge_weights(b, 4)
    np.testing.assert_allclose(host(w), wr, rtol=1e-15, atol=0)
    t = ctx.read_timing()
    assert t["assemble"][1] == 1 and t["assemble"][0] > 0.0
    ctx.set_timing(False)
    bad = b.copy()
    bad[0, 0, 0] = 0.0
    with pytest.raises(kp.KronPCGError):
        co.update(dev(bad))
    w2, _ = co.fields()
    assert torch.equal(w, w2)          # fields unchanged after a rejected update
    co.free()


@pytest.mark.parametrize("N", [72, 96, 128, 256])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed_bf16", 1e-2), ("mixed_fp16", 2e-3)])
def test_every_tile_configuration_matches(ctx, prec, tol, N):
    """The autotuner's candidates all compute the same operator: tune, then check the
    apply with every configuration, on a ragged size (N = 72, R = 3: edge tiles, K not
    a multiple of the K tile), on N = 96 (the circulant-in-LDS kernels with 32-row and
    96-row tiles, three 16-row fragments per wave), on N = 128 (interior tiles) and on
    N = 256 (also the wave-streamed kernels, whose last stage switches between three
    circulants along K)."""
    F = even_factors(N, 3, seed=N)
    pc = kp.Precond(ctx, N, precision=prec, factors=F)
    ncfg = 2 * (4 if prec == "fp64" else 18)     # tile shapes x two block orders
    table = pc.autotune(reps=1)
    assert len(table) == 3 * ncfg and all(t[6] > 0 for t in table)
    assert {t[4] for t in table} == {0, 1}
    if prec != "fp64":
        kinds = {t[5] for t in table}           # 0 streamed, 1 circulant in LDS, 2 wave-streamed
        assert kinds == ({0} if N == 72 else ({0, 1} if N in (96, 128) else {0, 1, 2})), kinds
        # entries name the tile that ran: 96-row tiles only where 96 divides N,
        # 256-row tiles only where 256 does
        rows = {t[1] for t in table}
        assert (96 in rows) == (N == 96) and (256 in rows) == (N == 256), rows
    tuned = pc.tiles
    assert all(0 <= t < ncfg for t in tuned)
    x = random_field(N, seed=8)
    ref = lr.kron_apply(F, x)
    for c in range(ncfg):
        pc.tiles = (c, c, c)
        z = host(pc.apply(dev(x)))
        assert np.linalg.norm(z - ref) / np.linalg.norm(ref) <= tol, c
    with pytest.raises(kp.KronPCGError):
        pc.tiles = (ncfg, 0, 0)
    pc.free()
