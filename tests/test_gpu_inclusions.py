"""GPU parity of the sub-cell inclusion coefficient (Section 3.1: the cell value
only on the centred sub-cell of edge 2 alpha / L, a background elsewhere)
against the oracle, through the C ABI.

Tolerances as in test_gpu_parity: assembly 1e-15 relative (the same voxel means
in double), stencil FP64 1e-13 and FP32 4e-6 relative to max |w| max |p|,
solves to a true relative residual 1e-8 by the oracle's operator, a_hom within
1e-6 relative of the oracle's (converged to 1e-12).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2007_06524_amd as kp  # noqa: E402
from oracle import assembly as asm  # noqa: E402
from oracle.homogenize import solve_correctors  # noqa: E402
from workloads import cells_bernoulli, cells_two_contrast, cells_uniform, random_field  # noqa: E402

# (L, n0, incl, background, law): the paper's alpha = 1/4 binary {1, lambda = 0.4}
# (Fig. Emp_a12_M20), a continuous law on a larger sub-cell, and odd ranges.
CASES = [(3, 4, 2, 0.4, "binary"), (4, 4, 2, 0.4, "binary"), (2, 6, 4, 2.0, "uniform"),
         (5, 8, 2, 0.4, "binary"), (3, 5, 3, 1.5, "uniform")]
# N = 256 with n0 = 4: the row-segment stencil kernel
BIG = [(64, 4, 2, 0.4, "binary")]


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


def make_cells(L, law, bg, seed):
    if law == "binary":
        c = cells_bernoulli(L, bg, 1.0, 0.5, seed=seed)
        c[0, 0, 0] = 1.0
        return c
    return cells_uniform(L, 1.0, 10.0, seed=seed)


@pytest.mark.parametrize("L,n0,k,bg,law", CASES)
def test_inclusion_assembly_parity(ctx, L, n0, k, bg, law):
    cells = make_cells(L, law, bg, seed=10 * L + k)
    co = kp.Coeff(ctx, cells, n0, "fp64", inclusion=k, background=bg)
    w, f = co.fields()
    wr = asm.edge_weights(cells, n0, k, bg)
    np.testing.assert_allclose(host(w), wr, rtol=1e-15, atol=0)
    fr = np.stack([asm.corrector_rhs(wr, i) for i in (1, 2, 3)])
    np.testing.assert_allclose(host(f), fr, rtol=0, atol=1e-15 * np.abs(wr).max() / (n0 * L))
    co.free()


@pytest.mark.parametrize("L,n0,k,bg,law", CASES + BIG)
def test_inclusion_stencil_parity(ctx, L, n0, k, bg, law):
    """FP64 and FP32 stencils (weights rebuilt from the cells with the sub-cell
    masks) against the oracle's operator; the FP64 apply also equals the stencil
    of the library's own assembled weights."""
    cells = make_cells(L, law, bg, seed=20 * L + k)
    N = L * n0
    p = random_field(N, seed=N + k)
    w = asm.edge_weights(cells, n0, k, bg)
    ref = asm.stiffness_apply(w, p)
    scale = np.abs(w).max() * np.abs(p).max()
    co = kp.Coeff(ctx, cells, n0, "fp64", inclusion=k, background=bg)
    q = host(kp.stiffness_apply(ctx, co, dev(p)))
    assert np.abs(q - ref).max() <= 1e-13 * scale
    co.free()
    cm = kp.Coeff(ctx, cells, n0, "mixed_bf16", inclusion=k, background=bg)
    q32 = host(kp.stiffness_apply(ctx, cm, dev(p), precision="mixed_bf16"))
    assert np.abs(q32 - ref).max() <= 4e-6 * scale
    cm.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16"])
@pytest.mark.parametrize("L,n0,k,bg,law", [CASES[1], CASES[2], CASES[3]])
def test_inclusion_solve_against_oracle(ctx, prec, L, n0, k, bg, law):
    cells = make_cells(L, law, bg, seed=30 * L + k)
    N = L * n0
    co = kp.Coeff(ctx, cells, n0, prec, inclusion=k, background=bg)
    pc = kp.Precond(ctx, N, 1e-3, 0, prec)
    ref = solve_correctors(cells, n0, tol=1e-12, k=k, background=bg)
    phis = []
    for i in (1, 2, 3):
        x, st, status = kp.solve(ctx, co, pc, rhs=i, tol=1e-8)
        assert status == kp.KP_OK, st
        xh = host(x)
        f = ref["fs"][i - 1]
        rr = np.linalg.norm(f - asm.stiffness_apply(ref["w"], xh)) / np.linalg.norm(f)
        assert rr <= 1e-8, (i, rr, st)
        phis.append(x)
    A = kp.homogenized_matrix(ctx, co, phis)
    assert np.abs(A - ref["ahom"]).max() <= 1e-6 * np.abs(ref["ahom"]).max(), (A, ref["ahom"])
    vox = asm.voxel_field(cells, n0, k, bg)
    for i in range(3):
        assert 1.0 / np.mean(1.0 / vox) <= A[i, i] <= vox.mean()
    co.free()
    pc.free()


@pytest.mark.parametrize("layered", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp16"])
def test_two_contrast_solve_against_oracle(ctx, prec, layered):
    """The two-contrast realizations of Section 2: alpha = 1/4 sub-cell inclusions
    of lambda + 0.3 or lambda + 0.6 on the background lambda = 0.4, the contrast
    drawn per inclusion or set by layers of two cells; solves against the
    oracle's (residual by its operator, a_hom, the mean bounds)."""
    L, n0, k, lam = 4, 4, 2, 0.4
    cells = cells_two_contrast(L, lam, (0.3, 0.6), 0.5, seed=70 + int(layered), layered=layered)
    N = L * n0
    co = kp.Coeff(ctx, cells, n0, prec, inclusion=k, background=lam)
    pc = kp.Precond(ctx, N, 1e-3, 0, prec)
    ref = solve_correctors(cells, n0, tol=1e-12, k=k, background=lam)
    phis = []
    for i in (1, 2, 3):
        x, st, status = kp.solve(ctx, co, pc, rhs=i, tol=1e-8)
        assert status == kp.KP_OK, st
        f = ref["fs"][i - 1]
        assert np.linalg.norm(f - asm.stiffness_apply(ref["w"], host(x))) <= 1e-8 * np.linalg.norm(f)
        phis.append(x)
    A = kp.homogenized_matrix(ctx, co, phis)
    assert np.abs(A - ref["ahom"]).max() <= 1e-6 * np.abs(ref["ahom"]).max(), (A, ref["ahom"])
    vox = asm.voxel_field(cells, n0, k, lam)
    for i in range(3):
        assert 1.0 / np.mean(1.0 / vox) <= A[i, i] <= vox.mean()
    co.free()
    pc.free()


def test_inclusion_batched_mixed_geometries(ctx):
    """One batch holding sub-cell realizations of two geometries and whole-cell
    ones on the same grid (separate groups): every system as the single solve's
    a_hom, the residual by the oracle's operator."""
    n0, L = 4, 4
    pc = kp.Precond(ctx, L * n0, 1e-3, 0, "mixed_bf16")
    specs = [(2, 0.4), (2, 0.4), (4, None), (2, 0.7)]
    cos, cells_list = [], []
    for j, (k, bg) in enumerate(specs):
        cells = make_cells(L, "binary" if bg else "uniform", bg or 0.4, seed=400 + j)
        cells_list.append(cells)
        cos.append(kp.Coeff(ctx, cells, n0, "mixed_bf16", inclusion=k, background=bg))
    xs, stats, A, status = kp.solve_batched(ctx, cos, [pc] * len(cos), tol=1e-8)
    assert status == kp.KP_OK
    for j, (k, bg) in enumerate(specs):
        w = asm.edge_weights(cells_list[j], n0, k, bg)
        for i in (1, 2, 3):
            f = asm.corrector_rhs(w, i)
            x = host(xs[3 * j + i - 1])
            assert np.linalg.norm(f - asm.stiffness_apply(w, x)) <= 1e-8 * np.linalg.norm(f)
        single = [kp.solve(ctx, cos[j], pc, rhs=i, tol=1e-8)[0] for i in (1, 2, 3)]
        As = kp.homogenized_matrix(ctx, cos[j], single)
        assert np.abs(A[j] - As).max() <= 1e-6 * np.abs(As).max()
    for o in cos + [pc]:
        o.free()


def test_inclusion_argument_errors(ctx):
    cells = cells_uniform(2, 1.0, 10.0, seed=1)
    for k, bg in ((3, 0.4), (0, 0.4), (6, 0.4), (2, 0.0), (2, -1.0), (2, float("nan"))):
        with pytest.raises(kp.KronPCGError) as e:
            kp.Coeff(ctx, cells, 4, "fp64", inclusion=k, background=bg)
        assert e.value.status == -1
    # whole cell: background ignored, same fields as setup_coeff
    a = kp.Coeff(ctx, cells, 4, "fp64", inclusion=4, background=-5.0)
    b = kp.Coeff(ctx, cells, 4, "fp64")
    assert torch.equal(a.fields()[0], b.fields()[0])
    a.free()
    b.free()
