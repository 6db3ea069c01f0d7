"""GPU parity of the batched corrector solver (pcg_solve_batched) against the oracle.

Every system must meet the true relative residual 1e-8 by the oracle's own
operator; solutions agree with the oracle's (solved to 1e-12 or 1e-13) to
1e-6 relative and a_hom to 1e-6 relative, as for the single solve.  Several
correct iterate paths exist (the batched control replaces residuals at other
points than the single solver), so iteration counts are not compared.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2007_06524_amd as kp  # noqa: E402
from oracle import assembly as asm  # noqa: E402
from oracle.homogenize import solve_correctors  # noqa: E402
from workloads import batched_realizations, cells_lognormal, cells_uniform  # noqa: E402


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


def relres(cells, n0, i, x):
    w = asm.edge_weights(cells, n0)
    f = asm.corrector_rhs(w, i)
    return np.linalg.norm(f - asm.stiffness_apply(w, x)) / np.linalg.norm(f)


def make_batch(ctx, cells_list, n0, prec, eps=1e-3):
    coeffs = [kp.Coeff(ctx, c, n0, prec) for c in cells_list]
    pcs = {}
    for c in coeffs:
        if c.N not in pcs:
            pcs[c.N] = kp.Precond(ctx, c.N, eps, 0, prec)
    return coeffs, [pcs[c.N] for c in coeffs], list(pcs.values())


def free(*objs):
    for group in objs:
        for o in group:
            o.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16", "mixed_fp16"])
def test_batched_matches_oracle(ctx, prec):
    """Five realizations of uneven L (N = 8, 12, 16, 20, 12), three correctors each."""
    cells_list = batched_realizations(5, sizes=(2, 3, 4, 5), sigma=1.0, seed=40)
    coeffs, pcs, owned = make_batch(ctx, cells_list, 4, prec)
    xs, stats, A, status = kp.solve_batched(ctx, coeffs, pcs, tol=1e-8, check_every=5)
    assert status == kp.KP_OK, stats
    for m, cells in enumerate(cells_list):
        ref = solve_correctors(cells, 4, tol=1e-13)
        for i in (1, 2, 3):
            st = stats[3 * m + i - 1]
            xh = host(xs[3 * m + i - 1])
            assert st["status"] == kp.KP_OK and st["iters"] > 0
            assert abs(xh.mean()) < 1e-13 * np.abs(xh).max()
            rr = relres(cells, 4, i, xh)
            assert rr <= 1e-8, (m, i, rr, st)
            assert abs(st["relres_true"] - rr) <= 1e-3 * rr + 1e-15
            ph = ref["phis"][i - 1]
            assert np.linalg.norm(xh - ph) <= 1e-6 * np.linalg.norm(ph), (m, i)
        assert np.abs(A[m] - ref["ahom"]).max() <= 1e-6 * np.abs(ref["ahom"]).max(), m
    free(coeffs, owned)


def test_batched_agrees_with_single_solves(ctx):
    """Same systems through pcg_solve and pcg_solve_batched (mixed BF16): both meet
    the tolerance, and their a_hom agree to the accuracy the tolerance gives."""
    cells_list = [cells_uniform(3, 1.0, 10.0, seed=s) for s in (1, 2)] + [cells_lognormal(4, 1.0, seed=3)]
    coeffs, pcs, owned = make_batch(ctx, cells_list, 4, "mixed_bf16")
    xs, stats, A, status = kp.solve_batched(ctx, coeffs, pcs, tol=1e-9)
    assert status == kp.KP_OK
    for m, (co, pc) in enumerate(zip(coeffs, pcs)):
        phis = [kp.solve(ctx, co, pc, rhs=i, tol=1e-9)[0] for i in (1, 2, 3)]
        A1 = kp.homogenized_matrix(ctx, co, phis)
        assert np.abs(A1 - A[m]).max() <= 1e-7 * np.abs(A1).max()
        for i in range(3):
            d = torch.linalg.norm(phis[i] - xs[3 * m + i]) / torch.linalg.norm(phis[i])
            assert float(d) <= 1e-6
    free(coeffs, owned)


@pytest.mark.parametrize("check_every", [1, 3, 16])
def test_batched_graph_chunks_give_one_answer(ctx, check_every):
    """The graph replays a chunk of iterations; systems stopped inside a chunk stay
    stopped, so the chunk length changes neither the iterates nor the counts."""
    cells_list = batched_realizations(4, sizes=(2, 3), sigma=1.0, seed=41)
    coeffs, pcs, owned = make_batch(ctx, cells_list, 4, "mixed_bf16")
    xs, stats, A, status = kp.solve_batched(ctx, coeffs, pcs, tol=1e-8, check_every=1)
    xs2, stats2, A2, status2 = kp.solve_batched(ctx, coeffs, pcs, tol=1e-8, check_every=check_every)
    assert status == status2 == kp.KP_OK
    assert [s["iters"] for s in stats] == [s["iters"] for s in stats2]
    for a, b in zip(xs, xs2):
        assert torch.equal(a, b)
    np.testing.assert_array_equal(A, A2)
    free(coeffs, owned)


def test_batched_edge_cases(ctx):
    const = np.full((3, 3, 3), 2.5)
    rough = cells_lognormal(3, 1.0, seed=7)
    coeffs, pcs, owned = make_batch(ctx, [const, rough], 4, "fp64")
    # constant coefficient: f = 0, x = 0 without iterating, a_hom = 2.5 I
    xs, stats, A, status = kp.solve_batched(ctx, coeffs, pcs)
    assert status == kp.KP_OK
    for i in range(3):
        assert stats[i]["iters"] == 0 and stats[i]["status"] == kp.KP_OK
        assert float(xs[i].abs().max()) == 0.0
    np.testing.assert_allclose(A[0], 2.5 * np.eye(3), atol=1e-14)
    # warm start from the solutions: stops without iterating
    xs2, stats2, _, status = kp.solve_batched(ctx, coeffs, pcs, xs=[x.clone() for x in xs], use_x0=True)
    assert status == kp.KP_OK and all(s["iters"] == 0 for s in stats2)
    # iteration limit: not converged, x valid, one iteration each
    xs3, stats3, _, status = kp.solve_batched(ctx, coeffs, pcs, tol=1e-12, maxit=1)
    assert status == kp.KP_NOT_CONVERGED
    assert all(s["status"] == kp.KP_NOT_CONVERGED and s["iters"] == 1 for s in stats3[3:])
    # mismatched sizes and precisions are refused
    pc_other = kp.Precond(ctx, 8, 1e-3, 2, "fp64")
    with pytest.raises(kp.KronPCGError) as e:
        kp.solve_batched(ctx, coeffs, [pcs[0], pc_other])
    assert e.value.status == -6
    cm = kp.Coeff(ctx, rough, 4, "mixed_bf16")
    pm = kp.Precond(ctx, 12, 1e-3, 0, "mixed_bf16")
    with pytest.raises(kp.KronPCGError) as e:
        kp.solve_batched(ctx, [coeffs[1], cm], [pcs[1], pm])
    assert e.value.status == -6
    with pytest.raises(kp.KronPCGError) as e:
        kp.solve_batched(ctx, coeffs, pcs, tol=0.0)
    assert e.value.status == -1
    free(coeffs, owned, [pc_other, cm, pm])


@pytest.mark.parametrize("prec", ["mixed_fp16", "mixed_bf16"])
def test_batched_c4_full_size(ctx, prec):
    """96 log-normal realizations, L cycling over {8, 12, 16, 24} (N = 32 .. 96), mixed
    FP16 (the benchmark's) and BF16: every system converges; sampled systems against
    the oracle; a_hom of every realization symmetric and inside the harmonic /
    arithmetic bounds."""
    cells_list = batched_realizations(96, sizes=(8, 12, 16, 24), sigma=1.0, seed=4)
    coeffs, pcs, owned = make_batch(ctx, cells_list, 4, prec)
    xs, stats, A, status = kp.solve_batched(ctx, coeffs, pcs, tol=1e-8)
    assert status == kp.KP_OK
    assert all(s["status"] == kp.KP_OK and s["relres_true"] <= 1e-8 for s in stats)
    for m in (0, 3):  # one L = 8 (oracle solve) and one L = 24 (oracle residual) realization
        for i in (1, 2, 3):
            assert relres(cells_list[m], 4, i, host(xs[3 * m + i - 1])) <= 1e-8
    ref = solve_correctors(cells_list[0], 4, tol=1e-12)
    assert np.abs(A[0] - ref["ahom"]).max() <= 1e-6 * np.abs(ref["ahom"]).max()
    for m, cells in enumerate(cells_list):
        harm, arith = 1.0 / np.mean(1.0 / cells), cells.mean()
        assert np.abs(A[m] - A[m].T).max() <= 1e-6 * np.abs(A[m]).max()
        assert all(harm <= A[m][i, i] <= arith for i in range(3))
    free(coeffs, owned)


def test_batched_n256_row_kernel(ctx):
    """Two realizations at L = 64 (N = 256, the row-segment stencil kernel with a
    batch of six systems): each system's a_hom as its single solve's."""
    from workloads import cells_bernoulli
    cos, cells = [], []
    for j in range(2):
        c = cells_bernoulli(64, 1.0, 10.0, 0.5, seed=700 + j)
        cells.append(c)
        cos.append(kp.Coeff(ctx, c, 4, "mixed_bf16"))
    pc = kp.Precond(ctx, 256, 1e-3, 5, "mixed_bf16")
    xs, stats, A, status = kp.solve_batched(ctx, cos, [pc, pc], tol=1e-8)
    assert status == kp.KP_OK and all(s["relres_true"] <= 1e-8 for s in stats)
    for j in range(2):
        single = [kp.solve(ctx, cos[j], pc, rhs=i, tol=1e-8)[0] for i in (1, 2, 3)]
        As = kp.homogenized_matrix(ctx, cos[j], single)
        assert np.abs(A[j] - As).max() <= 1e-6 * np.abs(As).max()
    for o in cos + [pc]:
        o.free()
