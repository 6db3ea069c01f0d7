"""Pins of the oracle's solve and homogenized matrix: closed forms, invariants,
bounds, brute force (Sections 3.4, 4.1, 5.2)."""

import numpy as np
import pytest

from oracle import assembly as asm
from oracle import fourier as fo
from oracle import lowrank as lr
from oracle.dense import dense_solve
from oracle.homogenize import (homogenized_energy, homogenized_flux, homogenized_matrix,
                               solve_correctors)
from oracle.pcg import lanczos_ritz_values, pcg
from workloads import cells_bernoulli, cells_uniform, random_field


def _zero_mean(u):
    return u - u.mean()


def test_constant_coefficient_closed_form():
    """a = c: correctors vanish, a_hom = c I; PCG with the exact preconditioner
    needs one iteration and returns the FFT closed form (Section 4.1)."""
    c = 2.75
    cells = np.full((3, 3, 3), c)
    res = solve_correctors(cells, 2)
    for f in res["fs"]:
        assert np.abs(f).max() < 1e-15
    np.testing.assert_allclose(res["ahom"], c * np.eye(3), atol=1e-14)
    w = res["w"]
    f = _zero_mean(random_field(6, seed=4))
    out = pcg(lambda u: asm.stiffness_apply(w, u), f, fo.apply_pinv_laplacian, tol=1e-12)
    assert out["iters"] == 1
    closed = fo.apply_symbol(fo.pinv_symbol(6) / c, f)
    np.testing.assert_allclose(out["x"], closed, atol=1e-13)


def test_manufactured_solution():
    cells = cells_uniform(4, 1.0, 10.0, seed=21)
    w = asm.edge_weights(cells, 3)
    ustar = _zero_mean(random_field(12, seed=22))
    f = asm.stiffness_apply(w, ustar)
    out = pcg(lambda u: asm.stiffness_apply(w, u), f, fo.apply_pinv_laplacian, tol=1e-13)
    assert out["converged"] and out["relres"] <= 1e-13
    assert np.linalg.norm(out["x"] - ustar) <= 1e-10 * np.linalg.norm(ustar)


@pytest.mark.parametrize("L,n0", [(2, 2), (2, 3), (3, 2)])
def test_dense_brute_force(L, n0):
    cells = cells_uniform(L, 1.0, 10.0, seed=31 + L * n0)
    res = solve_correctors(cells, n0, tol=1e-13)
    for i in range(3):
        ref = dense_solve(cells, n0, res["fs"][i])
        assert np.abs(ref.mean()) < 1e-12
        np.testing.assert_allclose(res["phis"][i], ref, atol=1e-10 * max(1e-300, np.abs(ref).max()))


def test_symmetry_and_identities():
    cells = cells_bernoulli(3, 1.0, 10.0, 0.5, seed=41)
    res = solve_correctors(cells, 3, tol=1e-12)
    A = res["ahom"]
    assert np.abs(A - A.T).max() < 1e-9 * np.abs(A).max()
    # flux form of the definition equals the linear form identically
    np.testing.assert_allclose(homogenized_flux(res["w"], res["phis"]), A, atol=1e-13)
    rnd = [random_field(9, seed=s) for s in (1, 2, 3)]
    np.testing.assert_allclose(homogenized_flux(res["w"], rnd),
                               homogenized_matrix(cells, rnd, res["fs"]), atol=1e-12)
    # energy form equals the linear form at the solution
    for i in range(3):
        assert abs(homogenized_energy(res["w"], res["phis"][i], i + 1) - A[i, i]) < 1e-9


def test_bounds_harmonic_arithmetic():
    """harmonic(a) <= 1/mean(1/w_i) <= a_ii <= mean(a)."""
    cells = cells_uniform(4, 1.0, 10.0, seed=51)
    res = solve_correctors(cells, 2, tol=1e-12)
    harm = 1.0 / np.mean(1.0 / cells)
    arith = cells.mean()
    for i in range(3):
        reuss = 1.0 / np.mean(1.0 / res["w"][i])
        assert harm <= reuss + 1e-14
        assert reuss <= res["ahom"][i, i] + 1e-10
        assert res["ahom"][i, i] <= arith + 1e-14


def test_laminate_exact():
    """a(c) = g(c1): a_11 = harmonic mean of g, a_22 = a_33 = arithmetic mean."""
    g = np.array([1.0, 7.0, 3.0, 0.5])
    cells = np.broadcast_to(g[:, None, None], (4, 4, 4)).copy()
    res = solve_correctors(cells, 2, tol=1e-13)
    A = res["ahom"]
    assert abs(A[0, 0] - 1.0 / np.mean(1.0 / g)) < 1e-10
    assert abs(A[1, 1] - g.mean()) < 1e-12 and abs(A[2, 2] - g.mean()) < 1e-12
    off = A - np.diag(np.diag(A))
    assert np.abs(off).max() < 1e-12


def test_checkerboard_2d_keller_dykhne():
    """x3-invariant regular 2D checkerboard {1, 4}: a_hom -> sqrt(1*4) = 2 as n0 grows."""
    cells = np.zeros((2, 2, 2))
    for c1 in range(2):
        for c2 in range(2):
            cells[c1, c2, :] = 1.0 if (c1 + c2) % 2 == 0 else 4.0
    errs = []
    for n0 in (4, 8, 16):
        A = solve_correctors(cells, n0, tol=1e-11)["ahom"]
        assert abs(A[0, 0] - A[1, 1]) < 1e-9
        assert abs(A[2, 2] - 2.5) < 1e-12
        assert abs(A[0, 1]) < 1e-9
        errs.append(A[0, 0] - 2.0)
    assert errs[0] > errs[1] > errs[2] > 0
    assert errs[2] < 0.03
    assert 1.5 < errs[1] / errs[2] < 3.0     # first order in h


def test_ritz_values_within_coefficient_range():
    """Lemma Cond_Number: x^T K x / x^T A_Delta x lies in [min w, max w], so the
    Ritz values of the exactly preconditioned operator do too."""
    cells = cells_bernoulli(4, 1.0, 10.0, 0.5, seed=61)
    w = asm.edge_weights(cells, 2)
    f = asm.corrector_rhs(w, 1)
    out = pcg(lambda u: asm.stiffness_apply(w, u), f, fo.apply_pinv_laplacian, tol=1e-10)
    ritz = lanczos_ritz_values(out["alphas"], out["betas"])
    assert ritz.min() >= w.min() * (1 - 1e-8)
    assert ritz.max() <= w.max() * (1 + 1e-8)


def test_prefactor_invariance():
    """The (1+lambda)/2 prefactor of B_Delta does not change the iterates (Section 4.1)."""
    cells = cells_uniform(3, 1.0, 10.0, seed=71)
    w = asm.edge_weights(cells, 2)
    f = asm.corrector_rhs(w, 2)
    K = lambda u: asm.stiffness_apply(w, u)
    a = pcg(K, f, fo.apply_pinv_laplacian, tol=1e-12)
    b = pcg(K, f, lambda r: 0.7 * fo.apply_pinv_laplacian(r), tol=1e-12)
    assert a["iters"] == b["iters"]
    np.testing.assert_allclose(a["history"], b["history"], rtol=1e-7)
    np.testing.assert_allclose(a["x"], b["x"], atol=1e-12 * np.abs(a["x"]).max())


def test_invariances_scaling_shift_permutation_reflection():
    cells = cells_uniform(3, 1.0, 10.0, seed=81)
    base = solve_correctors(cells, 2, tol=1e-12)
    A = base["ahom"]
    # scaling: phi unchanged, a_hom scales
    sc = solve_correctors(3.0 * cells, 2, tol=1e-12)
    np.testing.assert_allclose(sc["ahom"], 3.0 * A, rtol=1e-9)
    np.testing.assert_allclose(sc["phis"][0], base["phis"][0], atol=1e-9 * np.abs(base["phis"][0]).max())
    # whole-cell cyclic shift: a_hom unchanged
    sh = solve_correctors(np.roll(cells, 1, axis=1), 2, tol=1e-12)
    np.testing.assert_allclose(sh["ahom"], A, atol=1e-9)
    # axis permutation permutes a_hom
    perm = (2, 0, 1)
    pm = solve_correctors(np.transpose(cells, perm), 2, tol=1e-12)
    np.testing.assert_allclose(pm["ahom"], A[np.ix_(perm, perm)], atol=1e-9)
    # reflection x1 -> -x1 flips the sign of a_1j, j != 1
    rf = solve_correctors(cells[::-1].copy(), 2, tol=1e-12)
    S = np.diag([-1.0, 1.0, 1.0])
    np.testing.assert_allclose(rf["ahom"], S @ A @ S, atol=1e-9)


def test_paper_iteration_count_binary_contrast():
    """Section 5.2: at most 20 PCG iterations to 1e-7 (binary lambda = 0.4 contrast)."""
    cells = cells_bernoulli(8, 0.4, 1.0, 0.5, seed=91)
    w = asm.edge_weights(cells, 4)
    K = lambda u: asm.stiffness_apply(w, u)
    F, info = lr.canonical_preconditioner(32, 1e-3, 0)
    GR = lr.symbol_from_factors(F)
    for i in (1, 2, 3):
        f = asm.corrector_rhs(w, i)
        ex = pcg(K, f, fo.apply_pinv_laplacian, tol=1e-7)
        assert ex["converged"] and ex["iters"] <= 20
        lowrank = pcg(K, f, lambda r: fo.apply_symbol(GR, r), tol=1e-7)
        assert lowrank["converged"] and lowrank["iters"] <= 20


def test_lowrank_and_exact_preconditioner_same_solution():
    cells = cells_bernoulli(4, 1.0, 10.0, 0.5, seed=1)
    w = asm.edge_weights(cells, 4)
    K = lambda u: asm.stiffness_apply(w, u)
    f = asm.corrector_rhs(w, 1)
    F, _ = lr.canonical_preconditioner(16, 1e-3, 4)
    a = pcg(K, f, fo.apply_pinv_laplacian, tol=1e-12)
    b = pcg(K, f, lambda r: lr.kron_apply(F, r), tol=1e-12)
    np.testing.assert_allclose(a["x"], b["x"], atol=1e-10 * np.abs(a["x"]).max())


def test_inclusion_bounds_and_forms():
    """Sub-cell inclusions (alpha = 1/4, binary {1, lambda = 0.4}, the paper's
    Fig. Emp_a12_M20 setting): the corrector system still satisfies the
    harmonic / arithmetic bounds of the voxel field, the flux form equals the
    linear form, and the energy form equals the diagonal at the solution."""
    b = 0.4
    cells = cells_bernoulli(3, b, 1.0, 0.5, seed=61)
    res = solve_correctors(cells, 4, tol=1e-12, k=2, background=b)
    A = res["ahom"]
    vox = asm.voxel_field(cells, 4, 2, b)
    harm, arith = 1.0 / np.mean(1.0 / vox), vox.mean()
    for i in range(3):
        assert harm - 1e-12 <= A[i, i] <= arith + 1e-12
        assert homogenized_energy(res["w"], res["phis"][i], i + 1) == pytest.approx(A[i, i], rel=1e-9)
    np.testing.assert_allclose(homogenized_flux(res["w"], res["phis"]), A, atol=1e-12)
    np.testing.assert_allclose(A, A.T, atol=1e-10)


def test_empirical_statistics():
    """eq. A_hom_Empir and the M - 1 standard deviation: identical realizations give
    the value itself and zero spread; scaling every realization scales both; the
    entries equal numpy's mean and ddof = 1 standard deviation; order does not matter."""
    from oracle.homogenize import empirical_statistics
    g = np.random.default_rng(5)
    A = g.random((7, 3, 3))
    mean, std = empirical_statistics(A)
    np.testing.assert_allclose(mean, A.mean(axis=0), rtol=1e-15)
    np.testing.assert_allclose(std, A.std(axis=0, ddof=1), rtol=1e-13)
    m2, s2 = empirical_statistics(3.0 * A[::-1])
    np.testing.assert_allclose(m2, 3.0 * mean, rtol=1e-14)
    np.testing.assert_allclose(s2, 3.0 * std, rtol=1e-13)
    m3, s3 = empirical_statistics(np.stack([A[0]] * 4))
    np.testing.assert_allclose(m3, A[0], rtol=1e-15)
    assert np.all(s3 < 1e-15)
    # two realizations: std = |a - b| / sqrt(2)
    _, s4 = empirical_statistics(A[:2])
    np.testing.assert_allclose(s4, np.abs(A[0] - A[1]) / np.sqrt(2.0), rtol=1e-13)
    with pytest.raises(ValueError):
        empirical_statistics(A[:1])


def test_statistics_decay_rate():
    """eq. var: the standard deviation of a_hom over realizations decays like
    L^(-d/2) in the RVE size.  Oracle on whole cells (n0 = 1), Bernoulli{1, 10},
    M = 64 realizations at L = 4, 8, 16: the fitted log-log slope of sigma_L^M
    of a_11 lies within 0.4 of -3/2, and the empirical average barely moves
    (its change is within a few standard errors)."""
    from oracle.homogenize import empirical_statistics
    from workloads import mc_realizations
    Ls, sig, means = (4, 8, 16), [], []
    for L in Ls:
        cells = mc_realizations(L, 64, 1.0, 10.0, 0.5, seed=7)
        A = np.stack([solve_correctors(c, 1, tol=1e-10)["ahom"] for c in cells])
        m, s = empirical_statistics(A)
        sig.append(s[0, 0])
        means.append(m[0, 0])
    slope = np.polyfit(np.log(Ls), np.log(sig), 1)[0]
    assert -1.9 <= slope <= -1.1, slope
    assert abs(means[2] - means[1]) <= 4 * (sig[1] + sig[2]) / np.sqrt(64)
