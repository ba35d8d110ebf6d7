"""Pins for the oracle's Arnoldi cycles against what the paper and the
mathematics fix: the Arnoldi relation, orthogonality levels, uniqueness of H
(Householder Arnoldi as the independent reference), lagged vs explicit norms."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import diagnostics as D

GS_VARIANTS = [("igs1r", 2), ("igs2r", 2), ("igs2r", 1), ("mgs", 1)]


def first_cycle(a, b, m, variant, gs, tol=0.0, **kw):
    return O.gmres(a, b, restart=m, tol=tol, variant=variant, gs_iters=gs, max_cycles=1, **kw).first_cycle


def problems():
    """(name, matrix, rhs, restart, 2-norm) of the pinned test problems."""
    out = []
    a, b = W.make_convdiff2d_32()
    out.append(("convdiff2d_32", a, b, 50, D.norm2(O.as_operator(a))))
    s = W.simoncini_diag(100)
    bs = W.rhs_normal(100, 5)
    out.append(("simoncini", s, bs / np.linalg.norm(bs), 99, 100.0))
    wk = W.walker(10, 2000.0)
    out.append(("walker", wk, np.ones(10), 9, float(np.linalg.norm(wk, 2))))
    e = W.embree_bidiag(100, 0.1)
    out.append(("embree", e, W.rhs_normal(100, 3), 14, float(np.linalg.norm(e, 2))))
    r = W.random_wellcond(64, 11)
    out.append(("random64", r, W.rhs_normal(64, 12), 30, float(np.linalg.norm(r, 2))))
    # near-breakdown: six eigenvalue clusters of width 1e-12, subdiagonal ~5e-10 at step 6
    cl = W.clustered_spectrum(120, spread=1e-12, seed=0)
    out.append(("clustered", cl, W.rhs_normal(120, 1), 14, float(np.linalg.norm(cl, 2))))
    return out


PROBLEMS = problems()


@pytest.mark.parametrize("variant,gs", GS_VARIANTS + [("householder", 1)])
@pytest.mark.parametrize("prob", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_arnoldi_relation(prob, variant, gs):
    """A V_J = V_{J+1} H to O(eps) ||A|| (eq:arnoldi; backward stability section)."""
    name, a, b, m, anorm = prob
    c = first_cycle(a, b, m, variant, gs)
    assert c.J == m or c.status == "breakdown"
    if c.status == "breakdown":
        pytest.skip("cycle ended on breakdown; relation checked on the other problems")
    res = D.arnoldi_relation_residual(O.as_operator(a), c.V, c.H, anorm)
    assert res < 1e-13, (name, variant, gs, res)
    # first vector is r0/rho and the subdiagonal is positive
    assert np.allclose(c.V[:, 0], b / np.linalg.norm(b), atol=1e-15)
    assert np.all(np.diag(c.H, -1) > 0)


@pytest.mark.parametrize("variant", ["igs1r", "igs2r"])
@pytest.mark.parametrize("prob", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_two_sweeps_keep_orthogonality(prob, variant):
    """||I - V^T V||_F = O(eps) with two Gauss-Seidel sweeps (Sections 3-4)."""
    name, a, b, m, _ = prob
    c = first_cycle(a, b, m, variant, 2)
    assert D.orthogonality_loss(c.V[:, : c.J + 1]) < 1e-13, name


@pytest.mark.parametrize("variant,gs", [("mgs", 1), ("igs2r", 1)])
def test_one_sweep_loses_orthogonality_on_simoncini(variant, gs):
    """One sweep (MGS) loses orthogonality ~ eps kappa(B_k) on the ill-conditioned diagonal."""
    _, a, b, _, _ = PROBLEMS[1]
    c = first_cycle(a, b, 99, variant, gs)
    assert D.orthogonality_loss(c.V[:, : c.J + 1]) > 0.1
    # while the two-sweep variants stay at working precision on the same run
    c2 = first_cycle(a, b, 99, "igs1r", 2)
    assert D.orthogonality_loss(c2.V[:, : c2.J + 1]) < 1e-13


# Tolerance on H against Householder Arnoldi.  Two sweeps keep V orthogonal to
# O(eps), so H agrees to rounding; one sweep (MGS, Algorithm 4.1 with one
# iteration) loses orthogonality ~ eps kappa(B_k) (the one-sweep bound of
# Section 3), and B_k grows ill-conditioned as fast as the residual falls
# (Embree: 0.1^k).  Walker's non-normal matrix makes H itself sensitive at
# the 1e-9 level for every method, Householder included.
# Past the near-breakdown of the clustered problem (subdiagonal 5e-10 at step
# 6) the next basis vector is determined only to ~eps / 5e-10 by any method,
# so H is compared up to that step there.
H_TOL = {("walker", 2): 1e-8, ("walker", 1): 1e-8, ("embree", 1): 1e-6, ("random64", 1): 1e-9,
         ("clustered", 1): 1e-12, ("clustered", 2): 1e-12}
H_COLS = {"clustered": 6}


@pytest.mark.parametrize("variant,gs", GS_VARIANTS)
@pytest.mark.parametrize("prob", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_H_matches_householder_arnoldi(prob, variant, gs):
    """H is unique given v_0 and a positive subdiagonal: compare with Householder Arnoldi."""
    name, a, b, m, _ = prob
    sweeps = 2 if variant == "igs1r" or gs == 2 else 1
    tol = H_TOL.get((name, sweeps), 1e-13)
    k = min(10, m, H_COLS.get(name, m))
    ref = first_cycle(a, b, m, "householder", 1).H
    H = first_cycle(a, b, m, variant, gs).H
    for col in range(k):
        d = np.linalg.norm(H[: col + 2, col] - ref[: col + 2, col])
        assert d <= tol * np.linalg.norm(ref[: col + 2, col]), (name, col, d)


def test_lagged_norm_agrees_with_explicit_norm():
    """The one-reduce lagged gamma_j agrees with the two-reduce explicit ||w_j|| (Sec.5)."""
    for name, a, b, m, _ in PROBLEMS:
        c1 = first_cycle(a, b, m, "igs1r", 2)
        c2 = first_cycle(a, b, m, "igs2r", 2)
        k = min(c1.J, c2.J, H_COLS.get(name, m))
        g1, g2 = np.diag(c1.H, -1)[:k], np.diag(c2.H, -1)[:k]
        big = g2 > 1e-8 * np.max(g2)
        assert np.allclose(g1[big], g2[big], rtol=1e-11), name


def test_jacobi_reading_agrees():
    """t = V^T u (Jacobi) and t = (I+L)^{-1} V^T u (Gauss-Seidel) agree to rounding here."""
    _, a, b, m, anorm = PROBLEMS[0]
    c_gs = first_cycle(a, b, m, "igs1r", 2)
    c_j = first_cycle(a, b, m, "igs1r", 2, jacobi=True)
    assert np.allclose(c_gs.H, c_j.H, rtol=1e-12, atol=1e-13 * anorm)


@pytest.mark.parametrize("prob", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_arnoldi_residual_monotone(prob):
    """The Arnoldi residual decreases monotonically without stagnation (two sweeps)."""
    name, a, b, m, _ = prob
    c = first_cycle(a, b, m, "igs1r", 2)
    h = c.res_hist
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-12) + 1e-300), name


def test_L_is_the_loss_of_orthogonality_two_reduce():
    """For Algorithm 4.1, L_{j,0:j} = v_j^T V_{0:j} (the relation V^T V = I + L + L^T)."""
    _, a, b, m, _ = PROBLEMS[0]
    c = first_cycle(a, b, m, "igs2r", 2)
    G = c.V.T @ c.V
    L = c.L
    assert np.allclose(np.tril(G, -1)[: c.J, : c.J], L[: c.J, : c.J], atol=1e-15)


def test_tail_iteration_and_m_equals_n():
    """Full GMRES (m = n): the tail iteration breaks down exactly at the last column."""
    a = W.random_wellcond(16, 3)
    b = W.rhs_normal(16, 4)
    for variant, gs in GS_VARIANTS:
        c = first_cycle(a, b, 16, variant, gs)
        assert c.J == 16
        assert c.status in ("breakdown", "maxcols")
