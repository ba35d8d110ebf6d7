"""Planted mistakes in the oracle must be caught by the pins.

Each case replaces one step of the oracle (on the CPU, through monkeypatch)
with a plausible wrong version -- a dropped term, a wrong sign, a wrong index,
a transposed operand -- and checks that a pin fails:

* cycle-level pins (Arnoldi relation, orthogonality, H against Householder
  Arnoldi, exactness at m = n) on the pin problems, which include two
  near-breakdown problems (clustered spectra) where the second-sweep terms are
  large enough to matter;
* unit-level pins (forward substitution against a library solve, the
  projector identities on a non-orthogonal Q) for the triangular solve,
  whose effect inside a cycle is O(eps^2) because two sweeps keep L = O(eps).

Terms that enter H only at rounding level while V stays orthogonal (the
second-sweep coefficient t in the finished column, the correction in Stephen's
trick) are listed separately: dropping them must leave H unchanged to 1e-12,
which is what the paper's analysis (||L|| = O(eps) with two sweeps) predicts.
"""
import numpy as np
import pytest

import oracle as O
import oracle.arnoldi as OA
import oracle.lsq as OL
import oracle.projector as OP
import workloads as W
from oracle import diagnostics as D


def _pin_problems():
    a, b = W.make_convdiff2d_32()
    s = W.simoncini_diag(100)
    bs = W.rhs_normal(100, 5)
    bs /= np.linalg.norm(bs)
    out = [(a, b, 50, D.norm2(O.as_operator(a)), True), (s, bs, 99, 100.0, True)]
    for spread in (1e-7, 1e-12):
        out.append((W.clustered_spectrum(120, spread=spread, seed=0), W.rhs_normal(120, 1), 14, 13.0, False))
    return out


PINS = _pin_problems()


def _pins_hold(variant, gs):
    """True when every cycle-level pin holds for this variant."""
    try:
        for mat, rhs, m, anorm, compare_h in PINS:
            op = O.as_operator(mat)
            c = O.gmres(mat, rhs, restart=m, tol=0.0, variant=variant, gs_iters=gs, max_cycles=1).first_cycle
            if not np.all(np.isfinite(c.H)):
                return False
            if D.arnoldi_relation_residual(op, c.V, c.H, anorm) > 1e-13:
                return False
            if (variant == "igs1r" or gs == 2) and D.orthogonality_loss(c.V[:, : c.J + 1]) > 1e-13:
                return False
            if compare_h:
                ref = O.gmres(mat, rhs, restart=m, tol=0.0, variant="householder", max_cycles=1).first_cycle
                for col in range(10):
                    d = np.linalg.norm(c.H[: col + 2, col] - ref.H[: col + 2, col])
                    if d > 1e-13 * np.linalg.norm(ref.H[: col + 2, col]):
                        return False
        r = W.random_wellcond(16, 3)
        br = W.rhs_normal(16, 4)
        res = O.gmres(r, br, restart=16, tol=1e-15, variant=variant, gs_iters=gs, maxit=64)
        return bool(np.allclose(res.x, np.linalg.solve(r, br), rtol=1e-12, atol=1e-13))
    except (FloatingPointError, ValueError, np.linalg.LinAlgError, ZeroDivisionError, IndexError):
        return False


def test_pins_hold_unmutated():
    assert _pins_hold("igs1r", 2)
    assert _pins_hold("igs2r", 2)
    assert _pins_hold("igs2r", 1)


# ---- cycle-level mutations: must be caught -------------------------------

MUTATIONS = {
    "column: drop H correction": ("finish_column_1r", lambda H, j, r1p, t, tp, gp: r1p + t),
    "column: wrong sign of correction":
        ("finish_column_1r", lambda H, j, r1p, t, tp, gp: r1p + t + H[:j, : j - 1] @ (tp / gp)),
    "column: t_prev not scaled": ("finish_column_1r", lambda H, j, r1p, t, tp, gp: r1p + t - H[:j, : j - 1] @ tp),
    "column: wrong row block of H":
        ("finish_column_1r", lambda H, j, r1p, t, tp, gp: r1p + t - H[1:j + 1, : j - 1] @ (tp / gp)),
    "column: drop first-sweep coefficients":
        ("finish_column_1r", lambda H, j, r1p, t, tp, gp: t - H[:j, : j - 1] @ (tp / gp)),
    "trick: wrong sign": ("stephen_trick", lambda q, b, t, g: np.concatenate([q, [b + (t / g) @ q]])),
    "trick: unscaled t": ("stephen_trick", lambda q, b, t, g: np.concatenate([q, [b - t @ q]])),
    "trick: last coefficient dropped": ("stephen_trick", lambda q, b, t, g: np.concatenate([q, [0.0]])),
    "lagged norm: wrong sign": ("lagged_norm_sq", lambda alpha, p: alpha + float(p @ p)),
    "lagged norm: correction dropped": ("lagged_norm_sq", lambda alpha, p: alpha),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_one_reduce_mutations_caught(monkeypatch, name):
    attr, bad = MUTATIONS[name]
    monkeypatch.setattr(OA, attr, bad)
    assert not _pins_hold("igs1r", 2), name


@pytest.mark.parametrize("variant,gs", [("igs1r", 2), ("igs2r", 2), ("igs2r", 1)])
@pytest.mark.parametrize("which", ["q from u", "beta from u", "alpha squared"])
def test_reduction_mutations_caught(monkeypatch, variant, gs, which):
    orig = OA.one_reduction

    def bad(Vt_old, u, z):
        p, alpha, q, beta = orig(Vt_old, u, z)
        if which == "alpha squared":
            return p, alpha * alpha, q, beta
        if q is None:
            return p, alpha, q, beta
        if which == "q from u":
            q = Vt_old @ u
        else:
            beta = float(u @ u)
        return p, alpha, q, beta

    monkeypatch.setattr(OA, "one_reduction", bad)
    assert not _pins_hold(variant, gs)


def _back_sub_off_by_one(R, g):
    k = g.shape[0]
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - R[i, i:k - 1] @ y[i + 1:k]) / R[i, i]
    return y


def test_back_substitution_off_by_one_caught(monkeypatch):
    monkeypatch.setattr(OL, "back_substitution", _back_sub_off_by_one)
    assert not _pins_hold("igs1r", 2)


def test_givens_sign_caught(monkeypatch):
    orig = OL.GivensLS.add_column

    def bad(self, c, h):
        out = orig(self, c, h)
        self.sn[c] = -self.sn[c]
        return out

    monkeypatch.setattr(OL.GivensLS, "add_column", bad)
    assert not _pins_hold("igs1r", 2)


# ---- triangular-solve mutations: caught by the unit pins --------------------

def _fwd_transposed(L, r):
    x = np.array(r, dtype=np.float64, copy=True)
    for i in range(r.shape[0]):
        x[i] = r[i] - L[:i, i] @ x[:i]
    return x


def _fwd_plus(L, r):
    x = np.array(r, dtype=np.float64, copy=True)
    for i in range(r.shape[0]):
        x[i] = r[i] + L[i, :i] @ x[:i]
    return x


def _fwd_off_by_one(L, r):
    x = np.array(r, dtype=np.float64, copy=True)
    for i in range(r.shape[0]):
        k = max(i - 1, 0)
        x[i] = r[i] - L[i, :k] @ x[:k]
    return x


@pytest.mark.parametrize("bad", [_fwd_transposed, _fwd_plus, _fwd_off_by_one],
                         ids=["transposed L", "wrong sign", "off by one"])
def test_forward_substitution_mutations_caught_by_unit_pins(monkeypatch, bad):
    import test_oracle_primitives as P
    monkeypatch.setattr(OP, "forward_subst_unit_lower", bad)
    monkeypatch.setattr(O, "forward_subst_unit_lower", bad)
    monkeypatch.setattr(P.O, "forward_subst_unit_lower", bad)
    failed = 0
    for pin in (P.test_forward_substitution_against_library_solve,
                P.test_projector_identities_exact_algebra,
                P.test_projector_two_sweeps_matches_T2):
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed >= 2


# ---- rounding-level terms: harmless by the analysis -------------------------

ROUNDING_LEVEL = {
    "column: drop t": ("finish_column_1r", lambda H, j, r1p, t, tp, gp: r1p - H[:j, : j - 1] @ (tp / gp)),
    "trick: drop correction": ("stephen_trick", lambda q, b, t, g: np.concatenate([q, [b]])),
    "cycle: transposed L in the triangular solve": ("forward_subst_unit_lower", _fwd_transposed),
}


@pytest.mark.parametrize("name", sorted(ROUNDING_LEVEL))
def test_rounding_level_terms(monkeypatch, name):
    attr, bad = ROUNDING_LEVEL[name]
    mat, rhs, m, anorm, _ = PINS[0]
    ref = O.gmres(mat, rhs, restart=m, tol=0.0, variant="igs1r", max_cycles=1).first_cycle
    monkeypatch.setattr(OA, attr, bad)
    mut = O.gmres(mat, rhs, restart=m, tol=0.0, variant="igs1r", max_cycles=1).first_cycle
    for col in range(m):
        assert np.linalg.norm(mut.H[: col + 2, col] - ref.H[: col + 2, col]) <= \
            1e-12 * np.linalg.norm(ref.H[: col + 2, col])


# ---- diagnostics: planted mistakes caught by their pins ---------------------

def _run_pins(pins):
    failed = 0
    for pin, args in pins:
        try:
            pin(*args)
        except AssertionError:
            failed += 1
    return failed


BACKWARD_ERROR_MUTATIONS = {
    "denominator without ||b||":
        lambda op, b, x, an: np.linalg.norm(b - op.matvec(x)) / (an * np.linalg.norm(x)),
    "denominator without ||A|| ||x||":
        lambda op, b, x, an: np.linalg.norm(b - op.matvec(x)) / np.linalg.norm(b),
    "||A|| dropped from the denominator":
        lambda op, b, x, an: np.linalg.norm(b - op.matvec(x)) / (np.linalg.norm(b) + np.linalg.norm(x)),
    "squared norms":
        lambda op, b, x, an: float((b - op.matvec(x)) @ (b - op.matvec(x)))
        / (float(b @ b) + an * an * float(x @ x)),
    "residual with the wrong sign of A x":
        lambda op, b, x, an: np.linalg.norm(b + op.matvec(x)) / (np.linalg.norm(b) + an * np.linalg.norm(x)),
}


@pytest.mark.parametrize("name", sorted(BACKWARD_ERROR_MUTATIONS))
def test_backward_error_mutations_caught(monkeypatch, name):
    import test_oracle_primitives as P
    monkeypatch.setattr(D, "backward_error", BACKWARD_ERROR_MUTATIONS[name])
    pins = [(P.test_backward_error_rigal_gaches_construction, (k,)) for k in range(3)]
    pins.append((P.test_backward_error_hand_computed_2x2, ()))
    assert _run_pins(pins) >= 2, name


GS_RADIUS_MUTATIONS = {
    "L not transposed": lambda L: float(np.max(np.abs(np.linalg.eigvals(
        -np.linalg.solve(np.eye(L.shape[0]) + L, L))))) if L.shape[0] else 0.0,
    "Jacobi matrix": lambda L: float(np.max(np.abs(np.linalg.eigvals(-(L + L.T))))) if L.shape[0] else 0.0,
    "wrong sign inside (I - L)": lambda L: float(np.max(np.abs(np.linalg.eigvals(
        -np.linalg.solve(np.eye(L.shape[0]) - L, L.T))))) if L.shape[0] else 0.0,
    "no inverse": lambda L: float(np.max(np.abs(np.linalg.eigvals(-L.T)))) if L.shape[0] else 0.0,
}


@pytest.mark.parametrize("name", sorted(GS_RADIUS_MUTATIONS))
def test_gs_spectral_radius_mutations_caught(monkeypatch, name):
    import test_oracle_primitives as P
    monkeypatch.setattr(D, "gs_spectral_radius", GS_RADIUS_MUTATIONS[name])
    pins = [(P.test_gs_spectral_radius_closed_form_2x2, ()),
            (P.test_gs_spectral_radius_young_tridiagonal, ()),
            (P.test_gs_spectral_radius_small_for_near_orthogonal_basis, ()),
            (P.test_gs_spectral_radius_is_the_sweep_contraction_rate, ())]
    assert _run_pins(pins) >= 1, name
