"""One restart cycle of the Arnoldi-QR process, in four variants.

Every variant builds the Arnoldi pair of Section 1 (eq:arnoldi):
``v_0 = r0 / rho``, ``A V_J = V_{J+1} H_{J+1,J}`` with ``H`` upper Hessenberg
and positive subdiagonal, and reduces ``H`` with Givens rotations so that the
cycle can stop as soon as the Arnoldi residual ``|g_J|`` reaches the absolute
tolerance.  Indices here are 0-based: iteration ``j`` normalises basis vector
``j`` and finishes Hessenberg column ``j - 1``.

Variants
--------
cycle_mgs
    Textbook modified Gram-Schmidt Arnoldi (Saad and Schultz): ``j`` inner
    products, one after the other, for column ``j``.
cycle_householder
    Walker's Householder Arnoldi, the independent reference whose ``H`` all
    Gram-Schmidt variants must reproduce (Arnoldi is unique once the
    subdiagonal is positive).
cycle_igs_2r
    Algorithm 4.1 (two-reduce IGS-GMRES).  The unnormalised vector ``w_j`` is
    multiplied by ``A`` first; one reduction returns ``V^T w``, ``w^T w``,
    ``V^T A w`` and ``w^T A w``; the normalisation of ``w_j`` is lagged into
    this iteration; the last row of ``L`` is ``V^T w / gamma``; the first
    Gauss-Seidel sweep solves with ``I + L``.  With ``gs_iters=2`` a second
    reduction and sweep follow (steps 14-16) and the column is ``r1 + r3``
    (step 17); with ``gs_iters=1`` the column is ``r1``.
cycle_igs_1r
    Algorithm 4.2 (one-reduce hybrid MGS-CGS GMRES), read as follows where the
    printed listing is ambiguous: the reduction is
    ``[V_{0:j}, u_j]^T [u_j, A u_j]``; the second sweep of vector ``j`` is
    ``t = (I + L_{0:j,0:j})^{-1} V^T u_j`` (Gauss-Seidel; ``jacobi=True``
    takes ``t = V^T u_j`` instead); the lagged norm is
    ``gamma^2 = u^T u - p^T p``; ``v_j = (u_j - V t) / gamma`` uses the same
    ``t``; the stored row of ``L`` is ``p / gamma``; Stephen's trick gives the
    last first-sweep coefficient as ``(u^T A u - t^T q) / gamma^2``; and the
    column finished at iteration ``j`` is column ``j - 1``:
    ``H[0:j, j-1] = r1_prev + t - H[0:j, 0:j-1] (t_prev / gamma_prev)``,
    ``H[j, j-1] = gamma`` (from eq:Aw with the previous column's ``r1``).

Stopping, breakdown and the lagged-norm guard (the paper is silent on them):
a cycle ends after ``m`` columns, when ``|g_J| <= tol_abs``, when the
iteration budget is used up, or on breakdown ``gamma_j <= n eps ||H[0:j,
j-1]||``.  For the one-reduce variant, when ``u^T u - p^T p < tau u^T u`` the
norm is recomputed explicitly as ``||u - V t||`` (one extra reduction), the
column is finished with it, and the cycle ends so that the next cycle restarts
from the true residual.

Pinned by: tests/test_oracle_arnoldi.py -- the Arnoldi relation, O(eps)
orthogonality for two sweeps and visible loss for one sweep / MGS on the
ill-conditioned diagonal matrix, ``H`` equal to Householder-Arnoldi ``H``,
the lagged norm against the explicit norm, monotone Arnoldi residuals; and
tests/test_oracle_mutations.py, which plants mistakes in these steps and
checks that the pins catch them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .lsq import GivensLS
from .projector import forward_subst_unit_lower

EPS = np.finfo(np.float64).eps


@dataclass
class StopRule:
    """When a cycle ends (see module docstring)."""

    tol_abs: float = 0.0          # stop when |g_J| <= tol_abs
    its_left: int = 1 << 62       # iterations left in the solve's budget
    lagnorm_tau: float = 1e-4     # one-reduce lagged-norm cancellation guard


@dataclass
class CycleResult:
    V: np.ndarray                 # n x (J+1): v_0 .. v_J (v_J valid unless breakdown)
    H: np.ndarray                 # (J+1) x J, before rotation
    J: int                        # finished columns
    y: np.ndarray                 # least-squares solution (J)
    rho: float                    # ||r0||
    res_hist: np.ndarray          # |g_c| for c = 1..J (Arnoldi residual norms)
    status: str                   # "maxcols" | "converged" | "breakdown" | "lagnorm" | "maxit"
    L: np.ndarray | None = None   # strictly lower correction matrix (IGS variants)
    gammas: np.ndarray | None = None
    lagnorm_fallbacks: int = 0
    extra: dict = field(default_factory=dict)


def _breakdown(gamma: float, hcol: np.ndarray, n: int) -> bool:
    return gamma <= n * EPS * float(np.sqrt(hcol @ hcol))


def _pack(Vt, H, L, J, gls, rho, res, status, gammas, fallbacks=0):
    return CycleResult(V=Vt[: J + 1].T, H=H[: J + 1, :J].copy(), J=J, y=gls.solve(J),
                       rho=rho, res_hist=np.array(res), status=status,
                       L=None if L is None else L[: J + 1, : J + 1].copy(),
                       gammas=np.array(gammas), lagnorm_fallbacks=fallbacks)


# ---------------------------------------------------------------------------
# Modified Gram-Schmidt Arnoldi (textbook reference)
# ---------------------------------------------------------------------------

def cycle_mgs(op, r0: np.ndarray, m: int, stop: StopRule) -> CycleResult:
    n = r0.size
    rho = math.sqrt(r0 @ r0)
    Vt = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    Vt[0] = r0 / rho
    gls = GivensLS(m, rho)
    res, gammas = [], [rho]
    for c in range(m):
        w = op.matvec(Vt[c])
        for i in range(c + 1):
            H[i, c] = Vt[i] @ w
            w = w - H[i, c] * Vt[i]
        gamma = math.sqrt(w @ w)
        H[c + 1, c] = gamma
        gammas.append(gamma)
        res.append(gls.add_column(c, H[: c + 2, c]))
        if _breakdown(gamma, H[: c + 1, c], n):
            return _pack(Vt, H, None, c + 1, gls, rho, res, "breakdown", gammas)
        Vt[c + 1] = w / gamma
        if res[-1] <= stop.tol_abs:
            return _pack(Vt, H, None, c + 1, gls, rho, res, "converged", gammas)
        if c + 1 >= stop.its_left:
            return _pack(Vt, H, None, c + 1, gls, rho, res, "maxit", gammas)
    return _pack(Vt, H, None, m, gls, rho, res, "maxcols", gammas)


# ---------------------------------------------------------------------------
# Householder Arnoldi (independent reference for H)
# ---------------------------------------------------------------------------

def householder_arnoldi(op, r0: np.ndarray, m: int):
    """Walker's Householder Arnoldi; returns (V, H) with A V_m = V_{m+1} H.

    Signs are those the reflections produce; ``canonical_signs`` makes the
    first vector ``r0/||r0||`` and the subdiagonal positive.
    """
    n = r0.size
    W = np.zeros((m + 1, n))
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    z = np.array(r0, dtype=np.float64, copy=True)
    alpha0 = 0.0
    for j in range(m + 1):
        if j == n:
            # the Krylov space is the whole space: the last column is exact
            H[:n, n - 1] = z
            H[n, n - 1] = 0.0
            break
        x = z[j:]
        nx = math.sqrt(x @ x)
        alpha = -nx if x[0] >= 0 else nx
        w = np.zeros(n)
        w[j:] = x
        w[j] -= alpha
        nw = math.sqrt(w @ w)
        if nw > 0:
            w /= nw
        W[j] = w
        pz = np.zeros(j + 1)
        pz[:j] = z[:j]
        pz[j] = alpha
        if j == 0:
            alpha0 = alpha
        else:
            H[: j + 1, j - 1] = pz
        v = np.zeros(n)
        v[j] = 1.0
        for i in range(j, -1, -1):
            v -= 2.0 * W[i] * (W[i] @ v)
        V[:, j] = v
        if j < m:
            z = op.matvec(v)
            for i in range(j + 1):
                z -= 2.0 * W[i] * (W[i] @ z)
    return V, H, alpha0


def canonical_signs(V: np.ndarray, H: np.ndarray, first_sign: float):
    """Return (V S, S H S) with S = diag(+-1) making v_0 and the subdiagonal positive."""
    k = H.shape[1]
    s = np.ones(k + 1)
    s[0] = 1.0 if first_sign >= 0 else -1.0
    for i in range(k):
        s[i + 1] = (1.0 if H[i + 1, i] >= 0 else -1.0) * s[i]
    return V * s[None, :], (s[:, None] * H) * s[None, : k]


def cycle_householder(op, r0: np.ndarray, m: int, stop: StopRule) -> CycleResult:
    n = r0.size
    rho = math.sqrt(r0 @ r0)
    V, H, a0 = householder_arnoldi(op, r0, m)
    V, H = canonical_signs(V, H, a0)
    gls = GivensLS(m, rho)
    res = []
    J, status = m, "maxcols"
    for c in range(m):
        res.append(gls.add_column(c, H[: c + 2, c]))
        if _breakdown(H[c + 1, c], H[: c + 1, c], n):
            J, status = c + 1, "breakdown"
            break
        if res[-1] <= stop.tol_abs:
            J, status = c + 1, "converged"
            break
        if c + 1 >= stop.its_left:
            J, status = c + 1, "maxit"
            break
    return CycleResult(V=V[:, : J + 1], H=H[: J + 1, :J].copy(), J=J, y=gls.solve(J),
                       rho=rho, res_hist=np.array(res), status=status)


# ---------------------------------------------------------------------------
# Steps shared by the two IGS variants (module-level so tests can plant errors)
# ---------------------------------------------------------------------------

def one_reduction(Vt_old: np.ndarray, u: np.ndarray, z):
    """The single global reduction [V_old, u]^T [u, z].

    Returns ``(p, alpha, q, beta)`` = ``(V^T u, u^T u, V^T z, u^T z)``;
    ``q`` and ``beta`` are None when ``z`` is None (the tail iteration).
    """
    p = Vt_old @ u
    alpha = float(u @ u)
    if z is None:
        return p, alpha, None, None
    return p, alpha, Vt_old @ z, float(u @ z)


def finish_column_1r(H: np.ndarray, j: int, r1_prev, t, t_prev, gamma_prev):
    """H[0:j, j-1] = r1_prev + t - H[0:j, 0:j-1] (t_prev / gamma_prev)  (eq:Aw)."""
    return r1_prev + t - H[:j, : j - 1] @ (t_prev / gamma_prev)


def stephen_trick(q_scaled: np.ndarray, beta_scaled: float, t: np.ndarray, gamma: float):
    """First-sweep coefficients of A v_j against [V_{0:j}, v_j].

    ``q_scaled = V^T A u / gamma`` and ``beta_scaled = u^T A u / gamma^2``; the
    last coefficient is ``v_j^T A u / gamma = beta_scaled - (t/gamma)^T q_scaled``.
    """
    last = beta_scaled - (t / gamma) @ q_scaled
    return np.concatenate([q_scaled, [last]])


def normalise_after_second_sweep(Vt_old: np.ndarray, u: np.ndarray, t: np.ndarray,
                                 gamma: float) -> np.ndarray:
    """v_j = (u_j - V_{0:j} t) / gamma (steps 10-11 of Algorithm 4.2)."""
    return (u - Vt_old.T @ t) / gamma


def first_sweep_next(Vt_new: np.ndarray, z: np.ndarray, gamma: float, r1: np.ndarray) -> np.ndarray:
    """u_{j+1} = A u_j / gamma - V_{0:j+1} r1 (step 13 of Algorithm 4.2)."""
    return z / gamma - Vt_new.T @ r1


def lagged_norm_sq(alpha: float, p: np.ndarray) -> float:
    """||u - V V^T u||^2 by Pythagoras: u^T u - p^T p (step 6 of Algorithm 4.2)."""
    return alpha - float(p @ p)


# ---------------------------------------------------------------------------
# Algorithm 4.1: two-reduce IGS-GMRES (gs_iters = 1 or 2)
# ---------------------------------------------------------------------------

def cycle_igs_2r(op, r0: np.ndarray, m: int, stop: StopRule, gs_iters: int = 2) -> CycleResult:
    if gs_iters not in (1, 2):
        raise ValueError("gs_iters must be 1 or 2")
    n = r0.size
    Vt = np.zeros((m + 1, n))        # row j holds w_j until it is normalised
    H = np.zeros((m + 1, m))
    L = np.zeros((m + 1, m + 1))
    Vt[0] = r0
    gls = None
    res, gammas = [], []
    h_prev = None
    rho = 0.0
    for j in range(m + 1):
        w = Vt[j].copy()
        z = op.matvec(w) if j < m else None                 # step 4: A w_{j}
        c, alpha, q, beta = one_reduction(Vt[:j], w, z)     # step 5 + norm of step 6
        gamma = math.sqrt(alpha)                            # step 6
        gammas.append(gamma)
        if j == 0:
            rho = gamma
            gls = GivensLS(m, rho)
        else:
            H[:j, j - 1] = h_prev
            H[j, j - 1] = gamma
            res.append(gls.add_column(j - 1, H[: j + 1, j - 1]))
            if _breakdown(gamma, H[:j, j - 1], n):
                return _pack(Vt, H, L, j, gls, rho, res, "breakdown", gammas)
        Vt[j] = w / gamma                                   # step 7: lagged normalisation
        if j > 0 and res[-1] <= stop.tol_abs:
            return _pack(Vt, H, L, j, gls, rho, res, "converged", gammas)
        if j == m:
            return _pack(Vt, H, L, m, gls, rho, res, "maxcols", gammas)
        if j >= stop.its_left:
            return _pack(Vt, H, L, j, gls, rho, res, "maxit", gammas)
        L[j, :j] = c / gamma                                # step 10
        qs = q / gamma                                      # step 8
        bs = beta / gamma / gamma                           # steps 8-9
        zs = z / gamma                                      # step 11
        Lj = L[: j + 1, : j + 1]
        r1 = forward_subst_unit_lower(Lj, np.concatenate([qs, [bs]]))   # step 12
        u = zs - Vt[: j + 1].T @ r1                         # step 13: first sweep
        if gs_iters == 2:
            r2 = Vt[: j + 1] @ u                            # step 14: second reduction
            r3 = forward_subst_unit_lower(Lj, r2)           # step 15
            Vt[j + 1] = u - Vt[: j + 1].T @ r3              # step 16: second sweep
            h_prev = r1 + r3                                # step 17
        else:
            Vt[j + 1] = u
            h_prev = r1
    raise AssertionError("unreachable")


# ---------------------------------------------------------------------------
# Algorithm 4.2: one-reduce hybrid MGS-CGS GMRES
# ---------------------------------------------------------------------------

def cycle_igs_1r(op, r0: np.ndarray, m: int, stop: StopRule, jacobi: bool = False) -> CycleResult:
    n = r0.size
    Vt = np.zeros((m + 1, n))        # row j holds u_j until it is normalised
    H = np.zeros((m + 1, m))
    L = np.zeros((m + 1, m + 1))
    Vt[0] = r0
    gls = None
    res, gammas = [], []
    fallbacks = 0
    r1_prev = t_prev = None
    gamma_prev = 0.0
    rho = 0.0
    for j in range(m + 1):
        u = Vt[j].copy()
        z = op.matvec(u) if j < m else None                 # A u_j (used by step 13)
        p, alpha, q, beta = one_reduction(Vt[:j], u, z)     # step 4: one reduction
        t = p.copy() if jacobi else forward_subst_unit_lower(L[:j, :j], p)   # step 5
        fallback = False
        if j == 0:
            gamma = math.sqrt(alpha)
            rho = gamma
            gls = GivensLS(m, rho)
        else:
            g2 = lagged_norm_sq(alpha, p)                   # step 6: lagged norm
            if g2 < stop.lagnorm_tau * alpha:
                wexp = u - Vt[:j].T @ t                     # guard: explicit norm
                gamma = math.sqrt(wexp @ wexp)
                fallback = True
                fallbacks += 1
            else:
                gamma = math.sqrt(g2)
        gammas.append(gamma)
        if j > 0:                                           # steps 14-15: finish column j-1
            H[:j, j - 1] = finish_column_1r(H, j, r1_prev, t, t_prev, gamma_prev)
            H[j, j - 1] = gamma
            res.append(gls.add_column(j - 1, H[: j + 1, j - 1]))
            if _breakdown(gamma, H[:j, j - 1], n):
                return _pack(Vt, H, L, j, gls, rho, res, "breakdown", gammas, fallbacks)
        L[j, :j] = p / gamma                                # step 9
        Vt[j] = normalise_after_second_sweep(Vt[:j], u, t, gamma)   # steps 10-11
        if j > 0 and res[-1] <= stop.tol_abs:
            return _pack(Vt, H, L, j, gls, rho, res, "converged", gammas, fallbacks)
        if fallback:
            return _pack(Vt, H, L, j, gls, rho, res, "lagnorm", gammas, fallbacks)
        if j == m:
            return _pack(Vt, H, L, m, gls, rho, res, "maxcols", gammas, fallbacks)
        if j >= stop.its_left:
            return _pack(Vt, H, L, j, gls, rho, res, "maxit", gammas, fallbacks)
        qs = q / gamma                                      # step 7
        bs = beta / gamma / gamma                           # steps 7-8
        r1 = stephen_trick(qs, bs, t, gamma)                # step 12
        Vt[j + 1] = first_sweep_next(Vt[: j + 1], z, gamma, r1)     # step 13
        r1_prev, t_prev, gamma_prev = r1, t, gamma
    raise AssertionError("unreachable")
