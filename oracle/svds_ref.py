"""FP64 CPU oracle of the augmented, restarted Lanczos-bidiagonalization
truncated SVD (the method of Sec. 2.1: Alg. 1, Proposition 1, eqs. (2)-(7),
Alg. 2).

TEST INFRASTRUCTURE: this package is the CPU oracle.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does.  Plain NumPy/SciPy in float64, written for
readability, not speed: every step is done the way the paper states it, with
library primitives (sparse mat-vec, dense mat-vec, LAPACK gesvd) as the steps.

Readings of the paper used here (where it is silent or ambiguous):

* Re-orthogonalisation (Sec. 2.1, text after Alg. 1, and the remark after
  Alg. 2 that step 10 needs it too): classical Gram-Schmidt applied twice
  (CGS2) to the unnormalised vector, before its norm becomes alpha or beta.
* LBP(A, t+1) (Alg. 2 step 2) is run until v_{t+1} and beta_t exist; u_{t+1}
  and alpha_{t+1} are never used, so they are not formed.  Mat-vec count:
  2t for the first LBP, 2(t-k) per restart.
* An SVD of T(1:t,1:t) follows every Lanczos cycle; at most ``maxit`` cycles
  (maxit-1 restarts).  The output is formed from the last SVD.
* Convergence test (eq. (4), Alg. 2 step 5): |beta_t Uh(t,j)| / sigma_j < tol
  for every j <= k, strict; sigma_j is floored at max(2^-52 sigma_1,
  smallest normal) so a zero singular value cannot divide by zero.
* Breakdown (norm after CGS2 <= 1e-14 * sigma_est, sigma_est = largest
  alpha, beta or sigma_1 seen so far): the vector is replaced by a Philox
  normal vector (stream 1 + number of earlier breakdowns), re-orthogonalised
  by CGS2 against the same basis, normalised, and 0 is stored in T.
* Signs: each output pair (u_j, v_j) is flipped so that the entry of v_j of
  largest magnitude (lowest index on ties) is positive.
* Selective second pass (``selective=True``; eq. (8) counts one projection
  per vector): after h = Q^T w, w1 = w - Q h, the second pass runs only when
  |w1|^2 < |w|^2 / 2 (Daniel-Gragg-Kaufman-Stewart test); otherwise w1 is
  the re-orthogonalised vector.  Breakdown replacement vectors still get
  both passes.
* Smallest triplets (``which="smallest"``; Sec. 1 notes that the
  bidiagonalization also approximates the smallest singular values): the
  same cycle with the k smallest Ritz triplets of T kept instead of the k
  largest (eqs. (5)-(7) hold for any k Ritz triplets), returned in ascending
  order.  The sigma floor of eq. (4) still uses the largest Ritz value.
  ``harmonic=False`` restarts with the k smallest Ritz vectors (plain Ritz
  augmentation).
* Harmonic-Ritz augmentation (``which="smallest", harmonic=True``; the
  augmented restart of Baglama and Reichel that Sec. 1 cites, for the
  smallest values).  The convergence test and the outputs stay those of the
  Ritz triplets of T (eq. (4) holds for them at any cycle); only the restart
  subspace changes.  With A V_t = U_t T and A^T U_t = V_t T^T + beta_t
  v_{t+1} e_t^T, the harmonic Ritz values of A^T A on span(V_t) are the
  squared singular values of B = [T, beta_t e_t] (t x (t+1)); for the k
  smallest, with right singular vectors y_j of B, the harmonic Ritz vectors
  are V_t g_j, g_j = y_j(1:t) + beta_t y_j(t+1) z, z = T^{-1} e_t, and all
  their residuals (for A^T A) are parallel to f = v_{t+1} - beta_t V_t z.
  The restart keeps span{V_t g_1..V_t g_k, f} = V_{t+1} span{y_1..y_k, y_0}
  with y_0 the null vector of B ([-beta_t z; 1] normalized): the same
  subspace, written with B's orthonormal right singular vectors and no
  solve with T.  M = [y_1..y_k, y_0] is turned by the Householder
  reflection H that maps its last row r onto e_{k+1} (H r^T = -sign(r_{k+1})
  |r| e_{k+1}), so Q_C = M H has a zero last row in its first k columns
  (those lie in span(V_t)); its last column is taken with a positive last
  entry.  V becomes V_{t+1} Q_C and U_k = U_t Q_M with Q_M = [x_1..x_k] the
  matching left singular vectors of B (B y_j = s_j x_j): since
  B Q_C(:, 1:k) = [s_1 x_1 .. s_k x_k, B y_0] H(:, 1:k) and B y_0 = 0,
  A V_k = U_k R_M with R_M = Q_M^T B Q_C(:, 1:k) (k x k, in general full),
  and A^T U_k = V_{t+1} B^T Q_M = V_{t+1} [y_1 s_1 .. y_k s_k] lies in the
  kept span; both relations inherit only the backward error of the SVD of
  B, whatever the size of s_j.  (Building U_k from the QR of T Q_C(1:t,
  1:k) instead spans the same space in exact arithmetic, but its rounding
  errors are amplified by |B| / s_k, which for small wanted values stalls
  the eq. (4) test.)  The new T starts as R_M.  The restart vector u_{k+1}
  is A v_{k+1} re-orthogonalized (CGS2) against U_k, its two projections'
  coefficients summed into T(1:k, k+1) (A V_{k+1} = U_{k+1} T(1:k+1,
  1:k+1)); the Lanczos steps then go on from k+1 as usual.

* Partial re-orthogonalisation (``partial=True``; the PROPACK-style
  alternative that Sec. 1 names): instead of re-orthogonalising every new
  vector against its whole basis, the loss of orthogonality of the newest
  vector against each earlier one of its side is estimated by recurrences
  that follow from the two Lanczos relations A V = U T and A^T U = V T^T
  (see ``_omega_v`` / ``_omega_u``), plus a local rounding term
  EPS * sigma_est per step divided by the new norm.  When an estimate
  exceeds sqrt(EPS), the vector is re-orthogonalised by CGS2 against the
  earlier vectors whose estimate exceeds EPS^(3/4), those estimates are reset
  to EPS, and the next vector of the same side is re-orthogonalised against
  the same set as well (its estimates grew from the same pair).  The restart
  vector of eq. (7) is re-orthogonalised against all k kept vectors, as in
  the full mode; the estimates of v_{k+1} = v_{p+1} against the kept Ritz
  vectors are the old estimates rotated by the same right singular vectors.

t (the paper's Lanczos dimension) is called p here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .philox import normal_vector

BREAKDOWN_REL = 1e-14
TINY = np.finfo(np.float64).tiny
EPS = 2.0 ** -52
OMEGA_TRIGGER = EPS ** 0.5   # an estimate above this triggers a re-orthogonalisation
OMEGA_SELECT = EPS ** 0.75   # ... against the earlier vectors whose estimate is above this


@dataclass
class SvdsInfo:
    cycles: int = 0
    restarts: int = 0
    n_spmv: int = 0        # products A x
    n_spmvT: int = 0       # products A^T y
    breakdowns: int = 0
    converged: bool = False
    nconv: int = 0
    res_est: np.ndarray = field(default_factory=lambda: np.zeros(0))
    sigma_est: float = 0.0
    reorth_tests: int = 0          # selective mode: tests made
    reorth_second_passes: int = 0  # ... and second passes run
    partial_steps: int = 0         # partial mode: vectors re-orthogonalised ...
    partial_columns: int = 0       # ... against this many basis columns in all
    partial_possible: int = 0      # ... out of this many (the full mode's count)
    harmonic_restarts: int = 0     # harmonic mode: restarts with harmonic Ritz vectors


class _Op:
    """A as the two products the method needs; counts every call."""

    def __init__(self, A, info: SvdsInfo):
        self.A = A
        self.AT = A.T
        self.info = info
        self.m, self.n = A.shape

    def mv(self, x):
        self.info.n_spmv += 1
        return np.asarray(self.A @ x, dtype=np.float64).ravel()

    def rmv(self, y):
        self.info.n_spmvT += 1
        return np.asarray(self.AT @ y, dtype=np.float64).ravel()


def cgs2(w: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Full re-orthogonalisation w <- (I - Q Q^T) w, done twice (CGS2)."""
    if Q.shape[1] == 0:
        return w
    for _ in range(2):
        h = Q.T @ w
        w = w - Q @ h
    return w


def cgs_selective(w: np.ndarray, Q: np.ndarray):
    """One classical Gram-Schmidt pass, and a second one only when the first
    removed more than 1/sqrt(2) of the norm (|w1|^2 < |w|^2 / 2).
    Returns (vector, second pass taken)."""
    if Q.shape[1] == 0:
        return w, False
    w1 = w - Q @ (Q.T @ w)
    if float(w1 @ w1) >= 0.5 * float(w @ w):
        return w1, False
    return w1 - Q @ (Q.T @ w1), True


def omega_v_inner(T, mu, nu, i):
    """v_l^T w for l <= i, w = A^T u_i - T(i,i) v_i (the unnormalised v_{i+1},
    0-based), from the inner products mu[r] = u_r^T u_i (mu[i] = 1) and
    nu[l] = v_l^T v_i (nu[i] = 1): A V = U T gives A v_l = sum_r T(r,l) u_r,
    so v_l^T A^T u_i = sum_{r<=l} T(r,l) mu[r]."""
    return np.array([T[:l + 1, l] @ mu[:l + 1] - T[i, i] * nu[l] for l in range(i + 1)])


def omega_u_inner(T, mu, nu, i):
    """u_l^T w for l < i, w = A v_i - T(i-1,i) u_{i-1} (the unnormalised u_i),
    from nu[c] = v_c^T v_i (nu[i] = 1) and mu[l] = u_l^T u_{i-1}
    (mu[i-1] = 1): A^T U = V T^T (rows up to i-1) gives
    A^T u_l = sum_c T(l,c) v_c, so u_l^T A v_i = sum_{c<=i} T(l,c) nu[c]."""
    return np.array([T[l, :i + 1] @ nu[:i + 1] - T[i - 1, i] * mu[l] for l in range(i)])


class _State:
    """Workspace of one solve: U (m x p), V (n x (p+1)), T ((p+1) x (p+1))."""

    def __init__(self, op: _Op, p: int, seed: int, info: SvdsInfo, selective: bool = False,
                 partial: bool = False):
        self.op = op
        self.p = p
        self.seed = seed
        self.info = info
        self.selective = selective
        self.partial = partial
        self.U = np.zeros((op.m, p), order="F")
        self.V = np.zeros((op.n, p + 1), order="F")
        self.T = np.zeros((p + 1, p + 1))
        # partial mode: estimates of u_i^T u_l and v_i^T v_l for the newest
        # u_i and v_i against every earlier vector of their side (entry i = 1),
        # and the columns the next vector of each side must be taken against
        self.mu = np.zeros(p + 1)
        self.nu = np.zeros(p + 2)
        self.force_u = np.zeros(0, dtype=int)
        self.force_v = np.zeros(0, dtype=int)

    def _finish(self, w, Q):
        """CGS2 (or the selective form) against Q, norm, breakdown handling;
        returns (vector, norm)."""
        if self.selective and Q.shape[1] > 0:
            w, second = cgs_selective(w, Q)
            self.info.reorth_tests += 1
            self.info.reorth_second_passes += int(second)
        else:
            w = cgs2(w, Q)
        nrm = float(np.linalg.norm(w))
        if nrm <= BREAKDOWN_REL * self.info.sigma_est:
            self.info.breakdowns += 1
            r = normal_vector(w.shape[0], self.seed, self.info.breakdowns)
            r = cgs2(r, Q)
            return r / np.linalg.norm(r), 0.0
        self.info.sigma_est = max(self.info.sigma_est, nrm)
        return w / nrm, nrm

    def u_step(self, i, w, full=False):
        """u_i from w (0-based column i): re-orthogonalise against U[:, :i]
        (partial mode, unless ``full``: against the columns the estimates pick)."""
        if self.partial and not full and i > 0:
            self.U[:, i], a = self._partial(w, self.U, i, self._omega_u(i, w), "u")
        else:
            self.U[:, i], a = self._finish(w, self.U[:, :i])
            self.mu[:i] = EPS
        self.mu[i] = 1.0
        self.T[i, i] = a

    def v_step(self, i):
        """Alg. 1 steps 5-6: v_{i+1} = A^T u_i - alpha_i v_i, reorth, beta_i."""
        w = self.op.rmv(self.U[:, i]) - self.T[i, i] * self.V[:, i]
        if self.partial:
            self.V[:, i + 1], b = self._partial(w, self.V, i + 1, self._omega_v(i, w), "v")
        else:
            self.V[:, i + 1], b = self._finish(w, self.V[:, :i + 1])
        self.nu[i + 1] = 1.0
        self.T[i, i + 1] = b

    # --- partial re-orthogonalisation ---------------------------------------
    def _rounding(self, x, nrm):
        """Local rounding term of one step, with the sign of the estimate."""
        return (x + np.where(x >= 0, 1.0, -1.0) * EPS * self.info.sigma_est) / nrm

    def _omega_v(self, i, w):
        nrm = float(np.linalg.norm(w))
        x = omega_v_inner(self.T, self.mu, self.nu, i)
        return self._rounding(x, nrm) if nrm > 0 else np.full(i + 1, np.inf)

    def _omega_u(self, i, w):
        nrm = float(np.linalg.norm(w))
        x = omega_u_inner(self.T, self.mu, self.nu, i)
        return self._rounding(x, nrm) if nrm > 0 else np.full(i, np.inf)

    def _partial(self, w, Q, j, om, side):
        """Re-orthogonalise w against the columns of Q[:, :j] that the
        estimates ``om`` pick (plus the set forced by the previous vector of
        this side); store the new estimate row; return (vector, norm)."""
        forced = self.force_u if side == "u" else self.force_v
        self.info.partial_possible += j
        if np.all(np.abs(om) <= OMEGA_TRIGGER) and forced.size == 0:
            sel = np.zeros(0, dtype=int)
            nxt = sel
        else:
            sel = np.union1d(np.flatnonzero(np.abs(om) > OMEGA_SELECT), forced[forced < j]).astype(int)
            nxt = sel if np.any(np.abs(om) > OMEGA_TRIGGER) else np.zeros(0, dtype=int)
        nrm0 = float(np.linalg.norm(w))
        if sel.size:
            self.info.partial_steps += 1
            self.info.partial_columns += sel.size
            w = cgs2(w, Q[:, sel])
        nrm = float(np.linalg.norm(w))
        if nrm <= BREAKDOWN_REL * self.info.sigma_est:
            # invariant subspace: the full form (CGS2 against the whole basis,
            # replacement vector, 0 stored in T), so every estimate restarts at EPS
            vec, nrm = self._finish(w, Q[:, :j])
            om = np.full(j, EPS)
            nxt = np.zeros(0, dtype=int)
        else:
            om = om * (nrm0 / nrm)
            om[sel] = EPS
            self.info.sigma_est = max(self.info.sigma_est, nrm)
            vec = w / nrm
        if side == "u":
            self.mu[:j] = om
            self.force_u = nxt
        else:
            self.nu[:j] = om
            self.force_v = nxt
        return vec, nrm

    def lanczos(self, i0):
        """Alg. 1 loop from 0-based column i0 (u_{i0}, v_{i0} already set)
        until v_p and beta_{p-1} (0-based) exist."""
        p = self.p
        for i in range(i0, p):
            self.v_step(i)
            if i == p - 1:
                break
            # Alg. 1 steps 7-8: u_{i+1} = A v_{i+1} - beta_i u_i, reorth, alpha.
            w = self.op.mv(self.V[:, i + 1]) - self.T[i, i + 1] * self.U[:, i]
            self.u_step(i + 1, w)


def validate(m, n, k, p):
    if k < 1 or p <= k or p > m or p + 1 > n:
        raise ValueError(f"need 1 <= k < p <= m and p + 1 <= n (m={m}, n={n}, k={k}, p={p})")


def small_svd(Tp: np.ndarray):
    """SVD of T(1:t,1:t) by LAPACK gesvd (as LAPACKE_dgesvd in Sec. 2.2.2)."""
    Uh, s, Vht = sla.svd(Tp, lapack_driver="gesvd")
    return Uh, s, Vht.T


def residual_estimates(beta, Uh_last_row, s, k, s_max=None):
    """eq. (4): |beta_t Uh(t, j)| / sigma_j, j < k, with the sigma floor
    (2^-52 times the largest singular value of T, ``s_max`` or s[0])."""
    s1 = s[0] if s_max is None else s_max
    floor = max(EPS * s1, TINY) if s.size else TINY
    return np.abs(beta * Uh_last_row[:k]) / np.maximum(s[:k], floor)


def sign_normalize(U, V):
    """Flip (u_j, v_j) so the largest-|.| entry of v_j is positive."""
    idx = np.argmax(np.abs(V), axis=0)          # first index on ties
    sgn = np.sign(V[idx, np.arange(V.shape[1])])
    sgn[sgn == 0] = 1.0
    return U * sgn, V * sgn


def harmonic_restart_basis(T: np.ndarray, p: int, k: int):
    """The harmonic-Ritz restart of the smallest triplets (see the module
    notes): from the (p+1) x (p+1) Lanczos T (leading p x p block, beta_p at
    T[p-1, p]) the coefficient matrices Q_C ((p+1) x (k+1), V_{p+1} Q_C is
    the new V_{k+1}), Q_M (p x k, U_p Q_M is the new U_k) and R_M (k x k, the
    new T(1:k, 1:k))."""
    B = T[:p, :p + 1]
    Ub, sb, Yt = sla.svd(B, full_matrices=True, lapack_driver="gesvd")
    Y = Yt.T                                   # (p+1) x (p+1); column p spans null(B)
    idx = np.argsort(sb, kind="stable")[:k]    # the k smallest harmonic values
    M = np.column_stack([Y[:, idx], Y[:, p]])
    r = M[p].copy()
    v = r.copy()
    v[k] += np.copysign(np.linalg.norm(r), r[k])
    H = np.eye(k + 1) - (2.0 / (v @ v)) * np.outer(v, v)
    QC = M @ H
    QC[p, :k] = 0.0
    if QC[p, k] < 0:
        QC[:, k] = -QC[:, k]
    QM = Ub[:, idx]
    RM = QM.T @ (B @ QC[:, :k])
    return QC, QM, RM


def svds(A, k: int, p: int = 0, tol: float = 0.0, maxit: int = 0,
         v0: np.ndarray | None = None, seed: int = 0, callback=None, which: str = "largest",
         selective: bool = False, partial: bool = False, harmonic: bool = False):
    """k largest (``which="largest"``, descending) or smallest
    (``which="smallest"``, ascending) singular triplets of A (scipy sparse
    matrix or dense array).

    Defaults follow Alg. 2 and Sec. 3: p = max(15, 3k), tol = 1e-10; the paper
    fixes no default for r, 10 (its experiments' value) is used.
    ``callback(stage, state, extra)`` sees the internal state after the first
    LBP ("lbp"), after every small SVD ("svd") and after every restart vector
    ("restart"), for invariant tests.

    Returns (U m x k, s (k,), V n x k, SvdsInfo).
    """
    m, n = A.shape
    p = p or max(15, 3 * k)
    tol = tol or 1e-10
    maxit = maxit or 10
    validate(m, n, k, p)
    if which not in ("largest", "smallest"):
        raise ValueError(which)
    info = SvdsInfo()
    op = _Op(A, info)
    if selective and partial:
        raise ValueError("selective and partial re-orthogonalisation exclude each other")
    if harmonic and (which != "smallest" or selective or partial):
        raise ValueError("harmonic augmentation is for the smallest triplets with full re-orthogonalisation")
    st = _State(op, p, seed, info, selective, partial)

    # Alg. 1 step 1: v_1 = randn / norm.
    v = np.asarray(v0, dtype=np.float64).copy() if v0 is not None else normal_vector(n, seed, 0)
    st.V[:, 0] = v / np.linalg.norm(v)
    # Alg. 1 steps 2-3: u_1 = A v_1, alpha_1 = norm.
    st.u_step(0, op.mv(st.V[:, 0]))
    # Alg. 2 step 2: LBP(A, t+1).
    st.lanczos(0)
    if callback:
        callback("lbp", st, None)

    while True:
        info.cycles += 1
        # Alg. 2 step 4: SVD of T(1:t, 1:t).
        Uh, s, Vh = small_svd(st.T[:p, :p])
        s_max = float(s[0])
        info.sigma_est = max(info.sigma_est, s_max)
        if which == "smallest":  # Ritz triplets in ascending order
            Uh, s, Vh = Uh[:, ::-1], s[::-1], Vh[:, ::-1]
        beta = st.T[p - 1, p]
        # Alg. 2 step 5 / eq. (4).
        res = residual_estimates(beta, Uh[p - 1], s, k, s_max)
        info.res_est = res
        info.nconv = int(np.argmin(np.append(res < tol, False)))
        if callback:
            callback("svd", st, dict(Uh=Uh, s=s, Vh=Vh, beta=beta, res=res))
        if np.all(res < tol):
            info.converged = True
            break
        if info.cycles >= maxit:
            break
        if harmonic:
            QC, QM, RM = harmonic_restart_basis(st.T, p, k)
            Un = st.U[:, :p] @ QM
            Vn = st.V[:, :p + 1] @ QC
            st.T[:] = 0.0
            st.T[:k, :k] = RM
            st.U[:, :k] = Un
            st.V[:, :k + 1] = Vn
            # u_{k+1}: A v_{k+1} against U_k, coefficients into T(1:k, k+1)
            w = op.mv(st.V[:, k])
            Uk = st.U[:, :k]
            h1 = Uk.T @ w
            w = w - Uk @ h1
            h2 = Uk.T @ w
            w = w - Uk @ h2
            st.T[:k, k] = h1 + h2
            nrm = float(np.linalg.norm(w))
            if nrm <= BREAKDOWN_REL * info.sigma_est:
                st.U[:, k], st.T[k, k] = st._finish(w, Uk)  # replacement vector, 0 in T
            else:
                info.sigma_est = max(info.sigma_est, nrm)
                st.U[:, k], st.T[k, k] = w / nrm, nrm
            info.restarts += 1
            info.harmonic_restarts += 1
            if callback:
                callback("restart", st, dict(Uk=Un, rho=None))
            st.lanczos(k)
            continue
        # Alg. 2 step 8: Ritz vectors (Proposition 1, eq. (2)).
        Uk = st.U[:, :p] @ Uh[:, :k]
        Vk = st.V[:, :p] @ Vh[:, :k]
        # Alg. 2 step 9: new T = [Sigma_k, rho] with rho = beta_t Uh(t, 1:k)^T (eq. (6)).
        rho = beta * Uh[p - 1, :k]
        vnext = st.V[:, p].copy()
        st.T[:] = 0.0
        st.T[np.arange(k), np.arange(k)] = s[:k]
        st.T[:k, k] = rho
        st.U[:, :k] = Uk
        st.V[:, :k] = Vk
        # Alg. 2 step 10: v_{k+1} = v_{t+1}; u_{k+1} = A v_{k+1} - Uk rho (eq. (7)).
        st.V[:, k] = vnext
        if partial:
            # estimates of v_{t+1} against the kept Ritz vectors V Vh_k
            nu_old = st.nu[:p].copy()
            st.nu[:] = 0.0
            st.nu[:k] = Vh[:, :k].T @ nu_old
            st.nu[k] = 1.0
            st.force_u = st.force_v = np.zeros(0, dtype=int)
        w = op.mv(st.V[:, k]) - Uk @ rho
        # Alg. 2 step 11 (with re-orthogonalisation, as the text after Alg. 2 asks).
        st.u_step(k, w, full=True)
        info.restarts += 1
        if callback:
            callback("restart", st, dict(Uk=Uk, rho=rho))
        # Alg. 2 step 12: continue the Lanczos loop from column k+1.
        st.lanczos(k)

    # Alg. 2 steps 15-16.
    S = s[:k].copy()
    U = st.U[:, :p] @ Uh[:, :k]
    V = st.V[:, :p] @ Vh[:, :k]
    U, V = sign_normalize(U, V)
    return U, S, V, info


def lbp(A, p: int, v0: np.ndarray, seed: int = 0):
    """Alg. 1 alone (with CGS2) for p steps: returns (U m x p, T p x p, V n x p,
    beta_p, info).  Allows p = min(m, n) (complete bidiagonalisation, where
    the last beta is a breakdown)."""
    m, n = A.shape
    info = SvdsInfo()
    op = _Op(A, info)
    st = _State(op, p, seed, info)
    st.V[:, 0] = v0 / np.linalg.norm(v0)
    st.u_step(0, op.mv(st.V[:, 0]))
    st.lanczos(0)
    return st.U, st.T[:p, :p].copy(), st.V[:, :p], st.T[p - 1, p], info


def explicit_residuals(A, U, S, V):
    """FP64 |A v_j - s_j u_j| and |A^T u_j - s_j v_j| for each output triplet."""
    AV = np.asarray(A @ V)
    ATU = np.asarray(A.T @ U)
    r1 = np.linalg.norm(AV - U * S, axis=0)
    r2 = np.linalg.norm(ATU - V * S, axis=0)
    return r1, r2


def as_operator(csr_or_dense):
    """scipy CSR from an ``inputs.CSR``-like object, or a dense ndarray."""
    if isinstance(csr_or_dense, np.ndarray):
        return csr_or_dense
    c = csr_or_dense
    return sp.csr_matrix((np.asarray(c.val, dtype=np.float64), c.col_idx, c.row_ptr),
                         shape=(c.m, c.n))
