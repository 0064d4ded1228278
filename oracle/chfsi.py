"""FP64 oracle: Chebyshev filter, its adjoint, orthonormalisation and
Rayleigh-Ritz, following Algorithm 1 (ChFSI) of Sec. 3.4.

Test infrastructure only: imported by tests, the smoke check and the benchmark's
CPU-baseline leg, never by the GPU library.

Notation (Algorithm 1, Sec. 3.4): the unwanted spectrum [a, b] with
a = eps_ub^w (upper bound of the wanted spectrum) and b = eps_ub^uw (upper
bound of the unwanted spectrum); a0 = eps_0 is the scaling point below the
wanted spectrum.  e = (b - a)/2 and c = (b + a)/2 map [a, b] onto [-1, 1].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def csr_from_arrays(indptr, indices, data, N):
    """SciPy CSR view of the generator's natural-order matrix."""
    return sp.csr_matrix((data, indices, indptr), shape=(N, N))


def filter_parameters(a: float, b: float, a0: float):
    """Half-width e, centre c and the image tau of the scaling point
    (initialisation of Algorithm 1, Sec. 3.4).  Requires a0 < a < b."""
    if not (np.isfinite(a) and np.isfinite(b) and np.isfinite(a0) and a0 < a < b):
        raise ValueError("filter bounds must satisfy a0 < a < b")
    e = 0.5 * (b - a)
    c = 0.5 * (b + a)
    tau = (a0 - c) / e
    return e, c, tau


def chebyshev_T(m: int, x):
    """T_m(x) from the defining recurrence T_0 = 1, T_1 = x,
    T_{k+1} = 2 x T_k - T_{k-1} (elementwise on arrays)."""
    x = np.asarray(x, dtype=np.float64)
    t_prev, t = np.ones_like(x), x.copy()
    if m == 0:
        return t_prev
    for _ in range(1, m):
        t_prev, t = t, 2.0 * x * t - t_prev
    return t


def sigma_sequence(m: int, a: float, b: float, a0: float):
    """sigma_1 .. sigma_m of Algorithm 1: sigma_1 = e/(a0 - c),
    gamma = 2/sigma_1, sigma_{i} = 1/(gamma - sigma_{i-1})."""
    e, c, _ = filter_parameters(a, b, a0)
    s = [e / (a0 - c)]
    gamma = 2.0 / s[0]
    for _ in range(2, m + 1):
        s.append(1.0 / (gamma - s[-1]))
    return np.array(s)


def cheb_filter(H, X, m: int, a: float, b: float, a0: float):
    """The filtered block Y = T_m((H - cI)/e) X / T_m(tau) (Sec. 3.4).

    Plain definition: the matrix Chebyshev polynomial is built with the
    defining three-term recurrence on Hs = (H - cI)/e, then divided by the
    scalar T_m(tau).  No sigma scaling is used here; the scaled recurrence of
    Algorithm 1 reaches the same block up to rounding.
    """
    if m < 1:
        raise ValueError("degree m must be >= 1")
    e, c, tau = filter_parameters(a, b, a0)
    X = np.asarray(X, dtype=np.float64)

    def hs(V):
        return (H @ V - c * V) / e

    z_prev, z = X, hs(X)
    for _ in range(1, m):
        z_prev, z = z, 2.0 * hs(z) - z_prev
    return z / chebyshev_T(m, tau)


def cheb_filter_scaled(H, X, m: int, a: float, b: float, a0: float):
    """The filtered block formed through scaled iterates, the way the filter of
    Sec. 3.4 keeps its intermediate blocks of moderate size.

    The scaled iterate is Y_k = T_k(Hs) X / t_k with Hs = (H - cI)/e and
    t_j = T_j(tau), so Y_0 = X and Y_1 = Hs X / tau.  Dividing the defining
    relation T_{k+1}(Hs) = 2 Hs T_k(Hs) - T_{k-1}(Hs) by t_{k+1} gives

        Y_{k+1} = 2 (t_k / t_{k+1}) Hs Y_k - (t_{k-1} / t_{k+1}) Y_{k-1}.

    The coefficients here are ratios of Chebyshev values taken from
    chebyshev_T; Algorithm 1 obtains the same ratios by its sigma recursion
    (sigma_k = t_{k-1} / t_k).  The last iterate Y_m equals cheb_filter's
    result up to rounding.
    """
    if m < 1:
        raise ValueError("degree m must be >= 1")
    e, c, tau = filter_parameters(a, b, a0)
    X = np.asarray(X, dtype=np.float64)
    t = [float(chebyshev_T(j, tau)) for j in range(m + 1)]

    def hs(V):
        return (H @ V - c * V) / e

    y_prev, y = X, hs(X) / t[1]
    for k in range(1, m):
        y_prev, y = y, (2.0 * t[k] / t[k + 1]) * hs(y) - (t[k - 1] / t[k + 1]) * y_prev
    return y


def cheb_filter_schedule(H_early, H_late, m_late: int, X, m: int, a: float, b: float,
                         a0: float):
    """The filter with a precision schedule: the scaled iterates of
    cheb_filter_scaled, where the degree steps k = 0 .. m - m_late - 1 (the step
    forming Y_{k+1} from Y_k) take their product with H_early and the last
    m_late steps with H_late.  With H_early = H_late it is the filter of Sec. 3.4;
    here the two are the same Hamiltonian rounded to two precisions, so every
    step uses the same coefficients (ratios of T_j(tau)) and only the matrix
    changes with the step."""
    if m < 1:
        raise ValueError("degree m must be >= 1")
    if not 0 <= m_late <= m:
        raise ValueError("m_late must lie in 0 .. m")
    e, c, tau = filter_parameters(a, b, a0)
    X = np.asarray(X, dtype=np.float64)
    t = [float(chebyshev_T(j, tau)) for j in range(m + 1)]

    def hs(k, V):
        H = H_early if k < m - m_late else H_late
        return (H @ V - c * V) / e

    y_prev, y = X, hs(0, X) / t[1]
    for k in range(1, m):
        y_prev, y = y, (2.0 * t[k] / t[k + 1]) * hs(k, y) - (t[k - 1] / t[k + 1]) * y_prev
    return y


def cheb_filter_adjoint(H, X, dY, m: int, a: float, b: float, a0: float,
                        chunk: int = 1 << 16):
    """Gradients of L = <dY, Y> for Y = cheb_filter(H, X, ...).

    Reverse mode of the defining recurrence Z_0 = X, Z_1 = Hs Z_0,
    Z_{k+1} = 2 Hs Z_k - Z_{k-1}, Y = Z_m / T_m(tau), with Hs = (H - cI)/e:
      Zbar_m = dY / T_m(tau);  Zbar_k += 2 Hs Zbar_{k+1},  Zbar_{k-1} -= Zbar_{k+1};
      dL/dHs = sum_{k>=1} 2 Zbar_{k+1} Z_k^T + Zbar_1 Z_0^T;  dL/dH = dL/dHs / e.
    Returns dX (N x n) and dH restricted to H's stored pattern, as an array
    aligned with H.data (entry (i, j) is dL/dH_ij with H_ij and H_ji treated as
    independent entries).
    """
    if m < 1:
        raise ValueError("degree m must be >= 1")
    e, c, tau = filter_parameters(a, b, a0)
    H = sp.csr_matrix(H)
    X = np.asarray(X, dtype=np.float64)

    def hs(V):
        return (H @ V - c * V) / e

    Z = [X, hs(X)]
    for _ in range(1, m):
        Z.append(2.0 * hs(Z[-1]) - Z[-2])
    zbar = [np.zeros_like(X) for _ in range(m + 1)]
    zbar[m] = np.asarray(dY, dtype=np.float64) / chebyshev_T(m, tau)
    rows = np.repeat(np.arange(H.shape[0]), np.diff(H.indptr))
    cols = H.indices
    g = np.zeros(H.nnz)

    def sddmm(coef, A, B):
        for s in range(0, H.nnz, chunk):
            t = min(H.nnz, s + chunk)
            g[s:t] += coef * np.einsum("ij,ij->i", A[rows[s:t]], B[cols[s:t]])

    for k in range(m - 1, 0, -1):
        zbar[k] += 2.0 * hs(zbar[k + 1])
        zbar[k - 1] -= zbar[k + 1]
        sddmm(2.0, zbar[k + 1], Z[k])
    zbar[0] += hs(zbar[1])
    sddmm(1.0, zbar[1], Z[0])
    return zbar[0], g / e


def orth(Y):
    """Orthonormal basis of span(Y): the thin QR factor Q with positive
    diagonal R (unique for full-rank Y), from Householder QR."""
    import scipy.linalg as sla

    Q, R = sla.qr(np.asarray(Y, dtype=np.float64), mode="economic", check_finite=False)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def cholqr2(Y):
    """Cholesky-QR applied twice, with column scaling (step 2 of Algorithm 1
    carried out as Cholesky-QR).  Returns (Q, R) with Y = Q R."""
    Y = np.asarray(Y, dtype=np.float64)
    R_total = np.eye(Y.shape[1])
    Q = Y
    for _ in range(2):
        d = np.linalg.norm(Q, axis=0)
        Qs = Q / d
        G = Qs.T @ Qs
        L = np.linalg.cholesky(G)            # G = L L^T, R = L^T
        R = L.T
        Q = np.linalg.solve(R.T, Qs.T).T     # Qs R^{-1}
        R_total = (R * d[None, :]) @ R_total  # Q_old = Qs D = Q R D
    return Q, R_total


def dense_eigh(A):
    """Eigen-decomposition A Q = Q Lambda of a symmetric matrix, ascending
    (step 4 of Algorithm 1), by LAPACK."""
    A = np.asarray(A, dtype=np.float64)
    return np.linalg.eigh(0.5 * (A + A.T))


def rayleigh_ritz(H, Y):
    """Steps 2-5 of Algorithm 1 on the filtered block Y: X_F = Orth(Y),
    H_F = X_F^T H X_F, H_F Q = Q Lambda, Psi = X_F Q.  Returns (Lambda, Psi)."""
    XF = orth(Y)
    HF = XF.T @ (H @ XF)
    lam, Q = dense_eigh(HF)
    return lam, XF @ Q


def ritz_residuals(H, Psi, lam):
    """Residual norms || H psi_j - lambda_j psi_j ||_2 of Ritz pairs, the
    convergence test of the subspace iteration (Sec. 3.4): the definition,
    column by column."""
    R = H @ Psi - Psi * np.asarray(lam)[None, :]
    return np.sqrt(np.sum(R * R, axis=0))


def chfsi(H, X, m: int, a: float, b: float, a0: float, passes: int):
    """Algorithm 1 applied `passes` times (Sec. 3.4): each pass filters the
    previous Ritz vectors; after a pass the scaling point a0 and the cut a move
    to the smallest and largest Ritz values (b is kept).  Returns (Lambda, Psi,
    residual norms of the last pass)."""
    lam = Psi = None
    for _ in range(passes):
        lam, Psi = rayleigh_ritz(H, cheb_filter(H, X, m, a, b, a0))
        a0, a = float(lam.min()), float(lam.max())
        X = Psi
    return lam, Psi, ritz_residuals(H, Psi, lam)


def fermi_occupancies(eps, n_electrons: float, kT: float):
    """Fermi-Dirac occupancies f_i = 1 / (1 + exp((eps_i - mu) / kT)) with the
    Fermi energy mu fixed by the electron count 2 sum_i f_i = N_e (Sec. 2,
    occupancy and electron-count equations).  mu by SciPy's bracketing root
    finder on the increasing count, to full FP64 precision.  Returns (f, mu)."""
    from scipy.optimize import brentq

    eps = np.asarray(eps, dtype=np.float64)
    if not 0.0 < n_electrons < 2.0 * eps.size:
        raise ValueError("need 0 < N_e < 2n")

    def occ(mu):
        with np.errstate(over="ignore"):
            return 1.0 / (1.0 + np.exp((eps - mu) / kT))

    count = lambda mu: 2.0 * occ(mu).sum() - n_electrons
    lo, hi = eps.min() - kT, eps.max() + kT
    while count(lo) >= 0.0:
        lo -= hi - lo
    while count(hi) <= 0.0:
        hi += hi - lo
    mu = brentq(count, lo, hi, xtol=1e-16, rtol=8.9e-16, maxiter=500)
    return occ(mu), mu


def density_matrix_on_pattern(H, Psi, f):
    """Density matrix P = Psi diag(2 f) Psi^T of the occupied Ritz vectors at the
    stored entries of H (in H's CSR order): the electron density of Sec. 2 in a
    localized basis needs it where basis functions overlap."""
    H = sp.csr_matrix(H)
    rows = np.repeat(np.arange(H.shape[0]), np.diff(H.indptr))
    W = Psi * (2.0 * np.asarray(f))[None, :]
    return np.einsum("ij,ij->i", W[rows], Psi[H.indices])


def electron_density(Psi, f):
    """rho_r = 2 sum_i f_i psi_ri^2 (Sec. 2, density equation, at the lattice
    sites)."""
    return 2.0 * (Psi * Psi) @ np.asarray(f)
