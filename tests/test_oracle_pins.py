"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics:
closed forms, special cases, invariants, finite differences and the
Daleckii-Krein gradient.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workload

A, B, A0 = 2.0, 12.5, -3.0


def t_closed(m, x):
    """Chebyshev T_m from its trigonometric / hyperbolic closed form."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** m * np.cosh(m * np.arccosh(np.abs(xo)))
    return out


def small_h(r=5, h=2, seed=0):
    ip, ix, d, N = workload.lattice_hamiltonian(r, h, seed)
    return oracle.csr_from_arrays(ip, ix, d, N), N


def p_of(lam, m, a=A, b=B, a0=A0):
    e, c = (b - a) / 2, (b + a) / 2
    return t_closed(m, (lam - c) / e) / t_closed(m, np.array([(a0 - c) / e]))[0]


# ---------------------------------------------------------------- coefficients
def test_filter_parameters_config1():
    e, c, tau = oracle.filter_parameters(A, B, A0)
    assert e == 5.25 and c == 7.25
    assert tau == pytest.approx(-41.0 / 21.0, rel=0, abs=1e-15)


@pytest.mark.parametrize("bad", [(2.0, 12.5, 2.0), (2.0, 2.0, -3.0), (3.0, 2.0, -3.0),
                                 (np.nan, 12.5, -3.0), (2.0, np.inf, -3.0)])
def test_filter_parameters_reject(bad):
    with pytest.raises(ValueError):
        oracle.filter_parameters(*bad)


def test_sigma_is_ratio_of_chebyshev_values():
    # sigma_k = T_{k-1}(tau) / T_k(tau), closed-form T
    m = 24
    _, _, tau = oracle.filter_parameters(A, B, A0)
    s = oracle.sigma_sequence(m, A, B, A0)
    for k in range(1, m + 1):
        ratio = t_closed(k - 1, np.array([tau]))[0] / t_closed(k, np.array([tau]))[0]
        assert s[k - 1] == pytest.approx(ratio, rel=1e-14)


def test_chebyshev_T_matches_closed_form():
    x = np.linspace(-4.3, 4.3, 201)
    for m in (0, 1, 2, 7, 10, 20):
        np.testing.assert_allclose(oracle.chebyshev_T(m, x), t_closed(m, x),
                                   rtol=1e-12, atol=1e-12)


def test_T_m_tau_golden():
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "chebyshev_scaling.json")))
    _, _, tau = oracle.filter_parameters(g["a"], g["b"], g["a0"])
    for m, val in g["T_m_tau"].items():
        assert oracle.chebyshev_T(int(m), tau) == pytest.approx(val, rel=1e-12)
    np.testing.assert_allclose(oracle.sigma_sequence(10, g["a"], g["b"], g["a0"]),
                               g["sigma_1_to_10"], rtol=1e-13)


# ---------------------------------------------------------------- filter
@pytest.mark.parametrize("r,h,m", [(4, 1, 1), (4, 3, 10), (5, 2, 7), (6, 2, 16), (6, 3, 20)])
def test_filter_matches_spectral_closed_form(r, h, m):
    H, N = small_h(r, h)
    X = workload.gaussian_block(N, 6, 1)
    lam, V = np.linalg.eigh(H.toarray())
    ref = V @ (p_of(lam, m)[:, None] * (V.T @ X))
    for fn in (oracle.cheb_filter, oracle.cheb_filter_scaled):
        Y = fn(H, X, m, A, B, A0)
        assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) < 1e-13


# The C/OpenMP oracle (oracle/cheb_filter.c) computes the same definition; it is
# pinned on its own to the spectral closed form, and checked on the special cases
# that exercise its column blocks (a ragged last block, one column, blocks wider
# than the matrix) and its thread split.
@pytest.mark.parametrize("r,h,m,n,blk,threads", [(4, 1, 1, 3, 8, 1), (4, 3, 10, 7, 3, 2),
                                                 (5, 2, 7, 9, 4, 3), (6, 2, 16, 1, 8, 4),
                                                 (6, 3, 20, 17, 64, 2)])
def test_c_oracle_filter_matches_spectral_closed_form(r, h, m, n, blk, threads):
    H, N = small_h(r, h)
    lam, V = np.linalg.eigh(H.toarray())
    X = workload.gaussian_block(N, n, 7)
    Y = oracle.cheb_filter_c(H, X, m, A, B, A0, threads=threads, blk=blk)
    ref = V @ (p_of(lam, m)[:, None] * (V.T @ X))
    assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) <= 1e-12


def test_c_oracle_filter_special_cases():
    # m = 1: (H - cI) X / (a0 - c); H = c I: cos(m pi / 2) / T_m(tau) X
    H, N = small_h(4, 2)
    X = workload.gaussian_block(N, 5, 3)
    e, c, tau = oracle.filter_parameters(A, B, A0)
    Y1 = oracle.cheb_filter_c(H, X, 1, A, B, A0)
    assert np.allclose(Y1, (H @ X - c * X) / (A0 - c), rtol=0, atol=1e-13 * np.abs(X).max())
    Hc = sp.identity(N, format="csr") * c
    for m in (3, 4, 10):
        Y = oracle.cheb_filter_c(Hc, X, m, A, B, A0)
        assert np.allclose(Y, np.cos(m * np.pi / 2) / t_closed(m, np.array([tau]))[0] * X,
                           rtol=0, atol=1e-15)
    with pytest.raises(ValueError):
        oracle.cheb_filter_c(H, X, 0, A, B, A0)
    with pytest.raises(ValueError):
        oracle.cheb_filter_c(H, X, 5, A, A, A0)


def test_filter_config1_scaled_vs_definition():
    ip, ix, d, N = workload.lattice_hamiltonian(20, 3, 0)
    H = oracle.csr_from_arrays(ip, ix, d, N)
    X = workload.gaussian_block(N, 8, 0)
    Y1 = oracle.cheb_filter(H, X, 10, A, B, A0)
    Y2 = oracle.cheb_filter_scaled(H, X, 10, A, B, A0)
    assert np.linalg.norm(Y1 - Y2) / np.linalg.norm(Y1) < 1e-14


def u_closed(n, y):
    """Chebyshev U_n from its trigonometric / hyperbolic closed form (U_-1 = 0)."""
    y = np.asarray(y, dtype=np.float64)
    if n < 0:
        return np.zeros_like(y)
    out = np.empty_like(y)
    inside = np.abs(y) < 1
    th = np.arccos(y[inside])
    out[inside] = np.sin((n + 1) * th) / np.sin(th)
    yo = y[~inside]
    ph = np.arccosh(np.abs(yo))
    out[~inside] = np.sign(yo) ** n * np.sinh((n + 1) * ph) / np.sinh(ph)
    return out


def schedule_closed_form(lam, mu, m, m_late, a=A, b=B, a0=A0):
    """Scalar filter value when the first s = m - m_late degree steps use the
    eigenvalue lam and the rest mu (commuting matrices): the unscaled iterate
    is T_k(x) up to k = s, x = (lam - c)/e; after that the recurrence with
    y = (mu - c)/e continues from (T_{s-1}(x), T_s(x)), and any solution of
    f_{j+1} = 2 y f_j - f_{j-1} is f_0 T_j(y) + (f_1 - y f_0) U_{j-1}(y)."""
    e, c = (b - a) / 2, (b + a) / 2
    x, y = (lam - c) / e, (mu - c) / e
    tm = t_closed(m, np.array([(a0 - c) / e]))[0]
    s = m - m_late
    if s == 0:
        return t_closed(m, y) / tm
    f0, f1 = t_closed(s - 1, x), t_closed(s, x)
    j = m - s + 1
    return (f0 * t_closed(j, y) + (f1 - y * f0) * u_closed(j - 1, y)) / tm


@pytest.mark.parametrize("m,m_late", [(1, 0), (1, 1), (2, 1), (10, 0), (10, 3), (10, 10), (20, 4),
                                      (20, 19), (7, 1)])
def test_schedule_commuting_matrices_closed_form(m, m_late):
    # two symmetric matrices with the same eigenvectors: the scheduled filter
    # acts on each eigenvector by the scalar closed form above
    rng = np.random.default_rng(m * 100 + m_late)
    n = 40
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.sort(rng.uniform(-12.0, 11.0, n))
    mu = lam + rng.uniform(-0.3, 0.3, n)
    He, Hl = (V * lam) @ V.T, (V * mu) @ V.T
    X = rng.standard_normal((n, 5))
    Y = oracle.cheb_filter_schedule(He, Hl, m_late, X, m, A, B, A0)
    ref = V @ (schedule_closed_form(lam, mu, m, m_late)[:, None] * (V.T @ X))
    assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) < 1e-12


def test_schedule_reduces_to_the_filter():
    # no switch, or the same matrix on both sides: the plain filter (closed form)
    H, N = small_h(5, 2)
    X = workload.gaussian_block(N, 4, 5)
    lam, V = np.linalg.eigh(H.toarray())
    Hd = sp.diags(np.linspace(-3.0, 9.0, N)).tocsr()
    for m, m_late, He, Hl in ((10, 0, H, Hd), (10, 10, Hd, H), (12, 5, H, H), (1, 1, Hd, H)):
        Y = oracle.cheb_filter_schedule(He, Hl, m_late, X, m, A, B, A0)
        ref = V @ (p_of(lam, m)[:, None] * (V.T @ X))
        assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) < 1e-13
    with pytest.raises(ValueError):
        oracle.cheb_filter_schedule(H, H, 11, X, 10, A, B, A0)


def test_filter_degree_one():
    H, N = small_h()
    X = workload.gaussian_block(N, 3, 2)
    c = (A + B) / 2
    ref = (H @ X - c * X) / (A0 - c)
    np.testing.assert_allclose(oracle.cheb_filter(H, X, 1, A, B, A0), ref, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 9, 10])
def test_filter_of_shift_identity(m):
    # H = cI  =>  Y = T_m(0)/T_m(tau) X = cos(m pi/2)/T_m(tau) X
    N = 30
    c = (A + B) / 2
    H = sp.identity(N, format="csr") * c
    X = workload.gaussian_block(N, 4, 3)
    _, _, tau = oracle.filter_parameters(A, B, A0)
    scale = np.cos(m * np.pi / 2) / t_closed(m, np.array([tau]))[0]
    Y = oracle.cheb_filter(H, X, m, A, B, A0)
    np.testing.assert_allclose(Y, scale * X, atol=1e-15 * np.abs(X).max() + 1e-300)


def test_filter_diagonal_matrix_is_row_scaling():
    rng = np.random.default_rng(5)
    dvals = rng.uniform(-15, 12, 50)
    H = sp.diags(dvals, format="csr")
    X = rng.standard_normal((50, 3))
    Y = oracle.cheb_filter(H, X, 12, A, B, A0)
    np.testing.assert_allclose(Y, p_of(dvals, 12)[:, None] * X, rtol=1e-12)


def test_filter_scalar_case():
    H = sp.csr_matrix(np.array([[4.2]]))
    y = oracle.cheb_filter(H, np.array([[1.5]]), 9, A, B, A0)
    assert y[0, 0] == pytest.approx(1.5 * p_of(np.array([4.2]), 9)[0], rel=1e-14)


def test_filter_eigenvector_input():
    H, N = small_h(5, 2)
    lam, V = np.linalg.eigh(H.toarray())
    for i in (0, N // 2, N - 1):
        y = oracle.cheb_filter(H, V[:, i:i + 1], 10, A, B, A0)
        np.testing.assert_allclose(y[:, 0], p_of(lam[i:i + 1], 10)[0] * V[:, i],
                                   atol=1e-12 * max(1.0, abs(p_of(lam[i:i + 1], 10)[0])))


def test_filter_linearity_and_column_independence():
    H, N = small_h(5, 2)
    X = workload.gaussian_block(N, 5, 4)
    Z = workload.gaussian_block(N, 5, 5)
    f = lambda V: oracle.cheb_filter(H, V, 8, A, B, A0)
    YX, YZ = f(X), f(Z)
    np.testing.assert_allclose(f(2.5 * X - 0.5 * Z), 2.5 * YX - 0.5 * YZ,
                               rtol=1e-12, atol=1e-12 * np.abs(YX).max())
    perm = np.array([3, 0, 4, 1, 2])
    np.testing.assert_array_equal(f(X[:, perm]), YX[:, perm])
    np.testing.assert_array_equal(f(X[:, 2:3])[:, 0], YX[:, 2])


def test_filter_self_adjoint():
    H, N = small_h(5, 2)
    U = workload.gaussian_block(N, 1, 6)
    V = workload.gaussian_block(N, 1, 7)
    f = lambda Q: oracle.cheb_filter(H, Q, 11, A, B, A0)
    lhs, rhs = float(U[:, 0] @ f(V)[:, 0]), float(f(U)[:, 0] @ V[:, 0])
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_scaling_point_only_rescales():
    H, N = small_h(5, 2)
    X = workload.gaussian_block(N, 3, 8)
    m = 10
    Y1 = oracle.cheb_filter(H, X, m, A, B, -3.0)
    Y2 = oracle.cheb_filter(H, X, m, A, B, -7.0)
    e, c = (B - A) / 2, (B + A) / 2
    ratio = t_closed(m, np.array([(-7.0 - c) / e]))[0] / t_closed(m, np.array([(-3.0 - c) / e]))[0]
    np.testing.assert_allclose(Y1, ratio * Y2, rtol=1e-12, atol=1e-14 * np.abs(Y1).max())


def test_reject_degree_zero():
    H, N = small_h(4, 1)
    with pytest.raises(ValueError):
        oracle.cheb_filter(H, np.ones((N, 1)), 0, A, B, A0)


# ---------------------------------------------------------------- H X by row slabs
@pytest.mark.parametrize("nslabs", [1, 2, 3, 7])
def test_hx_as_sum_over_row_slabs(nslabs):
    # Eq. (reformat HX), Sec. 4.2: H X = sum_k (H_k)^T X_k over row slabs k,
    # checked with virtual ranks on the CPU.
    H, N = small_h(6, 2)
    X = workload.gaussian_block(N, 4, 9)
    tau, nu = divmod(N, nslabs)
    bounds, start = [], 0
    for k in range(nslabs):
        size = tau + (1 if k < nu else 0)
        bounds.append((start, start + size))
        start += size
    acc = np.zeros_like(X)
    for lo, hi in bounds:
        acc += H[lo:hi, :].T @ X[lo:hi, :]
    np.testing.assert_allclose(acc, H @ X, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- adjoint
def _loss(H, X, W, m):
    return float(np.sum(W * oracle.cheb_filter(H, X, m, A, B, A0)))


@pytest.mark.parametrize("m", [1, 2, 6])
def test_adjoint_dx_is_filter_of_weights(m):
    H, N = small_h(4, 2)
    X = workload.gaussian_block(N, 3, 10)
    W = workload.gaussian_block(N, 3, 10, stream="W")
    dX, _ = oracle.cheb_filter_adjoint(H, X, W, m, A, B, A0)
    # p(H) is symmetric for symmetric H, so dX = p(H) W
    ref = oracle.cheb_filter_scaled(H, W, m, A, B, A0)
    np.testing.assert_allclose(dX, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("m", [1, 3, 8])
def test_adjoint_finite_differences(m):
    H, N = small_h(4, 2)
    X = workload.gaussian_block(N, 3, 11)
    W = workload.gaussian_block(N, 3, 11, stream="W")
    dX, g = oracle.cheb_filter_adjoint(H, X, W, m, A, B, A0)
    hstep = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(6):                       # entries of X: only column j changes
        i, j = rng.integers(N), rng.integers(3)
        Xp, Xm = X.copy(), X.copy()
        Xp[i, j] += hstep
        Xm[i, j] -= hstep
        fd = np.sum(W[:, j] * (oracle.cheb_filter(H, Xp[:, j:j + 1], m, A, B, A0)[:, 0]
                               - oracle.cheb_filter(H, Xm[:, j:j + 1], m, A, B, A0)[:, 0])) / (2 * hstep)
        assert fd == pytest.approx(dX[i, j], rel=1e-6, abs=1e-7)
    rows = np.repeat(np.arange(N), np.diff(H.indptr))
    cols = H.indices
    for t in rng.choice(H.nnz, 8, replace=False):   # single entries (H as a general matrix)
        Hp, Hm = H.copy(), H.copy()
        Hp.data[t] += hstep
        Hm.data[t] -= hstep
        fd = (_loss(Hp, X, W, m) - _loss(Hm, X, W, m)) / (2 * hstep)
        assert fd == pytest.approx(g[t], rel=1e-6, abs=1e-7)
    # symmetric pair perturbation: dL = G_ij + G_ji
    pos = {(int(rows[t]), int(cols[t])): t for t in range(H.nnz)}
    for t in rng.choice(H.nnz, 8, replace=False):
        i, j = int(rows[t]), int(cols[t])
        tt = pos[(j, i)]
        Hp, Hm = H.copy(), H.copy()
        for s in {t, tt}:
            Hp.data[s] += hstep
            Hm.data[s] -= hstep
        fd = (_loss(Hp, X, W, m) - _loss(Hm, X, W, m)) / (2 * hstep)
        expect = g[t] + (g[tt] if tt != t else 0.0)
        assert fd == pytest.approx(expect, rel=1e-6, abs=1e-7)


def _cheb_divided_difference(m, x, y):
    """(T_m(x) - T_m(y)) / (x - y) by D_0 = 0, D_1 = 1,
    D_{k+1} = 2 x D_k + 2 T_k(y) - D_{k-1}; T_k(y) in closed form."""
    d_prev, d = np.zeros_like(x * y), np.ones_like(x * y)
    if m == 0:
        return d_prev
    for k in range(1, m):
        d_prev, d = d, 2 * x * d + 2 * t_closed(k, y) - d_prev
    return d


@pytest.mark.parametrize("r,h,m", [(4, 2, 5), (5, 2, 12)])
def test_adjoint_dense_daleckii_krein(r, h, m):
    H, N = small_h(r, h)
    X = workload.gaussian_block(N, 4, 12)
    W = workload.gaussian_block(N, 4, 12, stream="W")
    _, g = oracle.cheb_filter_adjoint(H, X, W, m, A, B, A0)
    lam, V = np.linalg.eigh(H.toarray())
    e, c = (B - A) / 2, (B + A) / 2
    tau = (A0 - c) / e
    x = (lam - c) / e
    F = _cheb_divided_difference(m, x[:, None], x[None, :]) / (e * t_closed(m, np.array([tau]))[0])
    G = V @ ((V.T @ W @ X.T @ V) * F) @ V.T
    rows = np.repeat(np.arange(N), np.diff(H.indptr))
    ref = G[rows, H.indices]
    assert np.max(np.abs(g - ref)) <= 1e-11 * np.max(np.abs(ref))


# ---------------------------------------------------------------- orthonormalisation
def test_orth_properties():
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((300, 40)) @ np.diag(np.logspace(0, 4, 40))
    Q = oracle.orth(Y)
    assert np.max(np.abs(Q.T @ Q - np.eye(40))) < 1e-14
    R = Q.T @ Y
    assert np.max(np.abs(np.tril(R, -1))) < 1e-10 * np.abs(R).max()
    assert np.all(np.diag(R) > 0)
    np.testing.assert_allclose(Q @ np.triu(R), Y, atol=1e-11 * np.abs(Y).max())


def test_cholqr2_properties_and_agreement():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((500, 30)) @ np.diag(np.logspace(0, 6, 30))
    Q, R = oracle.cholqr2(Y)
    assert np.max(np.abs(Q.T @ Q - np.eye(30))) < 1e-14
    assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R) > 0)
    np.testing.assert_allclose(Q @ R, Y, atol=1e-12 * np.abs(Y).max())
    # thin QR with positive diagonal R is unique: equals Householder's
    np.testing.assert_allclose(Q, oracle.orth(Y), atol=1e-11)


# ---------------------------------------------------------------- eigensolve and Rayleigh-Ritz
def test_dense_eigh_toeplitz_closed_form():
    n = 40
    T = np.diag(2.0 * np.ones(n)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    lam, Q = oracle.dense_eigh(T)
    k = np.arange(1, n + 1)
    np.testing.assert_allclose(lam, np.sort(2 - 2 * np.cos(k * np.pi / (n + 1))), atol=1e-13)
    np.testing.assert_allclose(T @ Q, Q * lam, atol=1e-13)


def test_rayleigh_ritz_full_space_gives_spectrum():
    H, N = small_h(4, 2)
    Y = workload.gaussian_block(N, N, 13)
    lam, Psi = oracle.rayleigh_ritz(H, Y)
    np.testing.assert_allclose(lam, np.linalg.eigvalsh(H.toarray()), atol=1e-12)
    np.testing.assert_allclose(H @ Psi, Psi * lam, atol=1e-11)


def test_rayleigh_ritz_invariant_subspace():
    H, N = small_h(5, 2)
    lam_all, V = np.linalg.eigh(H.toarray())
    idx = np.array([0, 3, 7, 20, 50])
    rng = np.random.default_rng(3)
    Y = V[:, idx] @ rng.standard_normal((5, 5))     # a basis of an invariant subspace
    lam, Psi = oracle.rayleigh_ritz(H, Y)
    np.testing.assert_allclose(lam, lam_all[idx], atol=1e-12)
    np.testing.assert_allclose(Psi.T @ Psi, np.eye(5), atol=1e-13)


def test_rayleigh_ritz_galerkin_condition():
    H, N = small_h(5, 2)
    Y = oracle.cheb_filter(H, workload.gaussian_block(N, 12, 14), 6, A, B, A0)
    lam, Psi = oracle.rayleigh_ritz(H, Y)
    Rres = H @ Psi - Psi * lam
    assert np.max(np.abs(Y.T @ Rres)) < 1e-10 * np.abs(Y).max()
    assert np.max(np.abs(Psi.T @ (H @ Psi) - np.diag(lam))) < 1e-12
    assert np.all(np.diff(lam) >= 0)


def test_ritz_residuals_exact_eigenpairs():
    # exact eigenpairs of a symmetric matrix have zero residual up to rounding
    ip, ix, d, N = workload.lattice_hamiltonian(5, 2, 3)
    H = oracle.csr_from_arrays(ip, ix, d, N)
    lam, V = np.linalg.eigh(H.toarray())
    res = oracle.ritz_residuals(H, V[:, :20], lam[:20])
    assert res.max() <= 1e-12 * np.abs(lam).max()


def test_ritz_residuals_closed_form():
    # psi = cos(t) v1 + sin(t) v2 for orthonormal eigenvectors (mu1, mu2) and any
    # value l: ||H psi - l psi||^2 = cos^2(t) (mu1 - l)^2 + sin^2(t) (mu2 - l)^2
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    mu = np.linspace(-3.0, 5.0, 30)
    H = sp.csr_matrix((Q * mu) @ Q.T)
    t = np.array([0.0, 0.3, 1.1, np.pi / 2])
    i1, i2 = 4, 17
    Psi = np.cos(t)[None, :] * Q[:, [i1]] + np.sin(t)[None, :] * Q[:, [i2]]
    l = np.array([0.5, -1.0, mu[i1], 2.0])
    want = np.sqrt(np.cos(t) ** 2 * (mu[i1] - l) ** 2 + np.sin(t) ** 2 * (mu[i2] - l) ** 2)
    np.testing.assert_allclose(oracle.ritz_residuals(H, Psi, l), want, rtol=1e-12, atol=1e-13)


def test_chfsi_passes_converge_to_lowest_eigenvalues():
    # repeated passes of Algorithm 1 from a random block: the lowest Ritz values
    # approach the lowest eigenvalues and their residuals shrink
    ip, ix, d, N = workload.lattice_hamiltonian(6, 2, 1)
    H = oracle.csr_from_arrays(ip, ix, d, N)
    exact = np.linalg.eigvalsh(H.toarray())
    X = workload.gaussian_block(N, 24, 1)
    b = exact[-1] + 0.1
    lam, Psi, res = oracle.chfsi(H, X, 10, float(exact[40]), b, float(exact[0]) - 1.0, passes=12)
    keep = 16
    assert np.abs(lam[:keep] - exact[:keep]).max() <= 1e-9
    assert res[:keep].max() <= 1e-6
    np.testing.assert_allclose(Psi.T @ Psi, np.eye(24), atol=1e-12)


def test_fermi_occupancies_degenerate_closed_form():
    # n equal levels e0: every f = N_e / (2n) and mu = e0 - kT ln(2n/N_e - 1)
    e0, n, ne, kT = -0.7, 40, 30.0, 0.01
    f, mu = oracle.fermi_occupancies(np.full(n, e0), ne, kT)
    np.testing.assert_allclose(f, ne / (2 * n), rtol=1e-13)
    assert abs(mu - (e0 - kT * np.log(2 * n / ne - 1))) <= 1e-13


def test_fermi_occupancies_symmetric_two_levels():
    # levels -d and +d, half filled: mu = 0 by symmetry, f = 1 / (1 + exp(-+d / kT))
    d, kT = 0.3, 0.05
    eps = np.r_[np.full(10, -d), np.full(10, d)]
    f, mu = oracle.fermi_occupancies(eps, 20.0, kT)
    assert abs(mu) <= 1e-14
    np.testing.assert_allclose(f[:10], 1 / (1 + np.exp(-d / kT)), rtol=1e-13)
    np.testing.assert_allclose(f[10:], 1 / (1 + np.exp(d / kT)), rtol=1e-13)


def test_fermi_occupancies_count_and_order():
    rng = np.random.default_rng(3)
    eps = np.sort(rng.uniform(-2, 1, 200))
    for ne in (1.0, 57.3, 300.0, 399.0):
        f, mu = oracle.fermi_occupancies(eps, ne, 1.5834e-3)
        assert abs(2 * f.sum() - ne) <= 1e-10 * ne
        assert np.all(np.diff(f) <= 0) and np.all((f >= 0) & (f <= 1))


def test_density_invariants():
    # for Ritz pairs: sum_r rho_r = 2 sum f (orthonormal Psi) and
    # tr(P H) = sum over the pattern of P_rs H_rs = 2 sum_i f_i lambda_i
    ip, ix, d, N = workload.lattice_hamiltonian(6, 2, 2)
    H = oracle.csr_from_arrays(ip, ix, d, N)
    lam, Psi = oracle.rayleigh_ritz(H, workload.gaussian_block(N, 30, 2))
    f, mu = oracle.fermi_occupancies(lam, 24.0, 0.05)
    rho = oracle.electron_density(Psi, f)
    assert abs(rho.sum() - 24.0) <= 1e-10
    Pv = oracle.density_matrix_on_pattern(H, Psi, f)
    assert abs(np.dot(Pv, H.data) - 2 * np.dot(f, lam)) <= 1e-10 * np.abs(lam).max()
    # the diagonal entries of P on the pattern are the density
    diag = np.array([Pv[H.indptr[r]:H.indptr[r + 1]][H.indices[H.indptr[r]:H.indptr[r + 1]] == r][0]
                     for r in range(N)])
    np.testing.assert_allclose(diag, rho, rtol=1e-12, atol=1e-15)


def test_density_matrix_complete_basis_is_twice_identity():
    # all orbitals of a complete orthonormal basis fully occupied: P = 2 I
    ip, ix, d, N = workload.lattice_hamiltonian(4, 1, 0)
    H = oracle.csr_from_arrays(ip, ix, d, N)
    _, V = np.linalg.eigh(H.toarray())
    Pv = oracle.density_matrix_on_pattern(H, V, np.ones(N))
    rows = np.repeat(np.arange(N), np.diff(H.indptr))
    np.testing.assert_allclose(Pv, np.where(rows == H.indices, 2.0, 0.0), atol=1e-13)
