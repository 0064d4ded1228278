"""GPU parity of steps 2-5 of Algorithm 1 (Cholesky-QR, projection, dense
eigensolve, rotation) against the FP64 oracle and LAPACK, through the C ABI."""
import numpy as np
import pytest

import oracle
import workload
from gpu_common import A, A0, B, make_case, normwise, require_gpu

pytestmark = pytest.mark.gpu


def _cuda(x):
    torch, _ = require_gpu()
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# (4096, 256) and (1600, 128): whole 128-column tiles and 16-row panels, which the Gram
# product moves by LDS-DMA; the other shapes take the register-staged tile
@pytest.mark.parametrize("rows,n,cond_exp", [(3000, 100, 4), (1000, 37, 2), (700, 130, 6),
                                             (64, 64, 1), (5000, 1, 0), (2049, 257, 3),
                                             (4096, 256, 3), (1600, 128, 1)])
def test_cholqr2_matches_householder(rows, n, cond_exp):
    print(f"cholqr2 rows={rows} n={n}", flush=True)
    torch, P = require_gpu()
    rng = np.random.default_rng(rows + n)
    Y = rng.standard_normal((rows, n)) * np.logspace(0, cond_exp, n)[None, :]
    Q = P.cholqr2(_cuda(Y)).cpu().numpy()
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 1e-13
    # thin QR with positive diagonal R is unique, so Q equals the oracle's
    ref = oracle.orth(Y)
    assert np.max(np.abs(Q - ref)) <= 1e-13 * 10 ** cond_exp * max(1, n) ** 0.5


def test_cholqr2_low_precision_input_and_in_place():
    torch, P = require_gpu()
    rng = np.random.default_rng(7)
    Y = rng.standard_normal((2000, 90))
    Y32 = _cuda(Y).float()
    Q = P.cholqr2(Y32).cpu().numpy()
    ref = oracle.orth(Y32.double().cpu().numpy())     # the FP32 values, exactly
    assert np.max(np.abs(Q - ref)) <= 1e-12
    Yd = _cuda(Y)
    P.cholqr2(Yd, out=Yd)                              # Q written over an FP64 Y
    assert np.max(np.abs(Yd.cpu().numpy() - oracle.orth(Y))) <= 1e-12


def test_cholqr2_reports_breakdown():
    torch, P = require_gpu()
    rng = np.random.default_rng(8)
    Y = rng.standard_normal((500, 20))
    Y[:, 7] = 0.0                                      # rank-deficient: no orthonormal Q spans Y
    with pytest.raises(P.TtdftError) as ei:
        P.cholqr2(_cuda(Y))
    assert ei.value.name == "TTDFT_ERR_NOT_POSDEF"


@pytest.mark.parametrize("ydtype", ["f64", "f32"])
def test_shifted_cholqr3_fallback_ill_conditioned(ydtype):
    # singular values down to 1e-12: the Gram matrix is singular to working
    # precision, the plain passes break down and the shifted pass takes over
    torch, P = require_gpu()
    rng = np.random.default_rng(9)
    U, _ = np.linalg.qr(rng.standard_normal((3000, 60)))
    V, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    Y = (U * np.logspace(0, -12, 60)) @ V.T
    Yd = _cuda(Y) if ydtype == "f64" else _cuda(Y).float()
    Yh = Yd.double().cpu().numpy()
    Q = P.cholqr2(Yd).cpu().numpy()
    assert np.max(np.abs(Q.T @ Q - np.eye(60))) <= 1e-13
    assert np.linalg.norm(Yh - Q @ (Q.T @ Yh)) <= 1e-12 * np.linalg.norm(Yh)


@pytest.mark.parametrize("ydtype", ["f64", "f32"])
def test_rayleigh_ritz_after_cholqr_breakdown(ydtype):
    """A block with singular values down to 1e-12 breaks the plain Cholesky-QR passes;
    the fused Rayleigh-Ritz then forms X_F explicitly by the shifted Cholesky-QR3.  The
    span of such a block is fixed only to about u / 1e-12, so the checks are the
    properties of the result: orthonormal Ritz vectors spanning Y, diagonal projection."""
    torch, P = require_gpu()
    n = 60
    Hc, Hb, _ = make_case(8, 3, n, seed=7)
    rng = np.random.default_rng(9)
    U, _ = np.linalg.qr(rng.standard_normal((Hc.shape[0], n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Y = (U * np.logspace(0, -12, n)) @ V.T
    Yb = P.to_blocked(_cuda(Y), Hb)
    if ydtype == "f32":
        Yb = Yb.float()
    Yh = P.from_blocked(Yb.double(), Hb).cpu().numpy()
    lam, Psib = P.rayleigh_ritz(Hb, Yb)
    lam, Psi = lam.cpu().numpy(), P.from_blocked(Psib, Hb).cpu().numpy()
    hn = np.abs(np.linalg.eigvalsh(Hc.toarray())).max()
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(Psi.T @ Psi - np.eye(n))) <= 1e-13
    assert np.max(np.abs(Psi.T @ (Hc @ Psi) - np.diag(lam))) <= 1e-12 * hn
    assert np.linalg.norm(Yh - Psi @ (Psi.T @ Yh)) <= 1e-12 * np.linalg.norm(Yh)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 37, 200, 513])
def test_syev_random_symmetric(n):
    print(f"syev n={n}", flush=True)
    torch, P = require_gpu()
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    S = (M + M.T) / 2
    lam, Z = P.syev(_cuda(S))
    lam, Z = lam.cpu().numpy(), Z.cpu().numpy()
    ref = np.linalg.eigvalsh(S)
    nrm = np.abs(ref).max()
    assert np.max(np.abs(lam - ref)) <= 1e-13 * nrm * max(1, n) ** 0.5
    assert np.max(np.abs(Z.T @ Z - np.eye(n))) <= 1e-13
    assert np.max(np.abs(S @ Z - Z * lam)) <= 1e-12 * nrm


def test_syev_closed_form_and_degenerate_spectra():
    torch, P = require_gpu()
    n = 300
    T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)     # known spectrum
    lam, Z = P.syev(_cuda(T))
    k = np.arange(1, n + 1)
    np.testing.assert_allclose(lam.cpu().numpy(), np.sort(2 - 2 * np.cos(k * np.pi / (n + 1))), atol=1e-13)
    # repeated eigenvalues: orthogonal conjugation of a diagonal with clusters.
    # Inverse iteration plus re-orthonormalisation gives eigenvector residuals of
    # order epsilon*|A| for groups separated by more than ~1e-8 |A|; inside a
    # group of nearly equal eigenvalues (0.5 and 0.5 + 1e-10 here) the vectors
    # may mix, and what is accurate is the group's invariant subspace.
    rng = np.random.default_rng(3)
    Qr, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = np.repeat([-3.0, 0.5, 0.5000000001, 7.0], n // 4)
    S = (Qr * d) @ Qr.T
    S = (S + S.T) / 2
    lam, Z = P.syev(_cuda(S))
    lam, Z = lam.cpu().numpy(), Z.cpu().numpy()
    assert np.max(np.abs(lam - np.sort(d))) <= 1e-13 * 7 * n ** 0.5
    assert np.max(np.abs(Z.T @ Z - np.eye(n))) <= 1e-13
    R = S @ Z - Z * lam
    q = n // 4
    sep = np.r_[0:q, 3 * q:n]                                  # the groups at -3 and 7
    assert np.max(np.abs(R[:, sep])) <= 1e-12 * 7
    grp = Z[:, q:3 * q]                                         # 0.5 and 0.5 + 1e-10 together
    assert np.max(np.abs(S @ grp - grp @ (grp.T @ S @ grp))) <= 1e-12 * 7
    lam, Z = P.syev(_cuda(np.eye(5) * 2.5))                  # identity: any orthonormal basis
    np.testing.assert_allclose(lam.cpu().numpy(), 2.5, atol=1e-15)
    assert np.max(np.abs(Z.cpu().numpy().T @ Z.cpu().numpy() - np.eye(5))) <= 1e-14


@pytest.mark.slow
def test_syev_two_launch_tridiagonalisation_above_8192():
    """n = 8200: the reflector no longer fits the 64 KiB of LDS of the fused step, so the
    product and the rank-2 update run as two launches per step.  The spectrum is fixed by
    construction, S = H2 H1 diag(d) H1 H2 with two Householder reflections (built on the
    GPU in FP64); the bounds are those of the n <= 513 cases scaled by sqrt(n / 513)."""
    torch, P = require_gpu()
    n = 8200
    print(f"syev n={n} (two-launch tridiagonalisation)", flush=True)
    rng = np.random.default_rng(11)
    d = np.linspace(-3.0, 7.0, n)
    S = torch.diag(_cuda(d))
    for _ in range(2):
        u = _cuda(rng.standard_normal(n))
        u = u / torch.linalg.vector_norm(u)
        Su = S @ u
        S = S - 2 * torch.outer(u, Su) - 2 * torch.outer(Su, u) + 4 * (u @ Su) * torch.outer(u, u)
    S = 0.5 * (S + S.T)
    lam, Z = P.syev(S)
    grow = (n / 513) ** 0.5
    nrm = 7.0
    assert float((lam.cpu() - torch.from_numpy(d)).abs().max()) <= 1e-13 * nrm * n ** 0.5
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    assert float((Z.T @ Z - eye).abs().max()) <= 1e-13 * grow
    assert float((S @ Z - Z * lam).abs().max()) <= 1e-12 * nrm * grow


# one diagonal tile; 3 x 3 tiles, ragged; 2 x 2 whole tiles (the LDS-DMA Gram product)
@pytest.mark.parametrize("n", [40, 300, 256])
def test_rotate_and_project(n):
    torch, P = require_gpu()
    Hc, Hb, X = make_case(8, 3, n, seed=5)
    Q = oracle.orth(X)
    Qb = P.to_blocked(_cuda(Q), Hb)
    Ad = P.project(Hb, Qb).cpu().numpy()
    ref = Q.T @ (Hc @ Q)
    ref = (ref + ref.T) / 2
    assert normwise(Ad, ref) <= 1e-13
    assert np.array_equal(Ad, Ad.T)
    rng = np.random.default_rng(2)
    Zq = rng.standard_normal((n, n))
    Psi = P.from_blocked(P.rotate(Qb, _cuda(Zq)), Hb).cpu().numpy()
    assert normwise(Psi, Q @ Zq) <= 1e-14


@pytest.mark.parametrize("r,h,n,m", [(20, 3, 64, 10), (10, 3, 16, 16), (12, 2, 150, 8)])
def test_rayleigh_ritz_matches_oracle(r, h, n, m):
    print(f"rayleigh_ritz r={r} h={h} n={n} m={m}", flush=True)
    torch, P = require_gpu()
    Hc, Hb, X = make_case(r, h, n)
    Xb = P.to_blocked(_cuda(X), Hb)
    Yb = P.cheb_filter(Hb, Xb, m, A, B, A0)
    lam, Psib = P.rayleigh_ritz(Hb, Yb)
    lam, Psi = lam.cpu().numpy(), P.from_blocked(Psib, Hb).cpu().numpy()
    Yref = oracle.cheb_filter(Hc, X, m, A, B, A0)
    lref, Pref = oracle.rayleigh_ritz(Hc, Yref)
    hn = np.abs(lref).max()
    assert np.max(np.abs(lam - lref)) <= 1e-10
    assert np.max(np.abs(Psi.T @ Psi - np.eye(n))) <= 1e-12
    assert np.max(np.abs(Psi.T @ (Hc @ Psi) - np.diag(lam))) <= 1e-12 * hn
    # Ritz vectors agree up to sign where the Ritz value is separated from its neighbours
    gaps = np.minimum(np.diff(lref, prepend=-np.inf), np.diff(lref, append=np.inf))
    sep = gaps > 1e-3
    ov = np.abs(np.sum(Psi * Pref, axis=0))
    assert np.all(np.abs(ov[sep] - 1) <= 1e-8)
    assert not Psib.cpu().numpy()[(Hb.perm < 0).cpu().numpy()].any()


@pytest.mark.parametrize("r,h", [(20, 3), (12, 4)])
def test_lanczos_upper_estimates(r, h):
    # theta_max <= lambda_max (a Ritz value of a Krylov subspace); theta plus its
    # Ritz residual reaches lambda_max; the safeguarded bound lies above it
    torch, P = require_gpu()
    Hc, Hb, _ = make_case(r, h, 1)
    lmax = float(np.linalg.eigvalsh(Hc.toarray())[-1])
    theta, est, safe, _ = P.lanczos_bounds(Hb, k=30, seed=1)
    print(f"lambda_max {lmax:.6f}: theta {theta:.6f}, estimate {est:.6f}, safeguarded {safe:.6f}")
    assert theta <= lmax + 1e-10
    assert lmax - theta <= 0.05 * abs(lmax)
    assert est >= lmax - 1e-10 and est - lmax <= 0.5
    assert safe >= est
