"""GPU parity of the convergence test of the subspace iteration (Ritz residual
norms), the Lanczos estimates of both ends of the spectrum (with breakdown),
one pass and the repeated Algorithm 1 (Sec. 3.4) run to convergence in the
library, and the reporting of non-finite blocks, through the C ABI."""
import numpy as np
import pytest

import oracle
import workload
from gpu_common import make_case, require_gpu

pytestmark = pytest.mark.gpu


def _blocked(P, torch, Hb, A):
    return P.to_blocked(torch.from_numpy(np.ascontiguousarray(A)).cuda(), Hb)


@pytest.mark.parametrize("r,h,n", [
    (8, 3, 37),        # 512 rows (one chunk), ragged column block
    (14, 2, 300),      # 14 -> 16 padded: 4096 rows (two chunks), two column blocks
    (5, 3, 1),         # one column
])
def test_ritz_residuals_match_oracle(r, h, n):
    print(f"residuals r={r} h={h} n={n}", flush=True)
    torch, P = require_gpu()
    Hc, Hb, X = make_case(r, h, n, seed=2)
    lam, Psi = oracle.rayleigh_ritz(Hc, X)           # Ritz pairs of a random subspace
    ref = oracle.ritz_residuals(Hc, Psi, lam)
    res = P.ritz_residuals(Hb, _blocked(P, torch, Hb, Psi), torch.from_numpy(lam).cuda())
    got = res.cpu().numpy()
    hnorm = float(np.abs(Hc).sum(axis=1).max())
    assert np.abs(got - ref).max() <= 1e-12 * hnorm
    res2 = P.ritz_residuals(Hb, _blocked(P, torch, Hb, Psi), torch.from_numpy(lam).cuda())
    assert torch.equal(res, res2)                    # fixed-order reductions


def test_ritz_residuals_of_eigenpairs_are_rounding_level():
    torch, P = require_gpu()
    Hc, Hb, _ = make_case(6, 2, 1, seed=5)
    lam, V = np.linalg.eigh(Hc.toarray())
    k = 50
    res = P.ritz_residuals(Hb, _blocked(P, torch, Hb, V[:, :k]), torch.from_numpy(lam[:k]).cuda())
    assert float(res.max()) <= 1e-12 * np.abs(lam).max()


@pytest.mark.parametrize("r,h", [(10, 3), (12, 4)])
def test_lanczos_bounds_bracket_the_spectrum(r, h):
    torch, P = require_gpu()
    Hc, Hb, _ = make_case(r, h, 1)
    ev = np.linalg.eigvalsh(Hc.toarray())
    th_max, est, safe, th_min = P.lanczos_bounds(Hb, k=40, seed=3)
    width = ev[-1] - ev[0]
    print(f"lanczos r={r} h={h}: [{th_min:.4f}, {th_max:.4f}] vs [{ev[0]:.4f}, {ev[-1]:.4f}], safe {safe:.4f}", flush=True)
    assert ev[0] - 1e-10 <= th_min <= ev[0] + 0.05 * width     # Ritz values lie inside the spectrum
    assert th_max <= ev[-1] + 1e-10 <= safe + 2e-10
    again = P.lanczos_bounds(Hb, k=40, seed=3)
    assert again == (th_max, est, safe, th_min)                 # fixed-order reductions


@pytest.mark.parametrize("r,h,k", [(2, 1, 20), (3, 2, 40), (2, 1, 8)])
def test_lanczos_breakdown_still_bounds_the_spectrum(r, h, k):
    # k >= N: the Krylov space becomes invariant after at most N steps (beta
    # vanishes); the bounds must still enclose the whole spectrum (Gershgorin)
    torch, P = require_gpu()
    Hc, Hb, _ = make_case(r, h, 1)
    ev = np.linalg.eigvalsh(Hc.toarray())
    A = np.abs(Hc.toarray())
    rad = A.sum(axis=1) - np.diag(A)
    g_lo, g_hi = float((Hc.diagonal() - rad).min()), float((Hc.diagonal() + rad).max())
    th_max, est, safe, th_min = P.lanczos_bounds(Hb, k=k, seed=1)
    print(f"breakdown r={r} k={k}: spectrum [{ev[0]:.4f}, {ev[-1]:.4f}], Gershgorin [{g_lo:.4f}, {g_hi:.4f}], "
          f"bounds [{th_min:.4f}, {safe:.4f}] est {est:.4f}", flush=True)
    assert np.all(np.isfinite([th_max, est, safe, th_min]))
    assert safe >= ev[-1] - 1e-12 and est >= ev[-1] - 1e-12
    assert th_min <= ev[0] + 1e-12
    assert th_max <= ev[-1] + 1e-10
    if k >= Hc.shape[0]:                 # certain breakdown: the Gershgorin bounds are taken
        assert safe >= g_hi - 1e-12 and th_min <= g_lo + 1e-12


def test_chfsi_pass_matches_oracle_and_next_bounds():
    # one pass through the C entry point against the oracle's filter + Rayleigh-Ritz
    torch, P = require_gpu()
    r, h, n, m = 10, 3, 24, 8
    Hc, H64, X = make_case(r, h, n, seed=7)
    bounds = (-3.0, 2.0, 12.5)
    lam, Psi, res, rec, nxt = P.chfsi_pass(H64, H64, _blocked(P, torch, H64, X), m, bounds, n_conv=20)
    lam_o, Psi_o = oracle.rayleigh_ritz(Hc, oracle.cheb_filter(Hc, X, m, bounds[1], bounds[2], bounds[0]))
    lam = lam.cpu().numpy()
    assert np.abs(lam - lam_o).max() <= 1e-10
    ref = oracle.ritz_residuals(Hc, P.from_blocked(Psi, H64).cpu().numpy(), lam)
    assert np.abs(res.cpu().numpy() - ref).max() <= 1e-11
    assert rec["m"] == m and rec["max_residual"] == pytest.approx(float(ref[:20].max()), abs=1e-11)
    assert nxt == (float(lam.min()), float(lam.max()), 12.5)
    assert P.updated_bounds(torch.from_numpy(lam).cuda(), 12.5) == nxt[:2]


def test_nonfinite_blocks_are_reported():
    torch, P = require_gpu()
    Hc, H64, X = make_case(6, 2, 8, seed=8)
    Xb = _blocked(P, torch, H64, X)
    assert P.check_finite(Xb) == 0
    bad = Xb.clone()
    bad[5, 3] = float("nan")
    bad[70, 0] = float("inf")
    assert P.check_finite(bad) == 2
    assert P.check_finite(P.cast(bad, torch.float32)) == 2
    assert P.check_finite(P.cast(bad, torch.bfloat16)) == 2
    with pytest.raises(P.TtdftError) as err:
        P.rayleigh_ritz(H64, bad)
    assert err.value.name == "TTDFT_ERR_NONFINITE"
    with pytest.raises(P.TtdftError) as err:
        P.cholqr2(bad)
    assert err.value.name == "TTDFT_ERR_NONFINITE"
    with pytest.raises(P.TtdftError) as err:
        P.chfsi_pass(H64, H64, bad, 4, (-3.0, 2.0, 12.5))
    assert err.value.name == "TTDFT_ERR_NONFINITE"


@pytest.mark.parametrize("hname,tol,m", [("f64", 1e-9, 12), ("f32", 1e-5, 12)])
def test_chfsi_solve_converges_to_lowest_eigenvalues(hname, tol, m):
    torch, P = require_gpu()
    r, h, n, n_conv = 10, 3, 40, 32
    Hc, H64, X = make_case(r, h, n, seed=4)
    ev = np.linalg.eigvalsh(Hc.toarray())
    Hf = H64 if hname == "f64" else P.bsr_astype(H64, torch.float32)
    Xb = _blocked(P, torch, H64, X)
    lam, Psi, res, hist = P.chfsi_solve(Hf, H64, Xb, m, tol, n_conv=n_conv, max_iter=60, m_first=2 * m)
    assert not any(h.get("rank_deficient") for h in hist)
    assert [h["pass"] for h in hist] == list(range(1, len(hist) + 1))
    print(f"chfsi {hname}: {len(hist)} passes, residual {hist[-1]['max_residual']:.3e}", flush=True)
    assert hist[-1]["max_residual"] <= tol
    lam = lam.cpu().numpy()
    # a Ritz value is within its residual norm of an eigenvalue
    assert np.abs(lam[:n_conv] - ev[:n_conv]).max() <= 2 * tol
    # the reported residuals are those of the returned pairs
    Psin = P.from_blocked(Psi, H64).cpu().numpy()
    ref = oracle.ritz_residuals(Hc, Psin, lam)
    assert np.abs(res.cpu().numpy() - ref).max() <= 1e-11
    np.testing.assert_allclose(Psin.T @ Psin, np.eye(n), atol=1e-12)
    # bounds follow the Ritz values of the previous pass
    for prev, nxt in zip(hist, hist[1:]):
        assert nxt["a0"] < nxt["a"] < nxt["b"] == prev["b"]


def test_chfsi_solve_converges_from_a_huge_first_degree():
    # degree 4000 from a random start spreads the components of a 128-column
    # block far beyond the FP64 range (condition ~3e19 at the rounding floor):
    # the first pass is either orthonormalised by the shifted Cholesky-QR3
    # fallback or redone at lower degree, and the solve still converges
    torch, P = require_gpu()
    Hc, H64, X = make_case(8, 3, 128, seed=6)
    ev = np.linalg.eigvalsh(Hc.toarray())
    lam, Psi, res, hist = P.chfsi_solve(H64, H64, _blocked(P, torch, H64, X), 10, 1e-9, n_conv=96,
                                        max_iter=40, m_first=4000)
    backed = [h["m"] for h in hist if h.get("rank_deficient")]
    done = [h for h in hist if not h.get("rank_deficient")]
    print(f"degree back-off: {backed}, first accepted degree {done[0]['m']}, {len(done)} passes", flush=True)
    assert done[-1]["max_residual"] <= 1e-9
    assert np.abs(lam.cpu().numpy()[:96] - ev[:96]).max() <= 2e-9
