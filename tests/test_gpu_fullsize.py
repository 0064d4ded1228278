"""Full-size parity (216,000 lattice rows, 2048 vectors, degree 20, FP64) in
the launch configuration the benchmark times: the filter is exact per column,
so sampled columns are compared with the oracle run on those columns; the
Rayleigh-Ritz step is compared with the oracle's on whole seeded blocks (all
2048 Ritz values, and the Ritz vectors of well-separated values), and its
output on the filtered block is checked through properties the oracle computes
row by row on the CPU (Ritz values, Galerkin residuals) for sampled pairs."""
import time

import numpy as np
import pytest

import oracle
import workload
from gpu_common import RowSlicedCSR, normwise, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fullsize():
    torch, P = require_gpu()
    cfg = workload.CONFIGS["lattice60_h4_n2048_m20"]
    t0 = time.time()
    ip, ix, d, N = workload.lattice_hamiltonian(cfg.r, cfg.h, cfg.seed)
    Hc = oracle.csr_from_arrays(ip, ix, d, N)
    Hb = P.bsr_build(ip, ix, d, cfg.r, dtype=torch.float64, device="cuda")
    X = workload.gaussian_block(N, cfg.n, cfg.seed)
    Xb = P.to_blocked(torch.from_numpy(X).cuda(), Hb)
    Yb = P.cheb_filter(Hb, Xb, cfg.m, cfg.a, cfg.b, cfg.a0)
    torch.cuda.synchronize()
    print(f"full-size inputs and filter ready in {time.time() - t0:.1f} s", flush=True)
    return cfg, Hc, Hb, X, Yb


def test_fullsize_filter_sampled_columns(fullsize):
    torch, P = require_gpu()
    cfg, Hc, Hb, X, Yb = fullsize
    cols = np.array([0, 1, 777, 1024, 2047])
    Y = P.from_blocked(Yb, Hb)[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    ref = oracle.cheb_filter(Hc, np.ascontiguousarray(X[:, cols]), cfg.m, cfg.a, cfg.b, cfg.a0)
    assert normwise(Y, ref) <= 1e-12
    for j in range(len(cols)):
        assert normwise(Y[:, j], ref[:, j]) <= 1e-11


def test_fullsize_rayleigh_ritz_properties(fullsize):
    torch, P = require_gpu()
    cfg, Hc, Hb, X, Yb = fullsize
    t0 = time.time()
    lam, Psib = P.rayleigh_ritz(Hb, Yb)
    torch.cuda.synchronize()
    print(f"full-size Rayleigh-Ritz {time.time() - t0:.2f} s", flush=True)
    lam = lam.cpu().numpy()
    assert np.all(np.diff(lam) >= 0) and np.all(np.isfinite(lam))
    Psi = P.from_blocked(Psib, Hb)
    G = (Psi.T @ Psi).cpu().numpy()                   # checker only (torch GEMM)
    assert np.max(np.abs(G - np.eye(cfg.n))) <= 1e-12
    Y = P.from_blocked(Yb, Hb).cpu().numpy()
    Psi = Psi.cpu().numpy()
    for i in (0, 1, 100, 1000, 1799, 2047):
        psi = Psi[:, i]
        hpsi = Hc @ psi
        theta = float(psi @ hpsi)
        assert abs(theta - lam[i]) <= 1e-10
        res = hpsi - lam[i] * psi
        # residual orthogonal to the filtered subspace (Galerkin condition)
        gal = Y.T @ res / (np.linalg.norm(Y, axis=0) * max(np.linalg.norm(res), 1e-300))
        # the filtered block has condition ~1e7 after column scaling, so its span is
        # known to ~1e7 * eps; the cosine is bounded by that over the residual size
        assert np.max(np.abs(gal)) <= 1e-6


@pytest.mark.timeout(900)
@pytest.mark.parametrize("block", ["gaussian", "cond1e7"])
def test_fullsize_rayleigh_ritz_vs_oracle(fullsize, block):
    """Steps 2-5 of Algorithm 1 at the full size (216,000 x 2048) against the
    oracle's (Householder basis, projection with the CSR H, LAPACK eigh,
    rotation) on the same seeded block: a Gaussian block (condition ~1.2) and a
    block of condition ~1e7 after column scaling, like the filtered block of the
    timed step.  Bars: every one of the 2048 Ritz values within 1e-10 Ha; for
    the eight Ritz values best separated from their neighbours (gap g), the
    GPU and oracle Ritz vectors within an angle of 1e-10/g (a perturbation of
    the projected matrix of norm 1e-10 moves an eigenvector by at most that,
    Davis-Kahan).  Measured on a 27,000-row proxy with 1024 vectors between two
    correct methods (Householder and Cholesky-QR2): 3.8e-11 Ha and
    angle*gap <= 2.0e-11 at condition 1e7."""
    torch, P = require_gpu()
    cfg, Hc, Hb, X, Yb = fullsize
    N = X.shape[0]
    t0 = time.time()
    Yn = workload.gaussian_block(N, cfg.n, 7) if block == "gaussian" else \
        workload.conditioned_block(N, cfg.n, 8, 1e7)
    print(f"{block}: block generated in {time.time() - t0:.1f} s", flush=True)
    lam, Psib = P.rayleigh_ritz(Hb, P.to_blocked(torch.from_numpy(Yn).cuda(), Hb))
    lam = lam.cpu().numpy()
    Psi = P.from_blocked(Psib, Hb).cpu().numpy()
    del Psib
    torch.cuda.empty_cache()
    t0 = time.time()
    lam_o, Psi_o = oracle.rayleigh_ritz(RowSlicedCSR(Hc), Yn)
    del Yn
    dl = np.abs(lam - lam_o)
    gaps = np.minimum(np.r_[np.inf, np.diff(lam_o)], np.r_[np.diff(lam_o), np.inf])
    worst = 0.0
    for i in np.argsort(-gaps)[:8]:
        sgn = 1.0 if float(Psi[:, i] @ Psi_o[:, i]) >= 0 else -1.0
        worst = max(worst, float(np.linalg.norm(Psi[:, i] - sgn * Psi_o[:, i])) * gaps[i])
    print(f"{block}: oracle Rayleigh-Ritz {time.time() - t0:.1f} s; max |dlambda| {dl.max():.3e} Ha "
          f"(median {np.median(dl):.1e}); max angle*gap {worst:.3e}", flush=True)
    assert dl.max() <= 1e-10
    assert worst <= 1e-10


def _seeded(seed, n, lo, hi):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def test_fullsize_ritz_residuals_sampled_columns(fullsize):
    # the residual definition holds for any block: a seeded random block and
    # seeded values stand in for Ritz pairs (inputs independent of the GPU path)
    torch, P = require_gpu()
    cfg, Hc, Hb, X, Yb = fullsize
    Xb = P.to_blocked(torch.from_numpy(X).cuda(), Hb)
    lam = _seeded(11, cfg.n, -15.0, 10.0)
    res = P.ritz_residuals(Hb, Xb, torch.from_numpy(lam).cuda()).cpu().numpy()
    cols = np.array([0, 5, 1023, 2000, 2047])
    ref = oracle.ritz_residuals(Hc, np.ascontiguousarray(X[:, cols]), lam[cols])
    np.testing.assert_allclose(res[cols], ref, rtol=1e-12)


def test_fullsize_occupancies_and_density_sampled(fullsize):
    torch, P = require_gpu()
    cfg, Hc, Hb, X, Yb = fullsize
    lam = np.sort(_seeded(12, cfg.n, -15.0, 10.0))
    ne = 1.5 * cfg.n
    f, mu = P.fermi_level(torch.from_numpy(lam).cuda(), ne, P.KT_500K_HARTREE)
    f_ref, mu_ref = oracle.fermi_occupancies(lam, ne, P.KT_500K_HARTREE)
    assert abs(mu - mu_ref) <= 1e-12 * max(1.0, abs(mu_ref))
    assert np.abs(f.cpu().numpy() - f_ref).max() <= 1e-12
    # density matrix and site density of the seeded block with these occupancies
    Xb = P.to_blocked(torch.from_numpy(X).cuda(), Hb)
    fd = torch.from_numpy(f_ref).cuda()
    Pv = P.density_matrix(Hb, Xb, fd).reshape(-1).cpu().numpy()
    rng = np.random.default_rng(13)
    entries = rng.choice(len(Hc.data), 3000, replace=False)
    rows = np.searchsorted(Hc.indptr, entries, side="right") - 1
    cols = Hc.indices[entries]
    want = 2.0 * np.einsum("ij,ij->i", X[rows] * f_ref[None, :], X[cols])
    got = Pv[Hb.entry_slot[entries]]
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12 * np.abs(want).max())
    rho = P.from_blocked(P.electron_density(Xb, fd).reshape(-1, 1), Hb).reshape(-1).cpu().numpy()
    sites = rng.choice(X.shape[0], 500, replace=False)
    np.testing.assert_allclose(rho[sites], oracle.electron_density(X[sites], f_ref), rtol=1e-12)


@pytest.mark.parametrize("fmt", ["f32", "bf16", "bf16x3"])
def test_fullsize_reduced_precision_filter_sampled_columns(fullsize, fmt):
    # the oracle filters the sampled columns with exactly the values the GPU holds:
    # fp32(h), bf16(fp32(h)), or hi + lo of the bf16x3 split formed on the CPU;
    # tolerances as at the small sizes: 4*m*u for FP32 (u = 2^-24) and bf16x3
    # (u = 2^-16), 2.5*2^-8 for bf16 tiles (a step's error is damped by the
    # later steps instead of accumulating)
    torch, P = require_gpu()
    cfg, Hc, Hb, X, Yb = fullsize
    ip, ix, d, N = workload.lattice_hamiltonian(cfg.r, cfg.h, cfg.seed)
    h32 = torch.from_numpy(d).float()
    if fmt == "f32":
        Hl, dr, u = P.bsr_astype(Hb, torch.float32), h32.double().numpy(), 2.0 ** -24
    elif fmt == "bf16":
        Hl, dr, u = P.bsr_astype(Hb, torch.bfloat16), h32.bfloat16().double().numpy(), None
    else:
        hi = h32.bfloat16().float()
        lo = (h32 - hi).bfloat16().float()
        Hl, dr, u = P.bsr_astype(Hb, "bf16x3"), hi.double().numpy() + lo.double().numpy(), 2.0 ** -16
    Xl = P.cast(P.to_blocked(torch.from_numpy(X).cuda(), Hb), torch.float32)
    Yl = P.cheb_filter(Hl, Xl, cfg.m, cfg.a, cfg.b, cfg.a0)
    cols = np.array([3, 1500, 2047])
    Y = P.from_blocked(P.cast(Yl, torch.float64), Hb)[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    Xr = np.ascontiguousarray(X[:, cols].astype(np.float32).astype(np.float64))
    ref = oracle.cheb_filter(oracle.csr_from_arrays(ip, ix, dr, N), Xr, cfg.m, cfg.a, cfg.b, cfg.a0)
    err = normwise(Y, ref)
    print(f"full-size {fmt} filter: normwise error {err:.3e}", flush=True)
    assert err <= (2.5 * 2.0 ** -8 if u is None else 4 * cfg.m * u)


def test_fullsize_precision_schedule_warm_ritz_values(fullsize):
    # precision schedule of Algorithm 1 step 1 (Sec. 3.4): BF16 tiles for the first
    # 2 of the 20 steps, bf16x3 split products for the last 18 (FP32 iterates).
    # From a warm start (the FP64 Ritz vectors of one pass), the lowest 1800 Ritz
    # values after the FP64 Rayleigh-Ritz stay within 1e-6 Ha of the FP64 pipeline's,
    # which test_fullsize_rayleigh_ritz_vs_oracle holds to the oracle.  The error a
    # BF16 step leaves grows with its position in the filter (measured 6.5e-7 Ha for
    # 2 steps, 1.2e-6 for 4, 4.1e-6 for 16).
    torch, P = require_gpu()
    cfg, Hc, Hb, X, Yb = fullsize
    lam_c, psi_c = P.rayleigh_ritz(Hb, Yb)
    lam_w, _ = P.rayleigh_ritz(Hb, P.cheb_filter(Hb, psi_c, cfg.m, cfg.a, cfg.b, cfg.a0))
    He, Hl = P.bsr_astype(Hb, torch.bfloat16), P.bsr_astype(Hb, "bf16x3")
    Ys = P.cheb_filter_schedule(He, Hl, cfg.m - 2, P.cast(psi_c, torch.float32), cfg.m, cfg.a, cfg.b,
                                cfg.a0)
    lam_s, _ = P.rayleigh_ritz(Hb, Ys)
    keep = 1800
    err = float((lam_s[:keep] - lam_w[:keep]).abs().max())
    print(f"full-size schedule BF16 x2 + bf16x3 x18, warm: max Ritz error {err:.3e} Ha", flush=True)
    assert err <= 1e-6
