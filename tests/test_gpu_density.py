"""GPU parity of the occupancies and density after the Rayleigh-Ritz step (the
Fermi-Dirac occupancy, the electron-count constraint and the density of Sec. 2)
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from gpu_common import make_case, require_gpu

pytestmark = pytest.mark.gpu


def _ritz(r, h, n, seed):
    torch, P = require_gpu()
    Hc, Hb, X = make_case(r, h, n, seed=seed)
    lam, Psi = oracle.rayleigh_ritz(Hc, X)
    Psib = P.to_blocked(torch.from_numpy(np.ascontiguousarray(Psi)).cuda(), Hb)
    return torch, P, Hc, Hb, lam, Psi, Psib


@pytest.mark.parametrize("kT,ne", [(0.05, 57.3), (1.5834e-3, 57.3), (0.2, 1.0), (0.01, 127.5)])
def test_fermi_level_matches_oracle(kT, ne):
    torch, P, Hc, Hb, lam, Psi, Psib = _ritz(8, 3, 64, 1)
    f, mu = P.fermi_level(torch.from_numpy(lam).cuda(), ne, kT)
    f_ref, mu_ref = oracle.fermi_occupancies(lam, ne, kT)
    print(f"fermi kT={kT} ne={ne}: mu {mu:.15f} vs {mu_ref:.15f}", flush=True)
    assert abs(mu - mu_ref) <= 1e-12 * max(1.0, abs(mu_ref))
    assert np.abs(f.cpu().numpy() - f_ref).max() <= 1e-12
    assert abs(2 * float(f.sum()) - ne) <= 1e-10 * ne


@pytest.mark.parametrize("r,h,n", [(8, 3, 37), (6, 2, 130), (5, 3, 1)])
def test_density_matrix_and_density_match_oracle(r, h, n):
    torch, P, Hc, Hb, lam, Psi, Psib = _ritz(r, h, n, 2)
    ne = min(1.6 * n, 2 * n - 0.5)
    f_ref, _ = oracle.fermi_occupancies(lam, ne, 0.05)
    f = torch.from_numpy(f_ref).cuda()
    Pv = P.density_matrix(Hb, Psib, f)
    flat = Pv.reshape(-1).cpu().numpy()
    ref = oracle.density_matrix_on_pattern(Hc, Psi, f_ref)
    got = flat[Hb.entry_slot]
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    off = np.ones(flat.size, bool)
    off[Hb.entry_slot] = False
    assert not flat[off].any()                          # outside the pattern: 0
    assert torch.equal(Pv, P.density_matrix(Hb, Psib, f))   # deterministic
    rho = P.electron_density(Psib, f)
    rho_nat = P.from_blocked(rho.reshape(-1, 1), Hb).reshape(-1).cpu().numpy()
    rho_ref = oracle.electron_density(Psi, f_ref)
    assert np.abs(rho_nat - rho_ref).max() <= 1e-13 * max(1.0, rho_ref.max())
    pad = (Hb.perm < 0).cpu().numpy()
    assert not rho.cpu().numpy()[pad].any()
    assert abs(float(rho.sum()) - ne) <= 1e-10 * ne


def test_density_trace_identity_on_gpu_ritz_pairs():
    # tr(P H) over the stored entries equals 2 sum_i f_i lambda_i for Ritz pairs
    torch, P = require_gpu()
    Hc, Hb, X = make_case(10, 3, 48, seed=3)
    Xb = P.to_blocked(torch.from_numpy(X).cuda(), Hb)
    lam, Psi = P.rayleigh_ritz(Hb, P.cheb_filter(Hb, Xb, 8, 2.0, 12.5, -3.0))
    f, mu = P.fermi_level(lam, 60.0, P.KT_500K_HARTREE)
    Pv = P.density_matrix(Hb, Psi, f)
    tr = float((Pv * Hb.vals).sum())
    want = 2.0 * float((f * lam).sum())
    assert abs(tr - want) <= 1e-10 * float(lam.abs().max())
