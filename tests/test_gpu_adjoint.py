"""GPU parity of the adjoint filter (gradients with respect to X and to the
stored entries of H) against the FP64 oracle, a dense Daleckii-Krein reference
and central finite differences, plus bitwise equality of stored and recomputed
checkpointing."""
import numpy as np
import pytest

import oracle
import workload
from gpu_common import A, A0, B, make_case, normwise, require_gpu

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -52


def _cuda(x):
    torch, _ = require_gpu()
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def gpu_grads(Hb, X, W, m, ckpt=0, xdtype=None):
    torch, P = require_gpu()
    Xb = P.to_blocked(_cuda(X), Hb)
    Wb = P.to_blocked(_cuda(W), Hb)
    if xdtype is not None:
        Xb, Wb = P.cast(Xb, xdtype), P.cast(Wb, xdtype)
    dXb, dH = P.cheb_filter_backward(Hb, Xb, Wb, m, A, B, A0, ckpt_every=ckpt)
    torch.cuda.synchronize()
    return dXb, dH


@pytest.mark.parametrize("r,h,n,m", [(8, 3, 24, 6), (10, 3, 16, 16), (6, 2, 70, 1), (9, 2, 33, 2)])
def test_adjoint_f64_matches_oracle(r, h, n, m):
    print(f"adjoint f64 r={r} h={h} n={n} m={m}", flush=True)
    torch, P = require_gpu()
    Hc, Hb, X = make_case(r, h, n, seed=11)
    W = workload.gaussian_block(Hc.shape[0], n, 11, stream="W")
    dXb, dH = gpu_grads(Hb, X, W, m)
    dX = P.from_blocked(dXb, Hb).cpu().numpy()
    rdX, rg = oracle.cheb_filter_adjoint(Hc, X, W, m, A, B, A0)
    assert normwise(dX, rdX) <= 1e-12
    flat = dH.reshape(-1).cpu().numpy()
    assert normwise(flat[Hb.entry_slot], rg) <= 1e-12
    off = np.ones(flat.size, bool)
    off[Hb.entry_slot] = False
    assert not flat[off].any()                       # padding and non-pattern entries are 0
    assert not dXb.cpu().numpy()[(Hb.perm < 0).cpu().numpy()].any()


def _t_closed(m, x):
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    ins = np.abs(x) <= 1
    out[ins] = np.cos(m * np.arccos(x[ins]))
    out[~ins] = np.sign(x[~ins]) ** m * np.cosh(m * np.arccosh(np.abs(x[~ins])))
    return out


def test_adjoint_dense_daleckii_krein_lattice10():
    # dense reference gradient G = V [(V^T W X^T V) o F] V^T, F the divided
    # differences of p at the eigenvalues (lattice 10 is padded to 12)
    torch, P = require_gpu()
    cfg = workload.CONFIGS["lattice10_h3_n16_m16"]
    Hc, Hb, X = make_case(cfg.r, cfg.h, cfg.n, seed=cfg.seed)
    W = workload.gaussian_block(Hc.shape[0], cfg.n, cfg.seed, stream="W")
    _, dH = gpu_grads(Hb, X, W, cfg.m)
    lam, V = np.linalg.eigh(Hc.toarray())
    e, c = (B - A) / 2, (B + A) / 2
    x = (lam - c) / e
    xi, xj = x[:, None], x[None, :]
    d_prev, d = np.zeros_like(xi * xj), np.ones_like(xi * xj)
    for k in range(1, cfg.m):
        d_prev, d = d, 2 * xi * d + 2 * _t_closed(k, xj) - d_prev
    F = d / (e * _t_closed(cfg.m, np.array([(A0 - c) / e]))[0])
    G = V @ ((V.T @ W @ X.T @ V) * F) @ V.T
    rows = np.repeat(np.arange(Hc.shape[0]), np.diff(Hc.indptr))
    ref = G[rows, Hc.indices]
    got = dH.reshape(-1).cpu().numpy()[Hb.entry_slot]
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.fixture(scope="module")
def lattice40():
    torch, P = require_gpu()
    cfg = workload.CONFIGS["lattice40_h3_n512_m16"]
    Hc, Hb, X = make_case(cfg.r, cfg.h, cfg.n, seed=cfg.seed)
    W = workload.gaussian_block(Hc.shape[0], cfg.n, cfg.seed, stream="W")
    return cfg, Hc, Hb, X, W


@pytest.mark.parametrize("ckpt", [3, 4, 5])
def test_adjoint_checkpointing_bitwise_f64(lattice40, ckpt):
    torch, P = require_gpu()
    cfg, Hc, Hb, X, W = lattice40
    dX0, dH0 = gpu_grads(Hb, X, W, cfg.m, ckpt=0)
    dX1, dH1 = gpu_grads(Hb, X, W, cfg.m, ckpt=ckpt)
    assert torch.equal(dX0, dX1) and torch.equal(dH0, dH1)


def test_adjoint_checkpointing_bitwise_f32(lattice40):
    torch, P = require_gpu()
    cfg, Hc, _, X, W = lattice40
    ip, ix, d, N = workload.lattice_hamiltonian(cfg.r, cfg.h, cfg.seed)
    H32 = P.bsr_build(ip, ix, d, cfg.r, dtype=torch.float32, device="cuda")
    dX0, dH0 = gpu_grads(H32, X, W, cfg.m, ckpt=0, xdtype=torch.float32)
    dX1, dH1 = gpu_grads(H32, X, W, cfg.m, ckpt=4, xdtype=torch.float32)
    assert torch.equal(dX0, dX1) and torch.equal(dH0, dH1)
    # FP32 adjoint against the FP64 adjoint of the same problem
    dX64, dH64 = gpu_grads(lattice40[2], X, W, cfg.m)
    assert normwise(dX0.double().cpu().numpy(), dX64.cpu().numpy()) <= 1e-4
    slot = lattice40[2].entry_slot
    assert normwise(dH0.reshape(-1).double().cpu().numpy()[slot],
                    dH64.reshape(-1).cpu().numpy()[slot]) <= 1e-4


def test_adjoint_finite_differences_fullsize(lattice40):
    """Central differences, step 1e-6, FP64, at the full adjoint workload: 64
    entries of X (one column changes, so the difference is formed per element
    before summing) and 64 symmetric pairs of H (dL = G_ij + G_ji).

    The loss is linear in X and a degree-m polynomial in H, so with h = 1e-6
    the central difference is limited by rounding: each check allows
    4 * eps * sum|w| (|y+| + |y-|) / (2h), evaluated from the two runs, plus
    1e-7 relative."""
    torch, P = require_gpu()
    cfg, Hc, Hb, X, W = lattice40
    hstep = 1e-6
    Xb = P.to_blocked(_cuda(X), Hb)
    Wb = P.to_blocked(_cuda(W), Hb)
    dXb, dH = P.cheb_filter_backward(Hb, Xb, Wb, cfg.m, A, B, A0)
    rng = np.random.default_rng(2024)
    inv = Hb.inv_perm.cpu().numpy()
    worst = 0.0
    for _ in range(64):
        i, j = int(rng.integers(Hc.shape[0])), int(rng.integers(cfg.n))
        bi = int(inv[i])
        col = Xb[:, j:j + 1].clone()
        col[bi, 0] += hstep
        yp = P.cheb_filter(Hb, col, cfg.m, A, B, A0)
        col[bi, 0] -= 2 * hstep
        ym = P.cheb_filter(Hb, col, cfg.m, A, B, A0)
        fd = float((Wb[:, j] * (yp[:, 0] - ym[:, 0])).sum()) / (2 * hstep)
        noise = EPS * float((Wb[:, j].abs() * (yp[:, 0].abs() + ym[:, 0].abs())).sum()) / (2 * hstep)
        g = float(dXb[bi, j])
        worst = max(worst, abs(fd - g) / (4 * noise + 1e-7 * abs(g)))
    assert worst <= 1.0, worst
    rows = np.repeat(np.arange(Hc.shape[0]), np.diff(Hc.indptr))
    pos = {}
    cols = Hc.indices
    flat_dH = dH.reshape(-1)
    vals = Hb.vals.view(-1)
    worst = 0.0
    for t in rng.choice(Hc.nnz, 64, replace=False):
        i, j = int(rows[t]), int(cols[t])
        lo, hi = Hc.indptr[j], Hc.indptr[j + 1]
        tt = lo + int(np.searchsorted(cols[lo:hi], i))
        slots = sorted({int(Hb.entry_slot[t]), int(Hb.entry_slot[tt])})
        orig = vals[slots].clone()
        vals[slots] = orig + hstep
        yp = P.cheb_filter(Hb, Xb, cfg.m, A, B, A0)
        vals[slots] = orig - hstep
        ym = P.cheb_filter(Hb, Xb, cfg.m, A, B, A0)
        vals[slots] = orig
        fd = float((Wb * (yp - ym)).sum()) / (2 * hstep)
        noise = EPS * float((Wb.abs() * (yp.abs() + ym.abs())).sum()) / (2 * hstep)
        g = float(sum(flat_dH[s] for s in slots))
        worst = max(worst, abs(fd - g) / (4 * noise + 1e-7 * abs(g)))
    assert worst <= 1.0, worst


def test_autograd_function_matches_backward():
    torch, P = require_gpu()
    Hc, Hb, X = make_case(8, 2, 20, seed=3)
    W = workload.gaussian_block(Hc.shape[0], 20, 3, stream="W")
    Xb = P.to_blocked(_cuda(X), Hb).requires_grad_(True)
    Wb = P.to_blocked(_cuda(W), Hb)
    Hb.vals.requires_grad_(True)
    Y = P.cheb_filter_autograd(Hb, Xb, 7, A, B, A0, ckpt_every=3)
    (Wb * Y).sum().backward()
    dX, dH = P.cheb_filter_backward(Hb, Xb.detach(), Wb, 7, A, B, A0)
    assert torch.equal(Xb.grad, dX) and torch.equal(Hb.vals.grad, dH)
    Hb.vals.requires_grad_(False)
