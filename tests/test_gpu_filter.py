"""GPU parity of the Chebyshev filter (Algorithm 1, step 1) against the FP64
oracle, through the C ABI.  FP64 bar: normwise relative error <= 1e-12."""
import numpy as np
import pytest

import oracle
from gpu_common import A, A0, B, make_case, normwise, require_gpu

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-12


def gpu_filter(Hb, X, m, a=A, b=B, a0=A0, xdtype=None):
    torch, P = require_gpu()
    xdtype = xdtype or torch.float64
    Xd = torch.from_numpy(X).cuda()
    Xb = P.to_blocked(Xd, Hb)
    if xdtype != torch.float64:
        Xb = P.cast(Xb, xdtype)
    Yb = P.cheb_filter(Hb, Xb, m, a, b, a0)
    if xdtype != torch.float64:
        Yb = P.cast(Yb, torch.float64)
    torch.cuda.synchronize()
    return Yb, P.from_blocked(Yb, Hb).cpu().numpy()


@pytest.mark.parametrize("r,h,n,m", [
    (20, 3, 64, 10),      # small full case: 8000 rows, 125 block rows
    (6, 2, 37, 7),        # lattice padded 6 -> 8, ragged column tile
    (5, 3, 1, 1),         # one vector, degree one
    (9, 3, 130, 3),       # three column tiles, the last ragged
    (10, 3, 16, 16),      # r not a multiple of 4
    (8, 4, 64, 2),        # widest stencil, exact blocks
])
def test_filter_f64_matches_oracle(r, h, n, m):
    print(f"filter f64 r={r} h={h} n={n} m={m}", flush=True)
    torch, P = require_gpu()
    Hc, Hb, X = make_case(r, h, n)
    Yb, Y = gpu_filter(Hb, X, m)
    ref = oracle.cheb_filter(Hc, X, m, A, B, A0)
    assert normwise(Y, ref) <= TOL_F64
    pad = (Hb.perm < 0).cpu().numpy()
    assert not Yb.cpu().numpy()[pad].any()      # padding rows stay zero


def test_filter_f64_bitwise_deterministic_and_column_equivariant():
    torch, P = require_gpu()
    Hc, Hb, X = make_case(12, 3, 96, seed=3)
    _, Y1 = gpu_filter(Hb, X, 9)
    _, Y2 = gpu_filter(Hb, X, 9)
    np.testing.assert_array_equal(Y1, Y2)
    perm = np.random.default_rng(0).permutation(96)
    _, Yp = gpu_filter(Hb, np.ascontiguousarray(X[:, perm]), 9)
    np.testing.assert_array_equal(Yp, Y1[:, perm])


def test_cheb_step_general_coefficients_and_in_place():
    torch, P = require_gpu()
    Hc, Hb, X = make_case(8, 3, 70, seed=4)
    Xd = P.to_blocked(torch.from_numpy(X).cuda(), Hb)
    Zp = P.to_blocked(torch.from_numpy(np.cos(X)).cuda(), Hb)
    alpha, c, beta = 0.37, -1.25, 0.81
    out = P.cheb_step(Hb, Xd, Zp, alpha, c, beta)
    ref = alpha * (Hc @ X - c * X) - beta * np.cos(X)
    got = P.from_blocked(out, Hb).cpu().numpy()
    assert normwise(got, ref) <= TOL_F64
    P.cheb_step(Hb, Xd, Zp, alpha, c, beta, out=Zp)          # Yout == Yprev
    np.testing.assert_array_equal(P.from_blocked(Zp, Hb).cpu().numpy(), got)
    out0 = P.cheb_step(Hb, Xd, None, 1.0, 0.0, 0.0)           # plain H X
    assert normwise(P.from_blocked(out0, Hb).cpu().numpy(), Hc @ X) <= TOL_F64


def test_filter_special_case_shift_identity():
    # H = cI gives Y = cos(m pi/2) / T_m(tau) X (zero for odd m)
    torch, P = require_gpu()
    r = 4
    N = r ** 3
    c = (A + B) / 2
    ip = np.arange(N + 1, dtype=np.int64)
    ix = np.arange(N, dtype=np.int32)
    d = np.full(N, c)
    Hb = P.bsr_build(ip, ix, d, r, dtype=torch.float64, device="cuda")
    X = np.random.default_rng(1).standard_normal((N, 8))
    for m in (3, 4):
        _, Y = gpu_filter(Hb, X, m)
        tau = (A0 - c) / ((B - A) / 2)
        expect = np.cos(m * np.pi / 2) / oracle.chebyshev_T(m, tau) * X
        np.testing.assert_allclose(Y, expect, atol=1e-15 * np.abs(X).max() / abs(oracle.chebyshev_T(m, tau)))


@pytest.mark.parametrize("r,h", [(12, 4), (12, 3), (10, 2)])
def test_zero_fragment_skipping_is_exact(r, h):
    # skipping all-zero 16x4 sub-blocks removes only products with zero operands
    torch, P = require_gpu()
    Hc, Hb, X = make_case(r, h, 150, seed=9)
    Xb = P.to_blocked(torch.from_numpy(X).cuda(), Hb)
    Y1 = P.cheb_filter(Hb, Xb, 6, A, B, A0)
    Hb.skip_zero_fragments = False
    Y0 = P.cheb_filter(Hb, Xb, 6, A, B, A0)
    Hb.skip_zero_fragments = True
    assert torch.equal(Y0, Y1)
    fm = Hb.frag_mask.cpu().numpy().view(np.uint64)
    skipped = 1 - np.mean([bin(int(v)).count("1") for v in fm]) / 64
    print(f"r={r} h={h}: {skipped:.1%} of matrix-core sub-blocks skipped", flush=True)
    assert skipped > 0
