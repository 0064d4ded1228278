"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, rejects bad arguments before any device work, and the host
BSR builder reproduces the CSR matrix exactly."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x10000  # never dereferenced: validation fails before any device access


def declared_symbols():
    syms = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            syms |= set(re.findall(r"^\S.*?\b(ttdft_\w+)\s*\(", txt, flags=re.M))
    return syms


def test_exports_every_declared_symbol(lib_built):
    from paper_2110_15853_amd import _lib
    lib = C.CDLL(lib_built)
    syms = declared_symbols()
    assert len(syms) >= 10
    for s in sorted(syms):
        assert hasattr(lib, s), s
    assert syms <= set(_lib.SIGNATURES), sorted(syms - set(_lib.SIGNATURES))


def _lib():
    from paper_2110_15853_amd import _lib as L
    return L


def _fake_bsr(nbr=8, nt=64, dtype=0):
    return _lib().Bsr(nbr, nt, FAKE, FAKE, FAKE, dtype, None)


def _filter(**kw):
    L = _lib()
    args = dict(H=_fake_bsr(), X=FAKE, ldx=16, Y=FAKE * 1000, ldy=16, n=16, m=10, a=2.0,
                b=12.5, a0=-3.0, dt=0, work=FAKE * 100000, wb=1 << 40, s=None)
    args.update(kw)
    H = args["H"]
    return L.load().ttdft_cheb_filter(C.byref(H) if H is not None else None, args["X"], args["ldx"],
                                      args["Y"], args["ldy"], args["n"], args["m"], args["a"],
                                      args["b"], args["a0"], args["dt"], args["work"], args["wb"],
                                      args["s"])


@pytest.mark.parametrize("kw,status", [
    (dict(H=None), "TTDFT_ERR_NULL"),
    (dict(X=None), "TTDFT_ERR_NULL"),
    (dict(a0=2.0), "TTDFT_ERR_BOUNDS"),
    (dict(b=2.0), "TTDFT_ERR_BOUNDS"),
    (dict(a=float("nan")), "TTDFT_ERR_BOUNDS"),
    (dict(b=float("inf")), "TTDFT_ERR_BOUNDS"),
    (dict(m=0), "TTDFT_ERR_DEGREE"),
    (dict(m=-3), "TTDFT_ERR_DEGREE"),
    (dict(n=0), "TTDFT_ERR_SHAPE"),
    (dict(ldx=8), "TTDFT_ERR_SHAPE"),
    (dict(dt=7), "TTDFT_ERR_DTYPE"),
    (dict(dt=1), "TTDFT_ERR_DTYPE"),          # F64 H with F32 X
    (dict(H=_fake_bsr(dtype=2), dt=0), "TTDFT_ERR_DTYPE"),
    (dict(H=_fake_bsr(nbr=0)), "TTDFT_ERR_SHAPE"),
    (dict(Y=FAKE + 8), "TTDFT_ERR_ALIAS"),    # Y overlaps X
    (dict(work=FAKE + 64), "TTDFT_ERR_ALIAS"),
    (dict(wb=10), "TTDFT_ERR_WORKSPACE"),
    (dict(work=None), "TTDFT_ERR_WORKSPACE"),
])
def test_filter_validation(lib_built, kw, status):
    L = _lib()
    st = _filter(**kw)
    assert L.STATUS[st] == status, L.load().ttdft_last_error()
    assert L.load().ttdft_last_error().decode() != ""


def test_filter_schedule_validation(lib_built):
    L = _lib()
    lib = L.load()

    def call(He=None, Hl=None, m_late=4, m=10, dt=1, work=FAKE * 100000, wb=1 << 40):
        He = He if He is not None else _fake_bsr(dtype=2)
        Hl = Hl if Hl is not None else _fake_bsr(dtype=1)
        return L.STATUS[lib.ttdft_cheb_filter_schedule(C.byref(He), C.byref(Hl), m_late, FAKE, 16,
                                                       FAKE * 1000, 16, 16, m, 2.0, 12.5, -3.0, dt,
                                                       work, wb, None)]

    assert call(m_late=11) == "TTDFT_ERR_DEGREE"
    assert call(m_late=-1) == "TTDFT_ERR_DEGREE"
    assert call(Hl=_fake_bsr(nbr=9, dtype=1)) == "TTDFT_ERR_SHAPE"
    assert call(Hl=_fake_bsr(nt=65, dtype=1)) == "TTDFT_ERR_SHAPE"
    assert call(Hl=_fake_bsr(dtype=0)) == "TTDFT_ERR_DTYPE"      # F64 tiles with F32 iterates
    assert call(wb=10) == "TTDFT_ERR_WORKSPACE"
    assert call(work=FAKE + 64) == "TTDFT_ERR_ALIAS"


def test_filter_noalloc_validation(lib_built):
    # the same argument checks as ttdft_cheb_filter, and a work block larger than
    # the fixed 64 MiB scratch is rejected before any device work
    L = _lib()
    lib = L.load()

    def call(H=None, X=FAKE, Y=FAKE * 1000, n=16, m=10, a0=-3.0, dt=0):
        H = H if H is not None else _fake_bsr()
        return L.STATUS[lib.ttdft_cheb_filter_noalloc(C.byref(H), X, n, Y, n, n, m, 2.0, 12.5, a0,
                                                      dt, None)]

    assert call(X=None) == "TTDFT_ERR_NULL"
    assert call(a0=2.0) == "TTDFT_ERR_BOUNDS"
    assert call(m=0) == "TTDFT_ERR_DEGREE"
    assert call(Y=FAKE + 8) == "TTDFT_ERR_ALIAS"
    assert call(dt=1) == "TTDFT_ERR_DTYPE"
    # 2048 block rows x 64 rows x 1024 vectors x 8 bytes = 1 GiB > 64 MiB
    big = _fake_bsr(nbr=2048)
    assert call(H=big, n=1024, Y=FAKE * 100000) == "TTDFT_ERR_WORKSPACE"
    assert "scratch" in lib.ttdft_last_error().decode()
    # the limit is 64 MiB = 128 block rows x 64 rows x 1024 vectors x 8 bytes: one
    # block row more is rejected (the accepted side runs on the GPU test)
    assert call(H=_fake_bsr(nbr=129), n=1024, Y=FAKE * 100000) == "TTDFT_ERR_WORKSPACE"


def test_step_and_cast_validation(lib_built):
    L = _lib()
    lib = L.load()
    H = _fake_bsr()
    st = lib.ttdft_cheb_step(C.byref(H), FAKE, 16, None, 0, FAKE * 1000, 16, 16, 1.0, 0.0, 0.5, 0, None)
    assert L.STATUS[st] == "TTDFT_ERR_NULL"            # beta != 0 needs Yprev
    st = lib.ttdft_cheb_step(C.byref(H), FAKE, 16, None, 0, FAKE, 16, 16, 1.0, 0.0, 0.0, 0, None)
    assert L.STATUS[st] == "TTDFT_ERR_ALIAS"           # Yout overlaps Yk
    st = lib.ttdft_cheb_step(C.byref(H), FAKE, 16, None, 0, FAKE * 1000, 16, 16, float("nan"), 0.0, 0.0, 0, None)
    assert L.STATUS[st] == "TTDFT_ERR_NONFINITE"
    st = lib.ttdft_cast(FAKE, 0, 16, FAKE + 8, 1, 16, 4, 16, None)
    assert L.STATUS[st] == "TTDFT_ERR_ALIAS"
    st = lib.ttdft_cast(FAKE, 0, 8, FAKE * 1000, 1, 16, 4, 16, None)
    assert L.STATUS[st] == "TTDFT_ERR_SHAPE"
    st = lib.ttdft_gather_rows(FAKE, 16, 4, FAKE * 1000, 16, 4, 16, None, 0, None)
    assert L.STATUS[st] == "TTDFT_ERR_NULL"
    assert lib.ttdft_status_string(8).decode() == "Cholesky breakdown"


def _bsr_host(r, h, dtype_code, seed=0):
    L = _lib()
    lib = L.load()
    ip, ix, d, N = workload.lattice_hamiltonian(r, h, seed)
    nbr, nt = C.c_int64(), C.c_int64()
    P = lambda a: C.c_void_p(a.ctypes.data)
    assert lib.ttdft_bsr_plan(r, P(ip), P(ix), C.byref(nbr), C.byref(nt)) == 0
    nbr, nt = nbr.value, nt.value
    tptr, tcol = np.empty(nbr + 1, np.int32), np.empty(nt, np.int32)
    vals = np.empty(nt * 4096, {0: np.float64, 1: np.float32, 2: np.uint16}[dtype_code])
    perm, slot, mask = np.empty(nbr * 64, np.int64), np.empty(len(d), np.int64), np.empty(nt * 64, np.uint64)
    fmask = np.empty(nt, np.uint64)
    assert lib.ttdft_bsr_build(r, P(ip), P(ix), P(d), dtype_code, P(tptr), P(tcol), P(vals), P(perm),
                               P(slot), P(mask), P(fmask)) == 0
    return (ip, ix, d, N), (nbr, nt, tptr, tcol, vals, perm, slot, mask, fmask)


def documented_block_coords(nb):
    """Block number -> lattice block coordinates, from the numbering rule stated
    with ttdft_bsr: complete 2x2x2 patches first, then incomplete ones."""
    np_ = (nb + 1) // 2
    out = []
    for complete in (True, False):
        for pi in range(np_):
            for pj in range(np_):
                for pk in range(np_):
                    full = 2 * pi + 1 < nb and 2 * pj + 1 < nb and 2 * pk + 1 < nb
                    if full != complete:
                        continue
                    for d in range(8):
                        b = (2 * pi + (d >> 2), 2 * pj + ((d >> 1) & 1), 2 * pk + (d & 1))
                        if max(b) < nb:
                            out.append(b)
    return np.array(out)


@pytest.mark.parametrize("r,h", [(4, 1), (6, 2), (10, 3), (8, 4), (5, 3), (12, 4)])
def test_bsr_builder_roundtrip(lib_built, r, h):
    (ip, ix, d, N), (nbr, nt, tptr, tcol, vals, perm, slot, mask, fmask) = _bsr_host(r, h, 0)
    nb = (r + 3) // 4
    assert nbr == nb ** 3 and tptr[-1] == nt
    Hd = oracle.csr_from_arrays(ip, ix, d, N).toarray()
    dense = np.zeros((nbr * 64, nbr * 64))
    # documented tile layout (fragment order): entry (i, j) at 64*(4*(j/4) + i/16) + 16*(j%4) + i%16
    ii, jj = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    pos = 64 * (4 * (jj // 4) + ii // 16) + 16 * (jj % 4) + ii % 16
    assert sorted(pos.ravel()) == list(range(4096))
    for B in range(nbr):
        assert np.all(np.diff(tcol[tptr[B]:tptr[B + 1]]) > 0)
        for t in range(tptr[B], tptr[B + 1]):
            dense[B * 64:(B + 1) * 64, tcol[t] * 64:(tcol[t] + 1) * 64] = vals[t * 4096:(t + 1) * 4096][pos]
    real = perm >= 0
    assert real.sum() == N and sorted(perm[real]) == list(range(N))
    back = np.zeros((N, N))
    back[np.ix_(perm[real], perm[real])] = dense[np.ix_(real, real)]
    np.testing.assert_array_equal(back, Hd)            # bitwise
    assert not dense[~real].any() and not dense[:, ~real].any()
    np.testing.assert_array_equal(vals[slot], d)
    # mask marks exactly the stored entries (bits in row-major (i, j) of each tile)
    stored = np.zeros(nt * 4096, bool)
    stored[slot] = True
    bits = stored.reshape(nt, 4096)[:, pos.ravel()].reshape(-1)
    weights = (np.uint64(1) << np.arange(64, dtype=np.uint64))
    words = (bits.reshape(nt * 64, 64).astype(np.uint64) * weights).sum(axis=1, dtype=np.uint64)
    np.testing.assert_array_equal(words, mask)
    # fragment mask: bit 4*kk + mb set iff the 16x4 sub-block holds a stored entry
    sub = bits.reshape(nt, 4, 16, 16, 4).any(axis=(2, 4))          # [t][mb][kk]
    fw = (sub.transpose(0, 2, 1).reshape(nt, 64).astype(np.uint64) * weights).sum(axis=1, dtype=np.uint64)
    np.testing.assert_array_equal(fw, fmask)
    # block numbering as documented: complete 2x2x2 patches first (8 consecutive
    # numbers each, blocks in (i, j, k) order, patches lexicographic), then the
    # blocks of incomplete patches; the row of site (i, j, k) is 64*block + local
    coords = documented_block_coords(nb)
    assert sorted(map(tuple, coords)) == [(a, b, c) for a in range(nb) for b in range(nb) for c in range(nb)]
    for row in np.flatnonzero(real)[:: max(1, real.sum() // 500)]:
        I = perm[row]
        i, j, k = I // (r * r), (I // r) % r, I % r
        assert tuple(coords[row // 64]) == (i // 4, j // 4, k // 4)
        assert row % 64 == 16 * (2 * ((i % 4) // 2) + (j % 4) // 2) + 4 * (2 * (i % 2) + j % 2) + k % 4
    if nb >= 2:
        assert [tuple(coords[q]) for q in range(8)] == [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    # lattice blocking: every tile couples blocks at most one block apart per axis when h <= 4
    for B in range(nbr):
        for t in range(tptr[B], tptr[B + 1]):
            assert np.abs(coords[tcol[t]] - coords[B]).max() <= 1


def test_bsr_builder_low_precision_rounding(lib_built):
    import torch
    (ip, ix, d, N), (_, _, _, _, v32, _, slot, _, _) = _bsr_host(5, 2, 1)
    np.testing.assert_array_equal(v32[slot], d.astype(np.float32))
    (ip, ix, d, N), (_, _, _, _, v16, _, slot, _, _) = _bsr_host(5, 2, 2)
    ref = torch.from_numpy(d.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(v16[slot], ref)


def test_bsr_builder_bf16_fragment_order(lib_built):
    # BF16 tiles are stored in the 16x32 fragment order of the bf16 op: entry
    # (i, j) of tile t at t*4096 + 512*(4*(j//32) + i//16) + 8*(i%16 + 16*((j%32)//8)) + j%8,
    # the same entries as the FP64 tiles (16x4 order) hold
    from paper_2110_15853_amd.api import _slots_16x32
    (_, _, d, _), (_, nt, _, _, v64, _, s64, _, _) = _bsr_host(6, 3, 0)
    (_, _, _, _), (_, nt16, _, _, v16, _, s16, _, _) = _bsr_host(6, 3, 2)
    assert nt16 == nt
    ii, jj = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    p4 = 64 * (4 * (jj // 4) + ii // 16) + 16 * (jj % 4) + ii % 16
    p32 = 512 * (4 * (jj // 32) + ii // 16) + 8 * (ii % 16 + 16 * ((jj % 32) // 8)) + jj % 8
    assert sorted(p32.ravel()) == list(range(4096))
    t, p = np.divmod(s64, 4096)
    inv4 = np.empty(4096, np.int64)
    inv4[p4.ravel()] = np.arange(4096)
    want = t * 4096 + p32.ravel()[inv4[p]]
    np.testing.assert_array_equal(s16, want)
    np.testing.assert_array_equal(_slots_16x32(s64, 4096), want)
    import torch
    ref = torch.from_numpy(d.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(v16[want], ref)
    stored = np.zeros(nt * 4096, bool)
    stored[want] = True
    assert not v16[~stored].any()


def test_bsr_builder_rejects_bad_csr(lib_built):
    L = _lib()
    lib = L.load()
    ip = np.array([0, 2, 3, 4, 5, 6, 7, 8, 9], np.int64)      # r = 2, N = 8
    ix = np.array([1, 0, 2, 3, 4, 5, 6, 7, 8], np.int32)       # row 0 unsorted; col 8 out of range
    nbr, nt = C.c_int64(), C.c_int64()
    P = lambda a: C.c_void_p(a.ctypes.data)
    st = lib.ttdft_bsr_plan(2, P(ip), P(ix), C.byref(nbr), C.byref(nt))
    assert L.STATUS[st] == "TTDFT_ERR_PATTERN"
    st = lib.ttdft_bsr_plan(0, P(ip), P(ix), C.byref(nbr), C.byref(nt))
    assert L.STATUS[st] == "TTDFT_ERR_SHAPE"


def test_rayleigh_ritz_and_backward_validation(lib_built):
    L = _lib()
    lib = L.load()
    H64, H32 = _fake_bsr(), _fake_bsr(dtype=1)
    big = 1 << 40
    # Rayleigh-Ritz needs an FP64 H
    st = lib.ttdft_rayleigh_ritz(C.byref(H32), FAKE, 16, 1, 16, FAKE * 10, FAKE * 1000, 16, FAKE * 100000, big, None)
    assert L.STATUS[st] == "TTDFT_ERR_DTYPE"
    st = lib.ttdft_rayleigh_ritz(C.byref(H64), FAKE, 16, 0, 16, None, FAKE * 1000, 16, FAKE * 100000, big, None)
    assert L.STATUS[st] == "TTDFT_ERR_NULL"
    st = lib.ttdft_rayleigh_ritz(C.byref(H64), FAKE, 16, 0, 16, FAKE * 10, FAKE * 1000, 16, FAKE * 100000, 8, None)
    assert L.STATUS[st] == "TTDFT_ERR_WORKSPACE"
    st = lib.ttdft_cholqr2(FAKE, 16, 0, 8, 16, FAKE * 1000, 16, FAKE * 100000, big, None)
    assert L.STATUS[st] == "TTDFT_ERR_SHAPE"                      # fewer rows than vectors
    st = lib.ttdft_cholqr2(FAKE, 16, 1, 100, 16, FAKE, 16, FAKE * 100000, big, None)
    assert L.STATUS[st] == "TTDFT_ERR_ALIAS"                      # F32 Y cannot alias Q
    st = lib.ttdft_syev(10, FAKE, 10, FAKE * 1000, FAKE + 8, 10, FAKE * 100000, big, None)
    assert L.STATUS[st] == "TTDFT_ERR_ALIAS"
    st = lib.ttdft_syev(0, FAKE, 10, FAKE * 1000, FAKE * 3000, 10, FAKE * 100000, big, None)
    assert L.STATUS[st] == "TTDFT_ERR_SHAPE"
    st = lib.ttdft_rotate(FAKE, 16, 100, 16, FAKE * 1000, 16, FAKE + 16, 16, None)
    assert L.STATUS[st] == "TTDFT_ERR_ALIAS"
    st = lib.ttdft_project(C.byref(H32), FAKE, 16, 16, FAKE * 1000, 16, FAKE * 100000, big, None)
    assert L.STATUS[st] == "TTDFT_ERR_DTYPE"
    # backward
    bw = lambda **kw: lib.ttdft_cheb_filter_backward(
        C.byref(kw.get("H", H64)), FAKE, 16, FAKE * 1000, 16, 16, kw.get("m", 10), 2.0, 12.5,
        kw.get("a0", -3.0), kw.get("dt", 0), kw.get("ck", 0), kw.get("dX", FAKE * 2000), 16,
        kw.get("dH", FAKE * 3000000), None, FAKE * 100000000, kw.get("wb", big), None)
    assert L.STATUS[bw(m=0)] == "TTDFT_ERR_DEGREE"
    assert L.STATUS[bw(a0=5.0)] == "TTDFT_ERR_BOUNDS"
    assert L.STATUS[bw(ck=-1)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[bw(dX=FAKE + 8)] == "TTDFT_ERR_ALIAS"
    assert L.STATUS[bw(dt=1)] == "TTDFT_ERR_DTYPE"
    assert L.STATUS[bw(wb=16)] == "TTDFT_ERR_WORKSPACE"
    assert L.STATUS[bw(dH=None)] == "TTDFT_ERR_NULL"


def test_backward_workspace_plan(lib_built):
    L = _lib()
    lib = L.load()
    H = _fake_bsr(nbr=10)
    blk = 10 * 64 * 32 * 8
    ws = lambda m, s: lib.ttdft_cheb_filter_backward_workspace(C.byref(H), 32, m, s, 0)
    assert ws(16, 0) == blk * 16                     # reverse buffer + Y_1..Y_15
    assert ws(16, 1) == ws(16, 2) == ws(16, 0)
    assert ws(16, 4) == blk * (1 + 7 + 2)            # pairs {1,4,5,8,9,12,13} + 2 segment slots
    assert ws(1, 4) == blk                           # nothing to store
    assert ws(16, 4) < ws(16, 0)


def test_lanczos_bounds_and_residuals_validation(lib_built):
    L = _lib()
    lib = L.load()
    H64, H32 = _fake_bsr(), _fake_bsr(dtype=1)
    out = (C.c_double * 4)()
    lb = lambda H=H64, perm=FAKE, k=10, o=out, wb=1 << 30: lib.ttdft_lanczos_bounds(C.byref(H), perm, k, 0, o, FAKE, wb, None)
    assert L.STATUS[lb(H=H32)] == "TTDFT_ERR_DTYPE"
    assert L.STATUS[lb(k=0)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[lb(perm=None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[lb(o=None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[lb(wb=8)] == "TTDFT_ERR_WORKSPACE"
    n = 32
    need = lib.ttdft_ritz_residuals_workspace(C.byref(H64), n)
    rows = H64.n_block_rows * 64
    assert need >= rows * n * 8
    W = FAKE + (1 << 36)            # fake addresses far apart: no overlap unless asked for
    psi, lam, res = FAKE, FAKE + (1 << 34), FAKE + (1 << 35)
    rr = lambda H=H64, p=psi, ld=n, l=lam, nv=n, r=res, w=W, wb=need: lib.ttdft_ritz_residuals(
        C.byref(H), p, ld, l, nv, r, w, wb, None)
    assert L.STATUS[rr(H=H32)] == "TTDFT_ERR_DTYPE"
    assert L.STATUS[rr(p=None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[rr(r=None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[rr(ld=n - 1)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[rr(nv=0)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[rr(wb=need - 8)] == "TTDFT_ERR_WORKSPACE"
    assert L.STATUS[rr(r=psi + 8)] == "TTDFT_ERR_ALIAS"
    assert L.STATUS[rr(w=psi)] == "TTDFT_ERR_ALIAS"


def test_density_entry_points_validation(lib_built):
    L = _lib()
    lib = L.load()
    H64, H32 = _fake_bsr(), _fake_bsr(dtype=1)
    mu = C.c_double()
    lam, f, w = FAKE, FAKE + (1 << 30), FAKE + (1 << 31)
    fl = lambda l=lam, n=16, ne=10.0, kT=0.01, ff=f, ww=w, wb=16: lib.ttdft_fermi_level(
        l, n, ne, kT, ff, C.byref(mu), ww, wb, None)
    assert lib.ttdft_fermi_level_workspace() == 16
    assert L.STATUS[fl(l=None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[fl(n=0)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[fl(kT=0.0)] == "TTDFT_ERR_BOUNDS"
    assert L.STATUS[fl(kT=float("inf"))] == "TTDFT_ERR_BOUNDS"
    assert L.STATUS[fl(ne=0.0)] == "TTDFT_ERR_BOUNDS"
    assert L.STATUS[fl(ne=32.0)] == "TTDFT_ERR_BOUNDS"          # = 2n: no finite mu
    assert L.STATUS[fl(wb=8)] == "TTDFT_ERR_WORKSPACE"
    assert L.STATUS[fl(ff=lam + 8)] == "TTDFT_ERR_ALIAS"
    psi, P_out = FAKE + (1 << 36), FAKE + (1 << 40)
    dm = lambda H=H64, p=psi, ld=32, ff=f, n=32, out=P_out: lib.ttdft_density_matrix(
        C.byref(H), p, ld, ff, n, out, None, None)
    assert L.STATUS[dm(H=H32)] == "TTDFT_ERR_DTYPE"
    assert L.STATUS[dm(p=None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[dm(out=None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[dm(ld=31)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[dm(out=psi + 64)] == "TTDFT_ERR_ALIAS"
    ed = lambda p=psi, ld=32, ff=f, rows=512, n=32, rho=P_out: lib.ttdft_electron_density(
        p, ld, ff, rows, n, rho, None)
    assert L.STATUS[ed(p=None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[ed(rows=0)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[ed(ld=16)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[ed(rho=psi + 8)] == "TTDFT_ERR_ALIAS"


def test_bsr_builder_bf16_split(lib_built):
    # hi = bf16(fp32(h)), lo = bf16(fp32(h) - hi), hi block then lo block per tile
    import torch
    (ip, ix, d, N), (nbr, nt, tptr, tcol, v64, perm, slot, mask, fmask) = _bsr_host(5, 2, 0)
    L = _lib()
    lib = L.load()
    P = lambda a: C.c_void_p(a.ctypes.data)
    vs = np.empty(nt * 8192, np.uint16)
    slot3 = np.empty(len(d), np.int64)
    tptr3, tcol3, perm3 = np.empty_like(tptr), np.empty_like(tcol), np.empty_like(perm)
    assert lib.ttdft_bsr_build(5, P(ip), P(ix), P(d), 3, P(tptr3), P(tcol3), P(vs), P(perm3), P(slot3),
                               None, None) == 0
    assert np.array_equal(tptr3, tptr) and np.array_equal(tcol3, tcol) and np.array_equal(perm3, perm)
    from paper_2110_15853_amd.api import _slots_16x32     # hi values in the BF16 fragment order
    np.testing.assert_array_equal(slot3, _slots_16x32(slot, 8192))
    bf = lambda u: torch.from_numpy(u.view(np.int16)).view(torch.bfloat16).float().numpy().astype(np.float64)
    hi, lo = bf(vs[slot3]), bf(vs[slot3 + 4096])
    h32 = d.astype(np.float32)
    ref_hi = torch.from_numpy(h32).to(torch.bfloat16).float().numpy()
    ref_lo = torch.from_numpy(h32 - ref_hi).to(torch.bfloat16).float().numpy()
    np.testing.assert_array_equal(hi, ref_hi)
    np.testing.assert_array_equal(lo, ref_lo)
    assert np.abs(hi + lo - d).max() <= 2.0 ** -16 * np.abs(d).max()
    # every other stored value is zero
    rest = np.ones(vs.size, bool)
    rest[slot3] = rest[slot3 + 4096] = False
    assert not vs[rest].any()


def test_split_and_step_validation(lib_built):
    L = _lib()
    lib = L.load()
    assert L.STATUS[lib.ttdft_split_bf16(None, 4, FAKE, None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[lib.ttdft_split_bf16(FAKE, -1, FAKE * 1000, None)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[lib.ttdft_split_bf16(FAKE, 4, FAKE + 64, None)] == "TTDFT_ERR_ALIAS"
    # split tiles step only FP32 iterates
    H = _fake_bsr(dtype=3)
    assert L.STATUS[_filter(H=H, dt=2)] == "TTDFT_ERR_DTYPE"
    assert L.STATUS[_filter(H=H, dt=0)] == "TTDFT_ERR_DTYPE"


def _np(a):
    return C.c_void_p(a.ctypes.data)


def test_bsr_build_size_matches_plan(lib_built):
    L = _lib()
    lib = L.load()
    ip, ix, d, N = workload.lattice_hamiltonian(6, 2, 0)
    ip = np.ascontiguousarray(ip, np.int64)
    ix = np.ascontiguousarray(ix, np.int32)
    nbr, nt, nt2 = C.c_int64(), C.c_int64(), C.c_int64()
    assert lib.ttdft_bsr_plan(6, _np(ip), _np(ix), C.byref(nbr), C.byref(nt)) == 0
    assert lib.ttdft_bsr_build_size(6, 4, _np(ip), _np(ix), C.byref(nt2)) == 0
    assert nt2.value == nt.value and nbr.value == 8
    assert L.STATUS[lib.ttdft_bsr_build_size(6, 3, _np(ip), _np(ix), C.byref(nt2))] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[lib.ttdft_bsr_build_size(6, 4, _np(ip), _np(ix), None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[lib.ttdft_bsr_build_size(6, 4, None, _np(ix), C.byref(nt2))] == "TTDFT_ERR_NULL"


def test_leading_dimension_limit_for_panel_offsets(lib_built):
    # the step kernel addresses a 64-row panel with 32-bit byte offsets:
    # 64 * ld * element size must stay below 2^31
    L = _lib()
    lib = L.load()
    big64, big32 = 1 << 22, 1 << 23
    assert L.STATUS[_filter(ldx=big64)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[_filter(ldy=big64)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[_filter(H=_fake_bsr(dtype=1), dt=1, ldx=big32)] == "TTDFT_ERR_SHAPE"
    H = _fake_bsr()
    assert L.STATUS[lib.ttdft_cheb_step(C.byref(H), FAKE, big64, None, 0, FAKE * 1000, 16, 16, 1.0,
                                        0.0, 0.0, 0, None)] == "TTDFT_ERR_SHAPE"
    need = lib.ttdft_cheb_filter_backward_workspace(C.byref(H), 16, 4, 0, 0)
    assert L.STATUS[lib.ttdft_cheb_filter_backward(
        C.byref(H), FAKE, 16, FAKE * 1000, 16, 16, 4, 2.0, 12.5, -3.0, 0, 0, FAKE * 2000, big64,
        FAKE * 3000, None, FAKE * 100000, need, None)] == "TTDFT_ERR_SHAPE"
    W = FAKE + (1 << 36)
    rneed = lib.ttdft_ritz_residuals_workspace(C.byref(H), 16)
    assert L.STATUS[lib.ttdft_ritz_residuals(C.byref(H), FAKE, big64, FAKE + (1 << 34), 16,
                                             FAKE + (1 << 35), W, rneed, None)] == "TTDFT_ERR_SHAPE"
    pneed = lib.ttdft_project_workspace(C.byref(H), 16)
    assert L.STATUS[lib.ttdft_project(C.byref(H), FAKE, big64, 16, FAKE + (1 << 34), 16, W, pneed,
                                      None)] == "TTDFT_ERR_SHAPE"


def test_next_bounds_validation(lib_built):
    L = _lib()
    lib = L.load()
    out = (C.c_double * 3)()
    assert L.STATUS[lib.ttdft_next_bounds(None, 8, 12.5, out, None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[lib.ttdft_next_bounds(FAKE, 8, 12.5, None, None)] == "TTDFT_ERR_NULL"
    assert L.STATUS[lib.ttdft_next_bounds(FAKE, 1, 12.5, out, None)] == "TTDFT_ERR_SHAPE"
    assert L.STATUS[lib.ttdft_next_bounds(FAKE, 8, float("inf"), out, None)] == "TTDFT_ERR_BOUNDS"


def _pass(**kw):
    L = _lib()
    lib = L.load()
    Hf, H64 = kw.pop("Hf", _fake_bsr()), kw.pop("H64", _fake_bsr())
    n = kw.pop("n", 16)
    args = dict(X=FAKE, ldx=n, dt=0, m=8, bounds=(-3.0, 2.0, 12.5), n_conv=n,
                lam=FAKE + (1 << 34), psi=FAKE + (1 << 35), ldpsi=n, res=FAKE + (1 << 33),
                nxt=(C.c_double * 3)(), work=FAKE + (1 << 36), wb=None)
    args.update(kw)
    if args["wb"] is None:
        args["wb"] = lib.ttdft_chfsi_pass_workspace(C.byref(Hf), C.byref(H64), n, args["dt"]) \
            if Hf is not None else 1 << 40
    b = (C.c_double * 3)(*args["bounds"]) if args["bounds"] is not None else None
    return L.STATUS[lib.ttdft_chfsi_pass(
        C.byref(Hf) if Hf is not None else None, C.byref(H64), args["X"], args["ldx"], args["dt"], n,
        args["m"], b, args["n_conv"], args["lam"], args["psi"], args["ldpsi"], args["res"], None,
        args["nxt"], args["work"], args["wb"], None)]


def test_chfsi_pass_validation(lib_built):
    L = _lib()
    assert _pass(Hf=None) == "TTDFT_ERR_NULL"
    assert _pass(H64=_fake_bsr(dtype=1)) == "TTDFT_ERR_DTYPE"         # Rayleigh-Ritz needs FP64
    assert _pass(dt=2) == "TTDFT_ERR_DTYPE"                           # iterates F64 or F32
    assert _pass(Hf=_fake_bsr(nbr=9)) == "TTDFT_ERR_SHAPE"            # not the same matrix
    assert _pass(m=0) == "TTDFT_ERR_DEGREE"
    assert _pass(bounds=(2.0, -3.0, 12.5)) == "TTDFT_ERR_BOUNDS"
    assert _pass(bounds=None) == "TTDFT_ERR_NULL"
    assert _pass(n_conv=0) == "TTDFT_ERR_SHAPE"
    assert _pass(n_conv=17) == "TTDFT_ERR_SHAPE"
    assert _pass(ldx=15) == "TTDFT_ERR_SHAPE"
    assert _pass(nxt=None) == "TTDFT_ERR_NULL"
    assert _pass(wb=1024) == "TTDFT_ERR_WORKSPACE"
    lib = L.load()
    H = _fake_bsr()
    w64 = lib.ttdft_chfsi_pass_workspace(C.byref(H), C.byref(H), 16, 0)
    w32 = lib.ttdft_chfsi_pass_workspace(C.byref(_fake_bsr(dtype=1)), C.byref(H), 16, 1)
    assert w64 >= 8 * 64 * 16 * 8 and 0 < w32
    assert lib.ttdft_chfsi_pass_workspace(C.byref(H), C.byref(H), 16, 2) == 0


def _solve(**kw):
    L = _lib()
    lib = L.load()
    Hf, H64 = kw.pop("Hf", _fake_bsr()), kw.pop("H64", _fake_bsr())
    n = 16
    args = dict(perm=FAKE, X=FAKE, ldx=n, dt=0, m=8, m_first=0, tol=1e-8, n_conv=n, max_passes=5,
                bounds=None, k=20, lam=FAKE + (1 << 34), psi=FAKE + (1 << 35), ldpsi=n,
                res=FAKE + (1 << 33), cap=0, nrec=C.c_int32(0), work=FAKE + (1 << 36), wb=None)
    args.update(kw)
    if args["wb"] is None:
        args["wb"] = lib.ttdft_chfsi_solve_workspace(C.byref(Hf), C.byref(H64), n, args["dt"],
                                                     0 if args["bounds"] else args["k"])
    b = (C.c_double * 3)(*args["bounds"]) if args["bounds"] is not None else None
    nrec = C.byref(args["nrec"]) if args["nrec"] is not None else None
    return L.STATUS[lib.ttdft_chfsi_solve(
        C.byref(Hf), C.byref(H64), args["perm"], args["X"], args["ldx"], args["dt"], n, args["m"],
        args["m_first"], args["tol"], args["n_conv"], args["max_passes"], b, args["k"], 0,
        args["lam"], args["psi"], args["ldpsi"], args["res"], None, args["cap"], nrec,
        args["work"], args["wb"], None)]


def test_chfsi_solve_validation(lib_built):
    assert _solve(H64=_fake_bsr(dtype=2)) == "TTDFT_ERR_DTYPE"
    assert _solve(perm=None) == "TTDFT_ERR_NULL"                      # Lanczos bounds need perm
    assert _solve(nrec=None) == "TTDFT_ERR_NULL"
    assert _solve(cap=4) == "TTDFT_ERR_NULL"                          # history NULL with a capacity
    assert _solve(m=0) == "TTDFT_ERR_DEGREE"
    assert _solve(m_first=-1) == "TTDFT_ERR_DEGREE"
    assert _solve(max_passes=0) == "TTDFT_ERR_SHAPE"
    assert _solve(k=0) == "TTDFT_ERR_SHAPE"
    assert _solve(tol=-1.0) == "TTDFT_ERR_BOUNDS"
    assert _solve(tol=float("nan")) == "TTDFT_ERR_BOUNDS"
    assert _solve(bounds=(1.0, 1.0, 12.5)) == "TTDFT_ERR_BOUNDS"
    assert _solve(wb=4096) == "TTDFT_ERR_WORKSPACE"
    assert _solve(psi=FAKE) == "TTDFT_ERR_ALIAS"                      # Psi overlaps X
    lib = _lib().load()
    H = _fake_bsr()
    w0 = lib.ttdft_chfsi_solve_workspace(C.byref(H), C.byref(H), 16, 0, 0)
    w32 = lib.ttdft_chfsi_solve_workspace(C.byref(_fake_bsr(dtype=1)), C.byref(H), 16, 1, 0)
    assert w0 == lib.ttdft_chfsi_pass_workspace(C.byref(H), C.byref(H), 16, 0)
    assert w32 > lib.ttdft_chfsi_pass_workspace(C.byref(_fake_bsr(dtype=1)), C.byref(H), 16, 1)


def test_check_finite_validation(lib_built):
    L = _lib()
    lib = L.load()
    cnt = C.c_int64(-1)
    cf = lambda A=FAKE, dt=0, rows=4, cols=4, ld=4, c=C.byref(cnt), w=FAKE * 100, wb=16: \
        L.STATUS[lib.ttdft_check_finite(A, dt, rows, cols, ld, c, w, wb, None)]
    assert lib.ttdft_check_finite_workspace() == 16
    assert cf(dt=3) == "TTDFT_ERR_DTYPE"
    assert cf(c=None) == "TTDFT_ERR_NULL"
    assert cf(A=None) == "TTDFT_ERR_NULL"
    assert cf(ld=3) == "TTDFT_ERR_SHAPE"
    assert cf(rows=-1) == "TTDFT_ERR_SHAPE"
    assert cf(wb=8) == "TTDFT_ERR_WORKSPACE"
    assert cf(w=FAKE + 8) == "TTDFT_ERR_ALIAS"
    assert cf(rows=0) == "TTDFT_OK" and cnt.value == 0                # empty block: no device work
