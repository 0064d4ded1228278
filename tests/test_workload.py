"""The seeded generator: structure, symmetry, counts, determinism. CPU only."""
import numpy as np
import pytest

import workload


def nnz_closed_form(r, h):
    # per axis, pairs (i, i+d) inside [0, r) number r - |d|
    per_axis = r + 2 * sum(max(r - d, 0) for d in range(1, h + 1))
    return per_axis ** 3


@pytest.mark.parametrize("r,h", [(3, 1), (4, 3), (5, 2), (20, 3), (10, 3), (7, 4)])
def test_nnz_and_symmetry(r, h):
    ip, ix, d, N = workload.lattice_hamiltonian(r, h, 0)
    assert N == r ** 3 and len(d) == nnz_closed_form(r, h) and ip[-1] == len(d)
    import scipy.sparse as sp
    H = sp.csr_matrix((d, ix, ip), shape=(N, N))
    assert (H - H.T).count_nonzero() == 0
    for row in range(N):                      # columns ascending within rows
        assert np.all(np.diff(ix[ip[row]:ip[row + 1]]) > 0)


def test_config1_nnz_pin():
    ip, ix, d, N = workload.lattice_hamiltonian(20, 3, 0)
    assert len(d) == 2_097_152


def test_brute_force_pattern_and_values_small():
    r, h = 4, 2
    ip, ix, d, N = workload.lattice_hamiltonian(r, h, 3)
    dense = np.zeros((N, N))
    for row in range(N):
        dense[row, ix[ip[row]:ip[row + 1]]] = d[ip[row]:ip[row + 1]]
    ratios = []
    for I in range(N):
        i, j, k = I // (r * r), (I // r) % r, I % r
        for J in range(N):
            p, q, s = J // (r * r), (J // r) % r, J % r
            near = max(abs(p - i), abs(q - j), abs(s - k)) <= h
            if I == J:
                assert -2.0 <= dense[I, J] < 10.0
            elif near:
                dist = np.sqrt((p - i) ** 2 + (q - j) ** 2 + (s - k) ** 2)
                ratios.append(dense[I, J] / (-0.5 * np.exp(-0.8 * dist)))
            else:
                assert dense[I, J] == 0.0
    ratios = np.array(ratios)          # = 1 + 0.1 z, z ~ N(0, 1)
    assert abs(ratios.mean() - 1.0) < 0.01 and abs(ratios.std() - 0.1) < 0.01


def test_determinism_and_streams():
    a = workload.lattice_hamiltonian(5, 2, 7)
    b = workload.lattice_hamiltonian(5, 2, 7)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)
    X = workload.gaussian_block(100, 4, 7)
    np.testing.assert_array_equal(X, workload.gaussian_block(100, 4, 7))
    assert not np.array_equal(X, workload.gaussian_block(100, 4, 7, stream="W"))


def test_positive_offsets():
    P = workload.positive_offsets(2)
    assert len(P) == (5 ** 3 - 1) // 2
    full = {tuple(p) for p in P} | {tuple(-p) for p in P}
    assert len(full) == 5 ** 3 - 1
    assert [tuple(p) for p in P] == sorted(tuple(p) for p in P)
