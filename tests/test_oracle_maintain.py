"""Pins of the map-maintenance oracle: the pruning selection against the properties that define
it (budget, ordering, frozen rows, the two extreme ratios) and the proximity filter against
scipy's k-d tree and hand-placed points."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import maintain_oracle as mo


@pytest.mark.parametrize("ratio", [0.0, 0.01, 0.05, 0.2, 1.0])
def test_prune_selection_properties(ratio):
    rng = np.random.default_rng(int(ratio * 100))
    n = 5000
    lg = rng.normal(0, 2, n).astype(np.float32)
    lg[::97] = -4.0  # ties at the threshold side
    seg = rng.integers(0, 6, n)
    thr = -1.5
    keep, rem = mo.prune_select(lg, thr, ratio, seg, 3)
    cand = (lg < np.float32(thr)) & (seg >= 3)
    k = int(np.floor(np.float64(np.float32(ratio)) * n))
    assert rem.sum() == min(cand.sum(), k)
    assert not np.any(rem & ~cand)                       # only candidates, never frozen rows
    assert np.array_equal(keep, np.nonzero(~rem)[0])     # survivors in row order
    if rem.any() and (cand & ~rem).any():
        assert lg[rem].max() <= lg[cand & ~rem].min()    # the smallest logits go first
        tie = lg[rem].max()
        # at the cut, equal logits are taken in ascending row order
        r_t = np.nonzero(rem & (lg == tie))[0]
        k_t = np.nonzero(cand & ~rem & (lg == tie))[0]
        if r_t.size and k_t.size:
            assert r_t.max() < k_t.min()
    if ratio == 1.0:
        assert np.array_equal(rem, cand)
    if ratio == 0.0:
        assert not rem.any()


def test_prune_without_segments_and_gather():
    lg = np.array([0.5, -3.0, -2.0, -3.0, 1.0, -5.0], np.float32)
    keep, rem = mo.prune_select(lg, -1.0, 0.5)  # k = 3: rows 5, 1, 3 (two -3.0 in row order)
    assert rem.tolist() == [False, True, False, True, False, True]
    keep, rem = mo.prune_select(lg, -1.0, 0.34)  # k = 2: rows 5 then 1
    assert keep.tolist() == [0, 2, 3, 4]
    A = np.arange(12).reshape(2, 6)
    assert mo.gather_rows(A, keep).tolist() == [[0, 2, 3, 4], [6, 8, 9, 10]]


def test_redundant_matches_kdtree_and_hand_cases():
    rng = np.random.default_rng(3)
    A = rng.uniform(-2, 2, (3, 4000)).astype(np.float32)
    B = np.concatenate([A[:, :500] + rng.normal(0, 0.03, (3, 500)), rng.uniform(-2, 2, (3, 1500))],
                       axis=1).astype(np.float32)
    d = 0.05
    got = mo.redundant(A, B, d)
    dist, _ = cKDTree(A.T.astype(np.float64)).query(B.T.astype(np.float64))
    clear = np.abs(dist - np.float64(np.float32(d))) > 1e-9
    assert np.array_equal(got[clear], (dist < np.float64(np.float32(d)))[clear])
    assert 100 < got.sum() < 1000
    # strict: exactly d_min apart is not redundant
    a = np.zeros((3, 1), np.float32)
    b = np.array([[0.25], [0.0], [0.0]], np.float32)
    assert not mo.redundant(a, b, 0.25)[0]
    assert mo.redundant(a, b, np.nextafter(np.float32(0.25), np.float32(1)))[0]
    assert not mo.redundant(np.zeros((3, 0), np.float32), b, 1.0).any()


def _interleave_by_string(x, y, z):
    # bit string of the Morton code, most significant first: z9 y9 x9 z8 y8 x8 ... z0 y0 x0
    bits = "".join(f"{c:010b}"[9 - b] for b in range(9, -1, -1) for c in (z, y, x))
    return int(bits, 2)


def test_morton_code_matches_bitstring_interleave():
    rng = np.random.default_rng(3)
    q = rng.integers(0, 1024, (3, 500))
    q[:, 0] = 0
    q[:, 1] = 1023
    codes = mo.morton_code(q)
    for k in range(q.shape[1]):
        assert codes[k] == _interleave_by_string(*q[:, k])


def test_row_order_hand_cases():
    # the 8 corners of a box: x varies fastest, then y, then z
    corners = np.array([[x, y, z] for z in (0.0, 2.0) for y in (0.0, 3.0) for x in (-1.0, 5.0)], np.float32).T
    perm = np.array([6, 1, 7, 0, 3, 5, 2, 4])
    order = mo.row_order(corners[:, perm])
    assert np.array_equal(perm[order], np.arange(8))
    cells = mo.morton_cells(corners)
    assert set(cells.ravel().tolist()) == {0, 1023}  # the maximum is clamped into the last cell
    # segments first, then space; equal points keep row order; a flat axis gives cell 0
    m = np.array([[0, 1, 0, 1, 0], [0, 0, 0, 0, 0], [5, 5, 5, 5, 5]], np.float32)
    seg = np.array([2, 1, 1, 2, -3])
    assert mo.row_order(m, seg).tolist() == [4, 2, 1, 0, 3]
    assert mo.morton_cells(m)[2].tolist() == [0] * 5


def test_row_order_is_a_locality_preserving_permutation():
    rng = np.random.default_rng(4)
    m = rng.uniform(-50, 50, (3, 20000)).astype(np.float32)
    seg = rng.integers(0, 4, 20000)
    order = mo.row_order(m, seg)
    assert np.array_equal(np.sort(order), np.arange(20000))
    assert np.all(np.diff(seg[order]) >= 0)
    step = np.linalg.norm(np.diff(m[:, order], axis=1), axis=0)
    rand = np.linalg.norm(m[:, :-1] - m[:, 1:], axis=0)
    assert np.median(step) < 0.1 * np.median(rand)
