"""Pins of the oracle's smoothed-aggregation AMG against invariants, closed
forms, brute force and library routines."""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen as mg
from oracle import amg, fem, krylov
from oracle.rng import splitmix64, uniform01, uniform01_vec
from tests.conftest import read_golden


def test_splitmix64_published_vectors():
    for seed, k, val in read_golden("splitmix64.txt"):
        x = (int(seed) + int(k) * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
        assert splitmix64(x) == int(val, 0)
    a = uniform01(0x5EED + 2, 257)
    assert np.array_equal(a, uniform01_vec(0x5EED + 2, 257))
    assert 0 <= a.min() and a.max() < 1


def _cube_system(n=4, deg=1, clamp=True):
    prob = mg.cube_problem(n, deg)
    if clamp:
        A, b, _, _ = fem.assemble_problem(prob)
        B = fem.rigid_body_modes(prob.mesh.coords, prob.mask)
    else:
        A, b0 = fem.assemble(prob.mesh.coords, prob.mesh.cells, deg, prob.E, prob.nu, prob.alpha,
                             prob.T_ref, prob.T)
        b = b0.reshape(-1)
        B = fem.rigid_body_modes(prob.mesh.coords)
    return prob, A, b, B


# ---------------------------------------------------------------------------
# Strength and aggregation
# ---------------------------------------------------------------------------

def _brute_aggregate(n, strong_sets, s):
    """Direct restatement of the two greedy phases on a tiny graph."""
    agg = [-1] * n
    na = 0
    for i in range(n):
        nb = strong_sets[i]
        if nb and agg[i] < 0 and all(agg[j] < 0 for j in nb):
            for j in [i] + sorted(nb):
                agg[j] = na
            na += 1
    snap = list(agg)
    for i in range(n):
        if not strong_sets[i] or snap[i] >= 0:
            continue
        cands = [(s[(i, j)], snap[j], j) for j in sorted(strong_sets[i]) if snap[j] >= 0]
        best = max(cands, key=lambda t: (t[0], -t[1]))
        agg[i] = best[1]
    return np.array(agg), na


def test_aggregation_brute_force_random_graphs():
    rng = np.random.default_rng(7)
    for trial in range(20):
        n = 12
        Ad = np.zeros((n, n))
        for _ in range(20):
            i, j = rng.integers(0, n, 2)
            if i != j:
                Ad[i, j] = Ad[j, i] = rng.uniform(0.01, 1.0)
        Ad += np.diag(Ad.sum(1) + 1.0)
        # 1x1 "blocks": a BSR with blocksize 1
        A = sp.bsr_matrix(sp.csr_matrix(Ad), blocksize=(1, 1))
        theta = 0.15
        rows, cols, s = amg.strength(A)
        sd = {(int(r), int(c)): v for r, c, v in zip(rows, cols, s)}
        strong_sets = [set() for _ in range(n)]
        for (r, c), v in sd.items():
            if r != c and v >= theta:
                strong_sets[r].add(c)
        agg, na, _ = amg.aggregate(A, theta)
        ref, nref = _brute_aggregate(n, strong_sets, sd)
        assert na == nref
        assert np.array_equal(agg, ref)


def test_phase2_tie_rule_hand_worked():
    """Phase 2's choice among aggregated strong neighbours (the reading of the
    aggregation step of Sec. 5.1: strongest neighbour wins; strengths within
    a relative 1e-9 are equal and the smaller aggregate id wins), worked by
    hand on one free node per case.  Catches a larger-id winner, a missing or
    an oversized tolerance and an unaggregated neighbour being taken."""
    s = 0.5
    cases = [
        # (neighbour aggregate ids, strengths, expected aggregate)
        ([5, 3], [s, s], 3),                                  # exact tie: smaller id
        ([3, 5], [s, s], 3),                                  # same, other visiting order
        ([4, 2], [s, s * (1.0 - 5e-10)], 2),                  # within 1e-9: a tie
        ([2, 4], [s * (1.0 - 5e-10), s], 2),
        ([4, 2], [s, s * (1.0 - 1e-8)], 4),                   # 1e-8 apart: strongest wins
        ([2, 4], [s * (1.0 - 1e-8), s], 4),
        ([7, -1, 6], [0.3, 0.9, 0.2], 7),                     # unaggregated neighbour ignored
        ([1, 0, 2], [0.2, 0.2 * (1 + 2e-10), 0.25], 2),
    ]
    nodes = []
    agg0 = []
    nbrs = []
    nid = 0
    for ids, sv, _ in cases:
        free = nid
        agg0.append(-1)
        nbrs_free = []
        nid += 1
        for a in ids:
            agg0.append(a)        # a neighbour node carrying aggregate a (or -1)
            nbrs_free.append(nid)
            nid += 1
        nodes.append((free, nbrs_free, sv))
    n = nid
    lists = [(np.zeros(0, np.int64), np.zeros(0)) for _ in range(n)]
    for free, nb, sv in nodes:
        lists[free] = (np.array(nb, np.int64), np.array(sv, float))
    # an unaggregated neighbour (-1) is itself a free node of phase 2: give it
    # one aggregated strong neighbour (the first of its case)
    agg0 = np.array(agg0, np.int64)
    for free, nb, sv in nodes:
        for j in nb:
            if agg0[j] < 0:
                lists[j] = (np.array([nb[0]], np.int64), np.array([0.9]))
    out = amg._attach_rest(agg0, lists)
    for (free, _, _), (_, _, want) in zip(nodes, cases):
        assert out[free] == want, (free, out[free], want)



@pytest.mark.parametrize("deg,n", [(1, 6), (2, 3)])
def test_aggregation_invariants(deg, n):
    prob, A, b, B = _cube_system(n, deg)
    agg, na, (rows, cols, s) = amg.aggregate(A, 0.08)
    N = prob.mesh.n_nodes
    strong = (s >= 0.08) & (rows != cols)
    has_strong = np.bincount(rows[strong], minlength=N) > 0
    # isolated nodes (here: the clamped face) are exactly the unaggregated ones
    assert np.array_equal(agg < 0, ~has_strong)
    assert np.all(prob.mask[~has_strong].all(axis=1))
    # ids are 0..na-1, every aggregate non-empty
    assert set(agg[agg >= 0].tolist()) == set(range(na))
    # strength is symmetric up to rounding
    S = sp.csr_matrix((s, (rows, cols)), shape=(N, N))
    assert abs(S - S.T).max() <= 1e-14


def test_tentative_prolongator_properties():
    prob, A, b, B = _cube_system(5, 1)
    agg, na, sinfo = amg.aggregate(A, 0.08)
    P, Bc, agg2 = amg.tentative_prolongator(agg, na, B, 3, sinfo)
    # orthonormal columns per aggregate, P_tent Bc = B
    PtP = (P.T @ P).toarray()
    assert np.abs(PtP - np.eye(PtP.shape[0])).max() < 1e-13
    assert np.abs(P @ Bc - B).max() < 1e-13 * np.abs(B).max()
    # R blocks upper triangular with positive diagonal
    R = Bc.reshape(-1, 6, 6)
    assert np.all(np.tril(R, -1) == 0)
    assert np.all(np.einsum("kii->ki", R) > 0)
    # QR agrees with numpy's after the sign fix, aggregate 0
    nodes = np.nonzero(agg2 == 0)[0]
    Q, Rn = np.linalg.qr(B.reshape(-1, 3, 6)[nodes].reshape(-1, 6))
    sg = np.sign(np.diag(Rn))
    assert np.abs(Rn * sg[:, None] - R[0]).max() < 1e-13 * np.abs(R[0]).max()


def test_rank_deficient_aggregate_is_merged():
    # aggregates made of a single P1 node (3 rows < 6) must be merged
    prob, A, b, B = _cube_system(3, 1)
    agg, na, sinfo = amg.aggregate(A, 0.08)
    forced = agg.copy()
    lone = int(np.nonzero(agg >= 0)[0][-1])
    forced[lone] = na  # a new one-node aggregate
    P, Bc, agg2 = amg.tentative_prolongator(forced, na + 1, B, 3, sinfo)
    assert agg2.max() + 1 == na
    assert np.abs(P @ Bc - B).max() < 1e-13 * np.abs(B).max()


def test_smoothed_prolongator_and_galerkin_preserve_nullspace():
    # on the unconstrained operator A B = 0, hence P B_c = B and A_c B_c = 0
    prob, A, b, B = _cube_system(4, 1, clamp=False)
    D = amg.point_diagonal(A)
    lam = amg.lanczos_max(A, D, 20, 0x5EED)
    agg, na, sinfo = amg.aggregate(A, 0.08)
    Pt, Bc, _ = amg.tentative_prolongator(agg, na, B, 3, sinfo)
    P = amg.smooth_prolongator(A, D, Pt, lam)
    assert np.abs(P @ Bc - B).max() <= 1e-10 * np.abs(B).max()
    Ac = amg.galerkin(A, P)
    Acd = Ac.toarray()
    assert np.abs(Acd - Acd.T).max() <= 1e-12 * np.abs(Acd).max()
    assert np.abs(Acd @ Bc).max() <= 1e-10 * np.abs(Acd).max() * np.abs(Bc).max()
    # and the Galerkin product equals the dense triple product
    Pd = P.toarray()
    assert np.abs(Acd - Pd.T @ A.toarray() @ Pd).max() <= 1e-12 * np.abs(Acd).max()


# ---------------------------------------------------------------------------
# Eigenvalue estimate, Chebyshev, V-cycle
# ---------------------------------------------------------------------------

def test_lanczos_estimate_brackets_dense_eigenvalue():
    for deg, n in [(1, 4), (2, 2)]:
        prob, A, b, B = _cube_system(n, deg)
        D = amg.point_diagonal(A)
        lam = amg.lanczos_max(A, D, 20, 0x5EED)
        Dh = 1 / np.sqrt(D)
        lmax = np.linalg.eigvalsh(Dh[:, None] * A.toarray() * Dh[None, :]).max()
        assert lam <= lmax * (1 + 1e-12)
        assert lam >= 0.9 * lmax


def test_lanczos_diagonal_known_spectrum():
    ev = np.linspace(1.0, 5.0, 400)
    A = sp.bsr_matrix(sp.diags(ev).tocsr(), blocksize=(1, 1))
    lam = amg.lanczos_max(A, np.ones(400), 20, 0x5EED)
    assert 0.95 * 5.0 <= lam <= 5.0 * (1 + 1e-12)
    # tiny dimension: Lanczos terminates early and is exact
    A = sp.bsr_matrix(sp.diags([1.0, 2.0, 7.0]).tocsr(), blocksize=(1, 1))
    assert abs(amg.lanczos_max(A, np.ones(3), 20, 0x5EED) - 7.0) < 1e-12


def _cheb_poly_factor(lmb, lam_hat, m=2):
    """Closed form: error factor T_m((theta - l)/delta) / T_m(sigma)."""
    b = 1.1 * lam_hat
    a = b / 10
    theta, delta = (a + b) / 2, (b - a) / 2
    T = np.polynomial.chebyshev.Chebyshev.basis(m)
    return T((theta - lmb) / delta) / T(theta / delta)


def test_chebyshev_error_propagation_closed_form():
    prob, A, b, B = _cube_system(3, 1)
    D = amg.point_diagonal(A)
    Ad = A.toarray()
    # eigenvectors of D^-1 A via the symmetric form
    Dh = 1 / np.sqrt(D)
    w, V = np.linalg.eigh(Dh[:, None] * Ad * Dh[None, :])
    lam_hat = 0.97 * w.max()
    for idx in [0, len(w) // 3, len(w) - 1]:
        e0 = Dh * V[:, idx]           # eigenvector of D^-1 A
        xs = np.random.default_rng(idx).normal(size=Ad.shape[0])
        g = Ad @ xs
        x = amg.chebyshev(A, D, g, xs - e0, lam_hat, 2)
        e1 = xs - x
        fac = _cheb_poly_factor(w[idx], lam_hat)
        assert np.abs(e1 - fac * e0).max() <= 1e-12 * np.abs(e0).max()


def test_vcycle_symmetric_positive_and_single_level_exact():
    prob, A, b, B = _cube_system(6, 1)
    lv = amg.setup(A, B, amg.AMGOptions(coarse_max=300))
    assert len(lv) >= 2
    rng = np.random.default_rng(0)
    x, y = rng.normal(size=(2, A.shape[0]))
    Mx, My = amg.vcycle(lv, x), amg.vcycle(lv, y)
    assert abs(x @ My - y @ Mx) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(My)
    assert x @ Mx > 0
    lv1 = amg.setup(A, B, amg.AMGOptions(coarse_max=10 ** 6))
    assert len(lv1) == 1
    assert np.abs(A @ amg.vcycle(lv1, b) - b).max() <= 1e-12 * np.abs(b).max()


def test_hierarchy_sizes_cube_config():
    prob, A, b, B = _cube_system(16, 1)
    lv = amg.setup(A, B)
    assert [lv_.bs for lv_ in lv] == [3, 6]
    assert lv[0].A.shape[0] == 14739 and lv[1].A.shape[0] <= 3000
