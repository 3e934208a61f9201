"""Pins of the oracle's parallel (MIS-2) aggregation.

* With fixed keys, the parallel rounds select exactly the roots that the
  sequential phase 1 selects when it visits the nodes in descending key order
  (Blelloch, Fineman & Shun, SPAA 2012): checked against that sequential
  greedy, written out here, on mesh strength graphs and random graphs.
* A 7-node path with keys equal to the node index, worked by hand.
* Distance-2 independence and maximality of the roots, through sparse
  boolean matrix powers (a different computation from the rounds).
* The aggregates partition the non-isolated nodes, each with one root whose
  strong neighbours are its phase-1 members.
* The hierarchy built on them preconditions CG to the same tolerance, in a
  comparable number of iterations."""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen as mg
from oracle import amg, fem, krylov


def _sequential_roots(n, rows, cols, flag, keys):
    """Phase 1 of the greedy aggregation, visiting nodes by descending key."""
    nb = [[] for _ in range(n)]
    for r, c in zip(rows[flag].tolist(), cols[flag].tolist()):
        nb[r].append(c)
    taken = np.zeros(n, bool)
    roots = np.zeros(n, bool)
    for i in np.argsort(-keys, kind="stable").tolist():
        if not nb[i] or taken[i] or any(taken[j] for j in nb[i]):
            continue
        roots[i] = True
        taken[i] = True
        taken[nb[i]] = True
    return roots


def _random_graph(n, deg, seed):
    rng = np.random.default_rng(seed)
    r = rng.integers(0, n, n * deg)
    c = rng.integers(0, n, n * deg)
    G = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(n, n)).tocsr()
    G = ((G + G.T + sp.identity(n)) > 0).astype(np.int8).tocsr()
    G.sort_indices()
    rows = np.repeat(np.arange(n), np.diff(G.indptr))
    cols = G.indices.astype(np.int64)
    return rows, cols, rows != cols


def _mesh_graph(prob, theta=0.08):
    A, _, _, _ = fem.assemble_problem(prob)
    n = A.shape[0] // 3
    flag, (rows, cols, s) = amg.symmetric_strong(A, theta)
    return A, n, rows, cols, flag


@pytest.mark.parametrize("case", ["disc_p1", "disc_p2", "cube_p1", "random"])
def test_rounds_equal_sequential_greedy_in_key_order(case):
    if case == "random":
        n = 3000
        rows, cols, flag = _random_graph(n, 3, 4)
    else:
        prob = {"disc_p1": lambda: mg.disc_problem(8, 34, 2, 1, seed=0),
                "disc_p2": lambda: mg.disc_problem(6, 26, 2, 2, seed=1),
                "cube_p1": lambda: mg.cube_problem(10, 1)}[case]()
        _, n, rows, cols, flag = _mesh_graph(prob)
    for seed in (amg.MIS_SEED, 12345):
        keys = amg.mis_keys(n, seed)
        roots, rounds = amg.mis2_rounds(n, rows, cols, flag, keys)
        assert np.array_equal(roots, _sequential_roots(n, rows, cols, flag, keys))
        assert rounds <= 40


def test_path_graph_worked_by_hand():
    """0-1-2-3-4-5-6 with key = index: 6 joins first (round 1), 4 and 5 are
    excluded (round 2), 3 joins (round 3), 1 and 2 are excluded (round 4), 0
    joins (round 5)."""
    n = 7
    rows = np.array([0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5, 6])
    cols = np.array([1, 0, 2, 1, 3, 2, 4, 3, 5, 4, 6, 5])
    flag = np.ones(rows.size, bool)
    roots, rounds = amg.mis2_rounds(n, rows, cols, flag, np.arange(n, dtype=np.int64))
    assert np.flatnonzero(roots).tolist() == [0, 3, 6] and rounds == 5
    # reversed keys: 0 first, then 3, then 6
    roots, _ = amg.mis2_rounds(n, rows, cols, flag, np.arange(n, 0, -1, dtype=np.int64))
    assert np.flatnonzero(roots).tolist() == [0, 3, 6]
    # keys favouring node 1: 1 joins, 0, 2, 3 excluded, then 4 (above 5, 6) joins
    keys = np.array([0, 9, 1, 2, 8, 7, 6], np.int64)
    roots, _ = amg.mis2_rounds(n, rows, cols, flag, keys)
    assert np.flatnonzero(roots).tolist() == [1, 4]


@pytest.mark.parametrize("case", ["disc_p2", "random"])
def test_roots_are_a_maximal_distance_2_independent_set(case):
    if case == "random":
        n = 4000
        rows, cols, flag = _random_graph(n, 2, 9)
    else:
        _, n, rows, cols, flag = _mesh_graph(mg.disc_problem(8, 34, 2, 2, seed=5))
    roots, _ = amg.mis2_rounds(n, rows, cols, flag, amg.mis_keys(n, amg.MIS_SEED))
    G = sp.csr_matrix((np.ones(int(flag.sum())), (rows[flag], cols[flag])), shape=(n, n))
    I = sp.identity(n, format="csr")
    within2 = ((I + G + G @ G) > 0).astype(np.int8)
    R = sp.diags(roots.astype(np.int8))
    # independence: no two roots within distance 2
    RR = (R @ within2 @ R).tocoo()
    assert np.all(RR.row == RR.col)
    # maximality: every node with a neighbour is within distance 2 of a root
    has = np.asarray(G.sum(axis=1)).ravel() > 0
    covered = np.asarray(within2 @ roots.astype(np.int64)).ravel() > 0
    assert np.all(covered[has]) and not np.any(roots[~has])


def test_aggregates_partition_with_one_root_each():
    prob = mg.disc_problem(8, 34, 2, 2, seed=5)
    A, n, rows, cols, flag = _mesh_graph(prob)
    agg, na, _ = amg.aggregate_mis2(A, 0.08, amg.MIS_SEED)
    roots, _ = amg.mis2_rounds(n, rows, cols, flag, amg.mis_keys(n, amg.MIS_SEED))
    has = np.bincount(rows[flag], minlength=n) > 0
    assert np.all(agg[has] >= 0) and np.all(agg[~has] == -1)
    assert na == roots.sum() and set(agg[has].tolist()) == set(range(na))
    # aggregate ids follow the roots in ascending node order
    assert np.array_equal(agg[roots], np.arange(na))
    # every strong neighbour of a root is in the root's aggregate
    sel = flag & roots[rows]
    assert np.array_equal(agg[cols[sel]], agg[rows[sel]])
    # every member is a root, a strong neighbour of its root, or a strong
    # neighbour of such a neighbour (phase 2)
    root_of = np.full(na, -1)
    root_of[agg[roots]] = np.flatnonzero(roots)
    G = sp.csr_matrix((np.ones(int(flag.sum())), (rows[flag], cols[flag])), shape=(n, n))
    within2 = ((sp.identity(n) + G + G @ G) > 0).tocsr()
    for i in np.flatnonzero(has)[::7].tolist():
        assert within2[i, root_of[agg[i]]]


def test_symmetric_strong_graph():
    """On a symmetric matrix the flags are the one-sided ones; an entry whose
    mirror alone passes the threshold is flagged both ways."""
    prob = mg.disc_problem(6, 26, 2, 1, seed=1)
    A, _, _, _ = fem.assemble_problem(prob)
    flag, (rows, cols, s) = amg.symmetric_strong(A, 0.08)
    own = (s >= 0.08) & (rows != cols)
    assert np.array_equal(flag, own)
    # scale one off-diagonal block (and not its mirror): s_IJ rises above theta
    A2 = A.copy()
    k = int(np.flatnonzero(~own & (rows != cols) & (s > 0))[0])
    A2.data[k] *= 0.2 / max(s[k], 1e-30)
    flag2, (_, _, s2) = amg.symmetric_strong(A2, 0.08)
    kt = int(np.flatnonzero((rows == cols[k]) & (cols == rows[k]))[0])
    assert s2[k] >= 0.08 and s2[kt] < 0.08 and flag2[k] and flag2[kt]


@pytest.mark.parametrize("deg,cm", [(1, 300), (2, 400)])
def test_amg_with_parallel_aggregation_converges(deg, cm):
    prob = mg.disc_problem(8, 34, 2, deg, seed=5)
    A, b, _, _ = fem.assemble_problem(prob)
    B = fem.rigid_body_modes(prob.mesh.coords, prob.mask)
    its = {}
    for mode in ("greedy", "mis2"):
        opt = amg.AMGOptions(coarse_max=cm, aggregation=mode)
        lv = amg.setup(A, B, opt)
        res = krylov.pcg(A, b, lambda r: amg.vcycle(lv, r, opt=opt))
        assert res.converged and np.linalg.norm(b - A @ res.u) <= 1e-8 * np.linalg.norm(b)
        its[mode] = res.iters
    assert its["mis2"] <= 1.3 * its["greedy"] + 2


def test_filtered_operator_keeps_strong_blocks_and_translations():
    """A^F (prolongator smoothing option): strong and diagonal blocks only,
    the dropped blocks lumped into the diagonal, so A^F t = A t for the three
    translations t; the smoothed prolongator gets fewer blocks and the
    hierarchy still preconditions CG to the tolerance."""
    prob = mg.disc_problem(8, 34, 2, 2, seed=5)
    A, b, _, _ = fem.assemble_problem(prob)
    n = A.shape[0] // 3
    Af = amg.filtered_operator(A, 0.08)
    flag, (rows, cols, s) = amg.symmetric_strong(A, 0.08)
    assert Af.nnz // 9 == int(flag.sum()) + n
    for q in range(3):
        t = np.zeros(3 * n)
        t[q::3] = 1.0
        assert np.abs(Af @ t - A @ t).max() <= 1e-12 * np.abs(A.data).max()
    # a rotation is not preserved in general (only the block row sums are)
    x = prob.mesh.coords
    rot = np.stack([-x[:, 1], x[:, 0], np.zeros(n)], axis=1).reshape(-1)
    assert np.abs(Af @ rot - A @ rot).max() > 1e-6 * np.abs(A @ rot).max()
    B = fem.rigid_body_modes(prob.mesh.coords, prob.mask)
    full = amg.setup(A, B, amg.AMGOptions(coarse_max=400))
    filt = amg.setup(A, B, amg.AMGOptions(coarse_max=400, smooth_filtered=True))
    assert filt[0].P.nnz < full[0].P.nnz and filt[1].A.nnz < full[1].A.nnz
    opt = amg.AMGOptions(coarse_max=400, smooth_filtered=True)
    res = krylov.pcg(A, b, lambda r: amg.vcycle(filt, r, opt=opt))
    assert res.converged and np.linalg.norm(b - A @ res.u) <= 1e-8 * np.linalg.norm(b)
