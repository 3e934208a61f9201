"""Pins of the oracle's message-passing network: backward against central
finite differences, the adjoint identities of the neighbour mean and the
directional sums, the direction weights worked by hand, masking, a
hand-computed forward on a 3-vertex graph, and the scaled energy loss
(finite differences, scale invariance, closed form)."""
import numpy as np

import meshgen as mg
from oracle import mpnn
from oracle import mpnn as om


def _small():
    m = mg.disc_mesh(3, 12, 2, 1)
    rng = np.random.default_rng(1)
    T = 300 + rng.uniform(0, 100, m.n_nodes)
    mask = mg.disc_clamp_bore(m)
    X = mpnn.features(m.coords, T, 300.0, None, mask)
    ptr, nbr = mpnn.vertex_graph(m.cells, m.n_nodes)
    ut = rng.normal(size=(m.n_nodes, 3)) * (1 - mask)
    w = mpnn.direction_weights(m.coords, ptr, nbr)
    return m, X, ptr, nbr, w, mask, ut


def test_vertex_graph_is_p1_pattern_without_diagonal():
    m = mg.disc_mesh(80, 344, 11, 1)
    ptr, nbr = mpnn.vertex_graph(m.cells, m.n_nodes)
    assert nbr.size == 4_426_592  # = 4,760,960 blocks - 334,368 diagonal
    rows = np.repeat(np.arange(m.n_nodes), np.diff(ptr))
    assert not np.any(rows == nbr)


def test_gradients_match_finite_differences():
    m, X, ptr, nbr, w, mask, ut = _small()
    p = mpnn.init_params(3)
    # non-zero biases so every ReLU branch is exercised
    rng = np.random.default_rng(9)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.normal(size=p[k].shape) * 0.1
    assert mpnn.grad_check(p, X, ptr, nbr, w, mask, ut, n_probe=4) < 1e-6


def test_neighbour_mean_adjoint():
    m, X, ptr, nbr, w, mask, ut = _small()
    rng = np.random.default_rng(2)
    a = rng.normal(size=(m.n_nodes, 5))
    b = rng.normal(size=(m.n_nodes, 5))
    lhs = (mpnn._mean_nbr(ptr, nbr, a) * b).sum()
    rhs = (a * mpnn._mean_nbr_T(ptr, nbr, b)).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_directional_sum_adjoint():
    m, X, ptr, nbr, w, mask, ut = _small()
    rng = np.random.default_rng(6)
    a = rng.normal(size=(m.n_nodes, 5))
    b = rng.normal(size=(m.n_nodes, 3, 5))
    lhs = (mpnn._dir_sum(ptr, nbr, w, a) * b).sum()
    rhs = (a * mpnn._dir_sum_T(ptr, nbr, w, b)).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_direction_weights_by_hand():
    # vertex 0 at the origin with neighbours at (2,0,0) and (0,1,0); vertex 1
    # and 2 each see vertex 0 only
    coords = np.array([[0.0, 0, 0], [2.0, 0, 0], [0.0, 1, 0]])
    ptr = np.array([0, 2, 3, 4])
    nbr = np.array([1, 2, 0, 0])
    w = mpnn.direction_weights(coords, ptr, nbr)
    # row 0: deg 2, mean edge length 1.5 -> (x_u - x_0) / 3
    assert np.allclose(w[0], [2 / 3, 0, 0]) and np.allclose(w[1], [0, 1 / 3, 0])
    # row 1: deg 1, length 2 -> (-2, 0, 0) / 2; row 2: (0, -1, 0) / 1
    assert np.allclose(w[2], [-1, 0, 0]) and np.allclose(w[3], [0, -1, 0])
    # the sums of a field h: d[v, k] = sum_u w[e, k] h_u
    h = np.array([[1.0], [4.0], [10.0]])
    d = mpnn._dir_sum(ptr, nbr, w, h)
    assert np.allclose(d[0, :, 0], [8 / 3, 10 / 3, 0]) and np.allclose(d[1, :, 0], [-1, 0, 0])


def test_masked_outputs_are_zero_and_param_count():
    m, X, ptr, nbr, w, mask, ut = _small()
    p = mpnn.init_params(0)
    y, _ = mpnn.forward(p, X, ptr, nbr, mask, w)
    assert np.all(y[mask.astype(bool)] == 0)
    n = sum(p[k].size for k in mpnn.PARAM_ORDER)
    assert n == 10 * 64 + 64 + 4 * (6 * 64 * 64 + 64) + 64 * 3 + 3


def test_forward_by_hand_three_vertices():
    # path graph 0 - 1 - 2 along x at 0, 1, 3: F_IN inputs, recomputed with
    # the stencil written out (w = (x_u - x_v) / (deg_v l_v))
    ptr = np.array([0, 1, 3, 4])
    nbr = np.array([1, 0, 2, 1])
    coords = np.array([[0.0, 0, 0], [1.0, 0, 0], [3.0, 0, 0]])
    w = mpnn.direction_weights(coords, ptr, nbr)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(3, mpnn.F_IN))
    p = mpnn.init_params(1)
    mask = np.zeros((3, 3))
    y, _ = mpnn.forward(p, X, ptr, nbr, mask, w)
    h = np.maximum(X @ p["W_in"] + p["b_in"], 0)
    for l in range(mpnn.L):
        m = np.stack([h[1], 0.5 * (h[0] + h[2]), h[1]])
        g = (h[0] + h[1] + h[2]) / 3
        # vertex 0: one edge of length 1 to x = 1; vertex 1: edges to 0 and
        # 3, mean length 1.5, deg 2; vertex 2: one edge of length 2 to x = 1
        dx = np.stack([1.0 * h[1], (-1.0 * h[0] + 2.0 * h[2]) / 3.0, -1.0 * h[1]])
        h = h + np.maximum(h @ p[f"W_s{l}"] + m @ p[f"W_n{l}"] + g @ p[f"W_g{l}"] + dx @ p[f"W_dx{l}"]
                           + p[f"b{l}"], 0)
    ref = h @ p["W_out"] + p["b_out"]
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_adam_first_step_closed_form():
    # bias-corrected first Adam step moves every weight by lr * sign(g)
    p = {k: np.ones(2) for k in mpnn.PARAM_ORDER}
    g = {k: np.array([3.0, -0.5]) for k in mpnn.PARAM_ORDER}
    mpnn.adam_step(p, g, {}, lr=0.01)
    for k in mpnn.PARAM_ORDER:
        assert np.allclose(p[k], [0.99, 1.01], rtol=0, atol=1e-9)


def test_grad_check_detects_a_planted_adjoint_mistake(monkeypatch):
    # the classic mistake: transpose of the neighbour mean weighted by 1/deg_u
    m, X, ptr, nbr, w, mask, ut = _small()
    p = mpnn.init_params(3)

    def wrong(ptr_, nbr_, gm):
        deg = np.diff(ptr_)
        rows = np.repeat(np.arange(gm.shape[0]), deg)
        out = np.zeros_like(gm)
        np.add.at(out, nbr_, gm[rows])
        return out / np.maximum(deg, 1)[:, None]

    monkeypatch.setattr(mpnn, "_mean_nbr_T", wrong)
    assert mpnn.grad_check(p, X, ptr, nbr, w, mask, ut, n_probe=4) > 1e-3


def test_grad_check_detects_a_planted_directional_mistake(monkeypatch):
    # the adjoint of the directional sums taken with the weights of the
    # reverse edge (w[e] of row u instead of row v)
    m, X, ptr, nbr, w, mask, ut = _small()
    p = mpnn.init_params(3)
    right = mpnn._dir_sum_T
    n = m.n_nodes
    rows = np.repeat(np.arange(n), np.diff(ptr))
    rev = {(int(a), int(b)): e for e, (a, b) in enumerate(zip(rows, nbr))}
    wr = w[[rev[(int(b), int(a))] for a, b in zip(rows, nbr)]]
    monkeypatch.setattr(mpnn, "_dir_sum_T", lambda ptr_, nbr_, w_, g: right(ptr_, nbr_, wr, g))
    assert mpnn.grad_check(p, X, ptr, nbr, w, mask, ut, n_probe=4) > 1e-3


def test_energy_loss_gradient_finite_differences():
    from oracle import fem
    prob = mg.disc_problem(3, 12, 2, 1, seed=0)
    A, b, _, _ = fem.assemble_problem(prob)
    rng = np.random.default_rng(3)
    n = prob.mesh.n_nodes
    keep = 1.0 - prob.mask
    t = rng.normal(size=(n, 3)) * keep
    y = rng.normal(size=(n, 3))
    L, g = om.energy_loss(y, t, A, keep)
    for _ in range(6):
        i, j = rng.integers(n), rng.integers(3)
        h = 1e-6
        y2 = y.copy()
        y2[i, j] += h
        Lp, _ = om.energy_loss(y2, t, A, keep)
        y2[i, j] -= 2 * h
        Lm, _ = om.energy_loss(y2, t, A, keep)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-6 * max(abs(fd), 1e-8) + 1e-10
    # the exact solution and any positive multiple of it have zero loss; the
    # loss of a guess is that of every positive multiple; it lies in [0, 1]
    assert abs(om.energy_loss(t, t, A, keep)[0]) <= 1e-14
    assert abs(om.energy_loss(3.7 * t, t, A, keep)[0]) <= 1e-14
    assert abs(om.energy_loss(2.5 * y, t, A, keep)[0] - L) <= 1e-13
    assert 0.0 <= L <= 1.0
    # closed form against a direct solve: 1 - L is the share of the solution's
    # energy the best multiple of the guess captures, ||g u - u*||_A^2 / ||u*||_A^2
    u = (om.S_U * y * keep).reshape(-1)
    ts = (om.S_U * t).reshape(-1)
    gam = (ts @ (A @ u)) / (u @ (A @ u))
    e = gam * u - ts
    assert abs((e @ (A @ e)) / (ts @ (A @ ts)) - L) <= 1e-12
    L0, g0 = om.energy_loss(0.0 * y, t, A, keep)   # a zero guess: loss 1, no gradient
    assert L0 == 1.0 and not g0.any()
