"""Oracle: message-passing network for the learned initial displacement guess
(test infrastructure only; see the package docstring).

The paper's transient runs start each solve from the previous step's solution
(Sec. 5.3); here a small network maps the load (temperature and body force)
to a starting displacement instead.  Architecture, on the P1 vertex graph of
the mesh (directed edges u -> v for every pair of distinct vertices of one
cell), hidden width H = 64, L = 4 message-passing layers:

    h0   = relu(X W_in + b_in)                                   X: [N, F]
    for l = 1..L:
        m    = mean_{u in N(v)} h_u           (neighbour mean, 1/deg_v)
        g    = mean_v h_v                      (global context, one row)
        d_k  = sum_{u in N(v)} w^k_vu h_u      (k = x, y, z; directional sums)
        h    = h + relu(h W_s[l] + m W_n[l] + g W_g[l]
                        + d_x W_dx[l] + d_y W_dy[l] + d_z W_dz[l] + b[l])
    y    = (h W_out + b_out) * (1 - mask)                        [N, 3]
    u0   = s_u * y

with w^k_vu = (x_u - x_v)_k / (deg_v l_v), l_v the mean length of the edges
at v: a first-difference stencil, so the layers can form the gradients and
divergences a displacement driven by thermal expansion is made of (the mean
and the global context alone are isotropic).

Losses: the mean over the N*3 entries of (y - u_true/s_u)^2, and the
relative energy error of the energy-optimally scaled guess,
1 - (t, A u)^2 / ((u, A u)(t, A t)) with u = s_u y, t = u_true: the quantity
the solve sees, since the guess is used at its optimal multiple.
Forward and backward are written out by hand in float64; `grad_check`
compares them with central finite differences.
"""
from __future__ import annotations

import numpy as np

H = 64
L = 4
F_IN = 10
S_T = 500.0
S_F = 2.0e9
S_X = 0.5
S_U = 1.0e-3


def features(coords, T, T_ref, f, mask):
    """X[N, 10] = [dT/S_T, f/S_F (3), mask (3), (x - centroid)/S_X (3)]."""
    n = coords.shape[0]
    X = np.zeros((n, F_IN))
    X[:, 0] = (T - T_ref) / S_T
    if f is not None:
        X[:, 1:4] = f / S_F
    X[:, 4:7] = mask
    X[:, 7:10] = (coords - coords.mean(axis=0)) / S_X
    return X


def vertex_graph(cells, n):
    """CSR (ptr, nbr) of the directed vertex graph, neighbours ascending."""
    c = cells[:, :4].astype(np.int64)
    I = np.repeat(c, 4, axis=1).ravel()
    J = np.tile(c, (1, 4)).ravel()
    sel = I != J
    keys = np.unique(I[sel] * n + J[sel])
    rows = keys // n
    ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=ptr[1:])
    return ptr, keys % n


LAYER_KEYS = ("W_s", "W_n", "W_g", "W_dx", "W_dy", "W_dz", "b")
N_IN = 6   # inputs of a layer's transform: h, m, g, d_x, d_y, d_z


def init_params(seed=0):
    """Deterministic init: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from
    numpy's default_rng(seed), drawn in the order listed."""
    rng = np.random.default_rng(seed)

    def u(fi, shape):
        a = 1.0 / np.sqrt(fi)
        return rng.uniform(-a, a, shape)

    p = {"W_in": u(F_IN, (F_IN, H)), "b_in": np.zeros(H)}
    for l in range(L):
        for k in LAYER_KEYS[:-1]:
            p[f"{k}{l}"] = u(N_IN * H, (H, H))
        p[f"b{l}"] = np.zeros(H)
    p["W_out"] = u(H, (H, 3))
    p["b_out"] = np.zeros(3)
    return p


PARAM_ORDER = ["W_in", "b_in"] + [f"{k}{l}" for l in range(L) for k in LAYER_KEYS] + ["W_out", "b_out"]


def direction_weights(coords, ptr, nbr):
    """w[e, k] = (x_u - x_v)_k / (deg_v l_v) for the directed edge e = (v, u)
    of row v, l_v the mean length of the edges at v."""
    n = coords.shape[0]
    deg = np.diff(ptr)
    rows = np.repeat(np.arange(n), deg)
    dx = coords[nbr] - coords[rows]
    elen = np.linalg.norm(dx, axis=1)
    lv = np.bincount(rows, weights=elen, minlength=n) / np.maximum(deg, 1)
    scale = 1.0 / (np.maximum(deg, 1) * np.where(lv > 0, lv, 1.0))
    return dx * scale[rows][:, None]


def _dir_sum(ptr, nbr, w, h):
    """d[v, k, :] = sum over the edges (v, u) of w[e, k] h_u."""
    rows = np.repeat(np.arange(h.shape[0]), np.diff(ptr))
    out = np.zeros((h.shape[0], 3, h.shape[1]))
    for k in range(3):
        np.add.at(out[:, k], rows, w[:, k:k + 1] * h[nbr])
    return out


def _dir_sum_T(ptr, nbr, w, g):
    """Adjoint of _dir_sum: dh_u = sum over the edges (v, u) of w[e, k] g[v, k]."""
    rows = np.repeat(np.arange(g.shape[0]), np.diff(ptr))
    out = np.zeros((g.shape[0], g.shape[2]))
    for k in range(3):
        np.add.at(out, nbr, w[:, k:k + 1] * g[rows, k])
    return out


def _mean_nbr(ptr, nbr, h):
    deg = np.diff(ptr)
    s = np.zeros_like(h)
    rows = np.repeat(np.arange(h.shape[0]), deg)
    np.add.at(s, rows, h[nbr])
    return s / np.maximum(deg, 1)[:, None]


def _mean_nbr_T(ptr, nbr, gm):
    """Adjoint of _mean_nbr: d h_u = sum over v with u in N(v) of gm_v / deg_v."""
    deg = np.diff(ptr)
    rows = np.repeat(np.arange(gm.shape[0]), deg)
    w = gm / np.maximum(deg, 1)[:, None]
    out = np.zeros_like(gm)
    np.add.at(out, nbr, w[rows])
    return out


def forward(p, X, ptr, nbr, mask, w):
    """w: direction_weights of the graph."""
    cache = {}
    a0 = X @ p["W_in"] + p["b_in"]
    h = np.maximum(a0, 0.0)
    cache["a_in"] = a0
    hs = [h]
    for l in range(L):
        m = _mean_nbr(ptr, nbr, h)
        g = h.mean(axis=0, keepdims=True)
        d = _dir_sum(ptr, nbr, w, h)
        a = (h @ p[f"W_s{l}"] + m @ p[f"W_n{l}"] + g @ p[f"W_g{l}"] + d[:, 0] @ p[f"W_dx{l}"]
             + d[:, 1] @ p[f"W_dy{l}"] + d[:, 2] @ p[f"W_dz{l}"] + p[f"b{l}"])
        cache[f"m{l}"], cache[f"g{l}"], cache[f"d{l}"], cache[f"a{l}"] = m, g, d, a
        h = h + np.maximum(a, 0.0)
        hs.append(h)
    keep = 1.0 - mask.astype(np.float64)
    y = (h @ p["W_out"] + p["b_out"]) * keep
    cache["hs"] = hs
    cache["keep"] = keep
    return y, cache


def loss(y, u_true_scaled):
    d = y - u_true_scaled
    return float((d * d).mean())


def backward(p, X, ptr, nbr, w, cache, y, u_true_scaled):
    """Gradients of the mean-squared loss with respect to every parameter."""
    gy = 2.0 * (y - u_true_scaled) / y.size
    return backward_from(p, X, ptr, nbr, w, cache, gy)


def energy_loss(y, u_true_scaled, A, keep):
    """Relative energy error of the energy-optimally scaled guess u = S_U y
    (masked): 1 - c^2 / (a e) with a = (u, A u), c = (t, A u), e = (t, A t),
    t = S_U u_true_scaled (A: assembled operator on [3N]); returns
    (loss, dL/dy).  A zero guess has loss 1 and gradient 0."""
    u = (S_U * y * keep).reshape(-1)
    t = (S_U * u_true_scaled).reshape(-1)
    Au, At = A @ u, A @ t
    a, c, e = float(u @ Au), float(u @ At), float(t @ At)
    if a <= 0.0:
        return 1.0, np.zeros_like(y)
    dLdu = -2.0 * c / (a * e) * At + 2.0 * c * c / (a * a * e) * Au
    return 1.0 - c * c / (a * e), S_U * dLdu.reshape(y.shape) * keep


def backward_from(p, X, ptr, nbr, w, cache, gy):
    """Gradients of a loss with dL/dy = gy with respect to every parameter."""
    n = X.shape[0]
    gy = gy * cache["keep"]
    hs = cache["hs"]
    g = {}
    g["W_out"] = hs[-1].T @ gy
    g["b_out"] = gy.sum(axis=0)
    gh = gy @ p["W_out"].T
    for l in reversed(range(L)):
        h_prev = hs[l]
        ga = gh * (cache[f"a{l}"] > 0)
        d = cache[f"d{l}"]
        g[f"W_s{l}"] = h_prev.T @ ga
        g[f"W_n{l}"] = cache[f"m{l}"].T @ ga
        g[f"W_g{l}"] = cache[f"g{l}"].T @ ga.sum(axis=0, keepdims=True)
        for k, key in enumerate(("W_dx", "W_dy", "W_dz")):
            g[f"{key}{l}"] = d[:, k].T @ ga
        g[f"b{l}"] = ga.sum(axis=0)
        gm = ga @ p[f"W_n{l}"].T
        gg = ga.sum(axis=0, keepdims=True) @ p[f"W_g{l}"].T
        gd = np.stack([ga @ p[f"{key}{l}"].T for key in ("W_dx", "W_dy", "W_dz")], axis=1)
        gh = (gh + ga @ p[f"W_s{l}"].T + _mean_nbr_T(ptr, nbr, gm) + np.repeat(gg / n, n, axis=0)
              + _dir_sum_T(ptr, nbr, w, gd))
    ga0 = gh * (cache["a_in"] > 0)
    g["W_in"] = X.T @ ga0
    g["b_in"] = ga0.sum(axis=0)
    return g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015) with bias correction; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in PARAM_ORDER:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def _pattern(cache):
    keys = ["a_in"] + [f"a{l}" for l in range(L)]
    return np.concatenate([(cache[k] > 0).ravel() for k in keys])


def grad_check(p, X, ptr, nbr, w, mask, ut, h=1e-6, n_probe=3, seed=0, abs_floor=1e-9):
    """Max relative difference between backward() and central differences
    over n_probe random entries of every parameter.  Probes whose +-h
    evaluations change a ReLU's active set are skipped (the loss has a kink
    there); the difference is measured as |fd - an| / (max(|fd|,|an|) + abs_floor/rel)
    with abs_floor covering the finite-difference rounding error."""
    y, cache = forward(p, X, ptr, nbr, mask, w)
    g = backward(p, X, ptr, nbr, w, cache, y, ut)
    rng = np.random.default_rng(seed)
    worst = 0.0
    checked = 0
    for k in PARAM_ORDER:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(n_probe, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            yp, cp = forward(p, X, ptr, nbr, mask, w)
            flat[idx] = old - h
            ym, cm = forward(p, X, ptr, nbr, mask, w)
            flat[idx] = old
            if not np.array_equal(_pattern(cp), _pattern(cm)):
                continue
            fd = (loss(yp, ut) - loss(ym, ut)) / (2 * h)
            an = g[k].reshape(-1)[idx]
            err = abs(fd - an) - abs_floor
            worst = max(worst, max(err, 0.0) / max(abs(fd), abs(an), 1e-30))
            checked += 1
    assert checked >= len(PARAM_ORDER), "too many probes fell on ReLU kinks"
    return worst
