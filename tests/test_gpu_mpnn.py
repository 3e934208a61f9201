"""GPU message-passing network (float32) against the float64 oracle, and the
gain of the trained network as an initial guess.

Tolerance: the GPU runs in float32 (unit roundoff 6e-8); forward outputs and
gradients of a 4-layer network with 64-wide sums and neighbour means agree
with the float64 oracle (same float32-rounded parameters) to ~1e-5 relative;
the bar is 1e-4 normwise per tensor."""
import numpy as np
import pytest

import meshgen as mg
from oracle import mpnn as om
from tests.gpu_util import dev, gpu_assemble, say, torch_cuda

pytestmark = pytest.mark.gpu


def _unflatten(flat):
    p, o = {}, 0
    ref = om.init_params(0)
    for k in om.PARAM_ORDER:
        n = ref[k].size
        p[k] = flat[o:o + n].reshape(ref[k].shape).astype(np.float64)
        o += n
    assert o == flat.size
    return p


def _flatten(p):
    return np.concatenate([p[k].ravel() for k in om.PARAM_ORDER])


@pytest.fixture(scope="module")
def small():
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.disc_problem(5, 20, 2, 1, seed=0)
    m = prob.mesh
    rng = np.random.default_rng(3)
    T = 300 + rng.uniform(-50, 250, m.n_nodes)
    f = np.tile(rng.normal(size=3) * 1e9, (m.n_nodes, 1))
    A, b, d = gpu_assemble(prob)
    net = te.MPNN(A, d["coords"])
    X = net.features(dev(T, torch.float64), prob.T_ref, d["mask"], dev(f, torch.float64))
    Xo = om.features(m.coords, T, prob.T_ref, f, prob.mask)
    ptr, nbr = om.vertex_graph(m.cells, m.n_nodes)
    w = om.direction_weights(m.coords, ptr, nbr)
    p32 = _flatten(om.init_params(1)).astype(np.float32)
    rng2 = np.random.default_rng(4)
    # non-zero biases so both ReLU branches occur
    po = _unflatten(p32)
    for k in po:
        if k.startswith("b"):
            po[k] = rng2.normal(size=po[k].shape).astype(np.float32).astype(np.float64) * 0.1
    p32 = _flatten(po).astype(np.float32)
    po = _unflatten(p32)
    target = (rng.normal(size=(m.n_nodes, 3)) * (1 - prob.mask)).astype(np.float32)
    return dict(prob=prob, net=net, X=X, Xo=Xo, ptr=ptr, nbr=nbr, w=w, p32=p32, po=po, target=target, d=d)


def test_features_match_oracle(small):
    X = small["X"].cpu().numpy()
    assert np.abs(X - small["Xo"]).max() <= 1e-6 * np.abs(small["Xo"]).max()


def test_forward_matches_oracle(small):
    torch = torch_cuda()
    s = small
    y = s["net"].forward(dev(s["p32"]), s["X"], s["d"]["mask"]).cpu().numpy()
    yo, _ = om.forward(s["po"], s["X"].cpu().numpy().astype(np.float64), s["ptr"], s["nbr"], s["prob"].mask,
                       s["w"])
    err = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    say(f"mpnn forward rel err {err:.2e}")
    assert err <= 1e-4


def test_gradients_match_oracle(small):
    s = small
    P = dev(s["p32"])
    s["net"].forward(P, s["X"], s["d"]["mask"])
    g, loss = s["net"].backward(P, dev(s["target"]))
    g = g.cpu().numpy()
    Xo = s["X"].cpu().numpy().astype(np.float64)
    yo, cache = om.forward(s["po"], Xo, s["ptr"], s["nbr"], s["prob"].mask, s["w"])
    go = om.backward(s["po"], Xo, s["ptr"], s["nbr"], s["w"], cache, yo, s["target"].astype(np.float64))
    lo = om.loss(yo, s["target"].astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * lo
    gg = _unflatten(g)
    for k in om.PARAM_ORDER:
        e = np.linalg.norm(gg[k] - go[k]) / max(np.linalg.norm(go[k]), 1e-30)
        assert e <= 1e-4, f"{k}: {e:.2e}"


def test_backward_from_gradient_and_energy_loss_match_oracle(small):
    import paper_1804_10060_amd as te
    from oracle import fem
    torch = torch_cuda()
    s = small
    P = dev(s["p32"])
    s["net"].forward(P, s["X"], s["d"]["mask"])
    rng = np.random.default_rng(12)
    gy = rng.normal(size=(s["prob"].mesh.n_nodes, 3)).astype(np.float32)
    g = s["net"].backward_from(P, dev(gy)).cpu().numpy()
    Xo = s["X"].cpu().numpy().astype(np.float64)
    yo, cache = om.forward(s["po"], Xo, s["ptr"], s["nbr"], s["prob"].mask, s["w"])
    go = om.backward_from(s["po"], Xo, s["ptr"], s["nbr"], s["w"], cache, gy.astype(np.float64))
    gg = _unflatten(g)
    for k in om.PARAM_ORDER:
        e = np.linalg.norm(gg[k] - go[k]) / max(np.linalg.norm(go[k]), 1e-30)
        assert e <= 1e-4, f"{k}: {e:.2e}"
    # energy loss and its gradient at the GPU's own output y, with the library
    # operator vs the oracle's: float64 arithmetic on the same y, so the loss
    # agrees to rounding (the operators agree to 1e-13) and the float32
    # gradient to its rounding
    prob = s["prob"]
    A, b, d = gpu_assemble(prob)
    h = te.AMG(A, d["coords"], d["mask"])
    y32 = s["net"].forward(P, s["X"], s["d"]["mask"]).cpu().numpy().astype(np.float64)
    gy_e, L = s["net"].energy_grad(h, dev(s["target"]))
    Ao, _, _, _ = fem.assemble_problem(prob)
    Lo, gyo = om.energy_loss(y32, s["target"].astype(np.float64), Ao, 1.0 - prob.mask)
    say(f"energy loss {L:.6e} vs oracle {Lo:.6e}")
    assert abs(L - Lo) <= 1e-10
    assert np.linalg.norm(gy_e.cpu().numpy() - gyo) <= 1e-6 * np.linalg.norm(gyo)
    # and the oracle's loss at its own float64 output is close (forward error 1e-5)
    Lf, _ = om.energy_loss(yo, s["target"].astype(np.float64), Ao, 1.0 - prob.mask)
    assert abs(L - Lf) <= 1e-4 * max(Lf, 1e-3)


def test_adam_step_matches_oracle(small):
    torch = torch_cuda()
    s = small
    rng = np.random.default_rng(8)
    g = rng.normal(size=s["p32"].size).astype(np.float32)
    P = dev(s["p32"].copy())
    m1 = torch.zeros_like(P)
    v1 = torch.zeros_like(P)
    for step in (1, 2):
        s["net"].adam_step(P, dev(g), m1, v1, step, lr=1e-2)
    po = _unflatten(s["p32"])
    go = _unflatten(g)
    st = {}
    for _ in range(2):
        om.adam_step(po, go, st, lr=1e-2)
    ref = _flatten(po)
    assert np.abs(P.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max()


def test_trained_guess_reduces_iterations():
    """Train on 192 method-generated solves of a small disc, test on 16
    held-out fields: the energy-scaled guess takes strictly fewer iterations
    on average than the zero guess.  Guaranteed by construction besides: the
    scaled guess is never worse than zero in the energy norm, and the solve
    from it reaches the same true residual and solution."""
    from paper_1804_10060_amd import learned
    torch = torch_cuda()
    pr = learned.Problem(16, 68, 3, max_nrhs=64)
    say("generate training data")
    train = pr.generate(list(range(10000, 10192)), log=say)
    test = pr.generate(list(range(20000, 20016)), log=say)
    params, hist, t_train = pr.train(train, epochs=24, lr=2e-3, log=say)
    assert hist[-1] < hist[0]
    res = pr.evaluate(params, test)
    iz = np.mean([r["iters_zero"] for r in res])
    ig = np.mean([r["iters_guess"] for r in res])
    say(f"learned guess: mean iterations {ig:.2f} vs zero {iz:.2f}; training {t_train:.1f}s; "
        f"rel err of the scaled guess {np.mean([r['rel_err0'] for r in res]):.3f}, "
        f"gamma {np.mean([r['gamma'] for r in res]):.3f}")
    assert all(r["relres_true_guess"] <= 1e-8 for r in res)
    assert all(r["rel_diff"] <= 1e-6 for r in res)
    # energy of the scaled guess below that of the zero guess: J(g u0) <= 0
    for i in range(4):
        b = pr.loads(test.T[i:i + 1].contiguous(), test.f[i:i + 1].contiguous()).reshape(-1).contiguous()
        u0 = pr.guess(params, test.T[i], test.f[i])
        pr.amg.energy_scale(b, u0)
        J = 0.5 * float(u0 @ pr.apply_A(u0)) - float(b @ u0)
        assert J <= 1e-12 * float(b.norm()) * float(u0.norm() + 1e-300)
    # the gain on the held-out fields: strictly fewer iterations on average
    # than from zero (the time, inference included, is measured at the full
    # size by forms.py learned)
    say(f"solve ms from the guess {np.mean([r['ms_guess'] for r in res]):.3f} + inference "
        f"{np.mean([r['ms_inference'] for r in res]):.3f} vs from zero {np.mean([r['ms_zero'] for r in res]):.3f}")
    assert ig < iz
