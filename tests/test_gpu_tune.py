"""Autotuner: every candidate launch configuration computes the same rows,
so tuned operators reproduce the untuned products bit for bit, the tuned
solve matches, and the choices survive a round trip through the cache file."""
import json

import numpy as np
import pytest

import meshgen as mg
from tests.gpu_util import dev, gpu_assemble, say, torch_cuda

pytestmark = pytest.mark.gpu


def test_autotune_keeps_results_and_caches(tmp_path):
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.disc_problem(10, 40, 3, 2, seed=2)
    A, b, d = gpu_assemble(prob)
    h = te.AMG(A, d["coords"], d["mask"], coarse_max=400)
    info = h.info()
    rng = np.random.default_rng(0)
    xs = [dev(rng.normal(size=n), torch.float64) for n in info["n_dof"]]
    before = [h.apply(l, te.TE_OP_A, xs[l]).cpu().numpy() for l in range(info["n_levels"])]
    before32 = h.apply(0, te.TE_OP_A, xs[0], precision=te.TE_PREC_MIXED).cpu().numpy()
    u0, r0 = h.solve(b)
    cache = str(tmp_path / "tune.json")
    rep = h.autotune(cache)
    say(rep)
    assert "best" in rep
    after = [h.apply(l, te.TE_OP_A, xs[l]).cpu().numpy() for l in range(info["n_levels"])]
    for a, c in zip(before, after):
        assert np.array_equal(a, c)
    assert np.array_equal(before32, h.apply(0, te.TE_OP_A, xs[0], precision=te.TE_PREC_MIXED).cpu().numpy())
    u1, r1 = h.solve(b)
    assert abs(r1.iters[0] - r0.iters[0]) <= 1
    assert float(((u1 - u0).norm() / u0.norm()).cpu()) <= 1e-10
    h2 = te.AMG(A, d["coords"], d["mask"], coarse_max=400)
    rep2 = h2.autotune(cache)
    assert "best" not in rep2 and "cached" in rep2
    u2, r2 = h2.solve(b)
    assert r2.iters[0] == r1.iters[0]
    assert float(((u2 - u1).norm() / u1.norm()).cpu()) == 0.0


def test_shared_x_entries_equal_own_loads(tmp_path):
    """The row-wave products (the 6x6-block coarse operators in symmetric
    float64 storage and full float32 copies, and the 6x3-block restrictions)
    with the x entries of a block column loaded once per slot and passed
    round by lane permutes use the same values in the same order as with
    every lane loading them: each level operator's and restriction's
    product, for several launch shapes and both precisions, and the float64
    and mixed solves agree bit for bit."""
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.disc_problem(10, 40, 3, 2, seed=5)
    A, b, d = gpu_assemble(prob)
    h = te.AMG(A, d["coords"], d["mask"], coarse_max=400)
    info = h.info()
    assert h.opts.coarse_sym == 1 and info["n_levels"] >= 3
    rng = np.random.default_rng(1)
    xs = [dev(rng.normal(size=n), torch.float64) for n in info["n_dof"]]
    path = str(tmp_path / "tune.json")
    h.autotune(path, use_cache=False)
    with open(path) as fh:
        keys = list(json.load(fh))

    def run(shape, xb):
        with open(path, "w") as fh:
            json.dump({k: [*shape, 4, 0, 0, xb] for k in keys}, fh)
        h.autotune(path, use_cache=True)
        nl = info["n_levels"]
        ys = [h.apply(l, te.TE_OP_A, xs[l]).cpu().numpy() for l in range(nl)]
        ys += [h.apply(l, te.TE_OP_A, xs[l], precision=te.TE_PREC_MIXED).cpu().numpy() for l in range(nl - 1)]
        ys += [h.apply(l, te.TE_OP_R, xs[l], precision=p).cpu().numpy()
               for l in range(nl - 1) for p in (te.TE_PREC_FP64, te.TE_PREC_MIXED)]
        u, rep = h.solve(b)
        um, repm = h.solve(b, precision="mixed")
        return ys, (u, um), (rep.iters[0], repm.iters[0])

    for shape in ([4, 1, 1, 0], [8, 2, 0, 1], [1, 4, 1, 0]):
        ya, ua, ia = run(shape, 0)
        yb, ub, ib = run(shape, 1)
        for q, (a, c) in enumerate(zip(ya, yb)):
            assert np.array_equal(a, c), (shape, q)
        assert ia == ib and all(torch.equal(p, q) for p, q in zip(ua, ub)), shape
        say(f"launch shape {shape}: level products and both solves ({ia} iterations) equal")
