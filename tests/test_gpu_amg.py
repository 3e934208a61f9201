"""GPU smoothed-aggregation hierarchy and its components against the oracle.

The hierarchy is built from the oracle's own matrix (uploaded), so both sides
make the integer decisions (strength threshold, aggregation, rank check) on
the same numbers: aggregates must agree exactly.  Level operators, transfer
operators, smoother and V-cycle then agree to rounding.

Tolerances (float64): a sparse product row with t terms differs between two
correct summation orders by at most ~t * eps * (|A||x|)_i; with t <= 6*80 terms
this is below 1e-13 relative to |A||x|, written as SPMV_TOL below.  Composite
operators (smoothed P, Galerkin product, V-cycle) compound a few such steps
and use 1e-11 relative to the operator scale."""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen as mg
from oracle import amg, fem
from tests.gpu_util import dev, oracle_bsr_to_device, say, torch_cuda

pytestmark = pytest.mark.gpu

SPMV_TOL = 1e-13
OP_TOL = 1e-11


def _oracle_system(prob):
    A, b, _, _ = fem.assemble_problem(prob)
    B = fem.rigid_body_modes(prob.mesh.coords, prob.mask)
    return A, b, B


def _gpu_amg_from_oracle_matrix(prob, A, **opts):
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    say("amg_setup from oracle matrix", prob.name)
    return te.AMG(oracle_bsr_to_device(A), dev(prob.mesh.coords, torch.float64), dev(prob.mask), **opts)


@pytest.fixture(scope="module")
def cube_case():
    prob = mg.cube_problem(16, 1)
    A, b, B = _oracle_system(prob)
    levels = amg.setup(A, B)
    h = _gpu_amg_from_oracle_matrix(prob, A)
    return prob, A, b, B, levels, h


@pytest.fixture(scope="module")
def disc_case():
    # P2 disc with three levels at a reduced coarse size
    prob = mg.disc_problem(8, 34, 2, 2, seed=5)
    A, b, B = _oracle_system(prob)
    opt = amg.AMGOptions(coarse_max=400)
    levels = amg.setup(A, B, opt)
    h = _gpu_amg_from_oracle_matrix(prob, A, coarse_max=400)
    return prob, A, b, B, levels, h


@pytest.mark.parametrize("case", ["cube_case", "disc_case"])
def test_hierarchy_matches_oracle(case, request):
    prob, A, b, B, levels, h = request.getfixturevalue(case)
    info = h.info()
    assert info["n_levels"] == len(levels)
    for l, lv in enumerate(levels):
        assert info["n_dof"][l] == lv.A.shape[0]
        if l + 1 < len(levels):
            assert np.array_equal(h.aggregates(l), lv.agg), f"aggregates differ at level {l}"
            assert abs(info["lambda_hat"][l] - lv.lam) <= 1e-10 * lv.lam
        rp, col, val = h.level_matrix(l)
        bs = lv.bs
        G = sp.bsr_matrix((val, col, rp), shape=lv.A.shape).tocsr()
        D = (G - lv.A.tocsr())
        scale = np.abs(lv.A.data).max()
        assert (abs(D).max() if D.nnz else 0.0) <= OP_TOL * scale, f"A_{l} differs"
        assert bs == info["bs"][l]


@pytest.mark.parametrize("case", ["cube_case", "disc_case"])
def test_level_operators_and_transfers(case, request):
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob, A, b, B, levels, h = request.getfixturevalue(case)
    rng = np.random.default_rng(1)
    for l, lv in enumerate(levels):
        x = rng.normal(size=lv.A.shape[0])
        y = h.apply(l, te.TE_OP_A, dev(x, torch.float64)).cpu().numpy()
        ref = lv.A @ x
        bound = (abs(lv.A) @ np.abs(x))
        assert np.all(np.abs(y - ref) <= SPMV_TOL * bound + 1e-300), f"A_{l} x"
        if l + 1 < len(levels):
            xc = rng.normal(size=lv.P.shape[1])
            yp = h.apply(l, te.TE_OP_P, dev(xc, torch.float64)).cpu().numpy()
            refp = lv.P @ xc
            assert np.abs(yp - refp).max() <= OP_TOL * (abs(lv.P) @ np.abs(xc)).max(), f"P_{l}"
            yr = h.apply(l, te.TE_OP_R, dev(x, torch.float64)).cpu().numpy()
            refr = lv.R @ x
            assert np.abs(yr - refr).max() <= OP_TOL * (abs(lv.R) @ np.abs(x)).max(), f"R_{l}"


@pytest.mark.parametrize("case", ["cube_case", "disc_case"])
def test_smoother_and_vcycle(case, request):
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob, A, b, B, levels, h = request.getfixturevalue(case)
    rng = np.random.default_rng(2)
    lv = levels[0]
    g = rng.normal(size=A.shape[0])
    x0 = rng.normal(size=A.shape[0])
    y = h.apply(0, te.TE_OP_SMOOTH, dev(g, torch.float64), dev(x0, torch.float64)).cpu().numpy()
    ref = amg.chebyshev(lv.A, lv.D, g, x0, lv.lam)
    assert np.abs(y - ref).max() <= OP_TOL * np.abs(ref).max()
    z = h.apply(0, te.TE_OP_VCYCLE, dev(g, torch.float64)).cpu().numpy()
    zr = amg.vcycle(levels, g)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    # float32 V-cycle: close to the float64 one at single-precision level
    z32 = h.apply(0, te.TE_OP_VCYCLE, dev(g, torch.float64), precision=te.TE_PREC_MIXED).cpu().numpy()
    assert np.abs(z32 - zr).max() <= 1e-3 * np.abs(zr).max()


def test_imposed_aggregates_reproduce_hierarchy(disc_case):
    """amg_setup_with_aggregates with the oracle's maps gives the same hierarchy."""
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob, A, b, B, levels, h = disc_case
    aggs = [lv.agg for lv in levels[:-1]]
    h2 = te.AMG(oracle_bsr_to_device(A), dev(prob.mesh.coords, torch.float64), dev(prob.mask), aggregates=aggs,
                coarse_max=400)
    assert h2.info()["n_dof"] == h.info()["n_dof"]
    for l in range(len(levels) - 1):
        assert np.array_equal(h2.aggregates(l), levels[l].agg)


def test_rank_deficient_aggregate_takes_the_host_path(disc_case):
    """A one-node aggregate (3 rows for 6 modes) cannot be factored on the
    device: the level goes back to the host QR, which merges it into the
    neighbour aggregate of largest summed strength, as the oracle does; the
    resulting hierarchy matches the oracle's."""
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob, A, b, B, levels, h = disc_case
    agg0 = levels[0].agg.copy()
    i = int(np.flatnonzero(agg0 >= 0)[len(agg0) // 2])
    agg0[i] = agg0.max() + 1
    opt = amg.AMGOptions(coarse_max=400)
    lv2 = amg.setup(A, B, opt, aggregates=[agg0])
    assert lv2[0].agg.max() + 1 == levels[0].agg.max() + 1      # the lone node was merged back
    h2 = te.AMG(oracle_bsr_to_device(A), dev(prob.mesh.coords, torch.float64), dev(prob.mask), aggregates=[agg0],
                coarse_max=400)
    info = h2.info()
    assert info["n_levels"] == len(lv2)
    assert np.array_equal(h2.aggregates(0), lv2[0].agg)
    for l, lv in enumerate(lv2):
        rp, col, val = h2.level_matrix(l)
        G = sp.bsr_matrix((val, col, rp), shape=lv.A.shape).tocsr()
        D = G - lv.A.tocsr()
        assert (abs(D).max() if D.nnz else 0.0) <= OP_TOL * np.abs(lv.A.data).max(), f"A_{l} differs"


def test_filtered_smoothing_matches_oracle():
    """amg_options.smooth_filtered: the prolongators smoothed with the
    filtered operator, level by level against the oracle's, and the solve."""
    from oracle import krylov
    prob = mg.disc_problem(8, 34, 2, 2, seed=5)
    A, b, B = _oracle_system(prob)
    opt = amg.AMGOptions(coarse_max=400, smooth_filtered=True)
    levels = amg.setup(A, B, opt)
    h = _gpu_amg_from_oracle_matrix(prob, A, coarse_max=400, smooth_filtered=1)
    info = h.info()
    assert info["n_levels"] == len(levels)
    for l, lv in enumerate(levels):
        if l + 1 < len(levels):
            assert np.array_equal(h.aggregates(l), lv.agg), f"aggregates differ at level {l}"
            assert info["p_nnzb"][l] * lv.bs * 6 >= lv.P.nnz  # block pattern holds the scalar nonzeros
        rp, col, val = h.level_matrix(l)
        G = sp.bsr_matrix((val, col, rp), shape=lv.A.shape).tocsr()
        D = G - lv.A.tocsr()
        assert (abs(D).max() if D.nnz else 0.0) <= OP_TOL * np.abs(lv.A.data).max(), f"A_{l} differs"
    full = amg.setup(A, B, amg.AMGOptions(coarse_max=400))
    assert levels[1].A.nnz < full[1].A.nnz
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    u, rep = h.solve(dev(b, torch.float64))
    res = krylov.pcg(A, b, lambda r: amg.vcycle(levels, r, opt=opt))
    say(f"filtered smoothing: iters gpu {rep.iters[0]} oracle {res.iters}")
    assert rep.converged == [1] and abs(rep.iters[0] - res.iters) <= 1
    assert np.linalg.norm(u.cpu().numpy() - res.u) <= 1e-8 * np.linalg.norm(res.u)


def test_coarse_symmetric_storage_matches_full(disc_case):
    """Coarse operators stored by their blocks on/above the diagonal
    (coarse_sym = 1, the default) against the full storage of the same
    hierarchy: level matrices agree to the rounding asymmetry of the Galerkin
    product, products and V-cycles to SPMV_TOL / 1e-10, and the solve takes
    the same iterations."""
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob, A, b, B, levels, h = disc_case
    hf = _gpu_amg_from_oracle_matrix(prob, A, coarse_max=400, coarse_sym=0)
    assert h.opts.coarse_sym == 1 and hf.opts.coarse_sym == 0 and hf.info()["n_dof"] == h.info()["n_dof"]
    rng = np.random.default_rng(5)
    for l in range(1, h.info()["n_levels"]):
        rp, col, val = h.level_matrix(l)
        rpf, colf, valf = hf.level_matrix(l)
        assert np.array_equal(rp, rpf) and np.array_equal(col, colf)
        assert np.abs(val - valf).max() <= 1e-13 * np.abs(valf).max(), f"A_{l} values"
        G = sp.bsr_matrix((valf, colf, rpf)).tocsr()
        x = rng.normal(size=G.shape[0])
        y = h.apply(l, te.TE_OP_A, dev(x, torch.float64)).cpu().numpy()
        yf = hf.apply(l, te.TE_OP_A, dev(x, torch.float64)).cpu().numpy()
        bound = abs(G) @ np.abs(x)
        assert np.all(np.abs(y - yf) <= 2 * SPMV_TOL * bound + 1e-300), f"A_{l} x"
        # float32 work runs on a full-storage copy: the same float32 product
        x32 = dev(x, torch.float64)
        y32 = h.apply(l, te.TE_OP_A, x32, precision=te.TE_PREC_MIXED).cpu().numpy()
        yf32 = hf.apply(l, te.TE_OP_A, x32, precision=te.TE_PREC_MIXED).cpu().numpy()
        assert np.array_equal(y32, yf32), f"float32 A_{l} x"
    g = rng.normal(size=A.shape[0])
    z = h.apply(0, te.TE_OP_VCYCLE, dev(g, torch.float64)).cpu().numpy()
    zf = hf.apply(0, te.TE_OP_VCYCLE, dev(g, torch.float64)).cpu().numpy()
    assert np.abs(z - zf).max() <= 1e-10 * np.abs(zf).max()
    u, rep = h.solve(dev(b, torch.float64))
    uf, repf = hf.solve(dev(b, torch.float64))
    assert rep.iters == repf.iters
    assert float((u - uf).norm() / uf.norm()) <= 1e-8
    # the float32 V-cycle runs on full storage in both hierarchies (its
    # Chebyshev intervals come from float64 Lanczos runs, whose summation
    # orders differ, hence not bit for bit)
    um, repm = h.solve(dev(b, torch.float64), precision="mixed")
    umf, repmf = hf.solve(dev(b, torch.float64), precision="mixed")
    assert repm.iters == repmf.iters and repm.converged == [1]
    assert float((um - umf).norm() / umf.norm()) <= 1e-8
