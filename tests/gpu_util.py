"""Helpers shared by the GPU tests: move seeded inputs to the device and run
the library through its Python binding.  Each helper prints what it runs so a
failing GPU step names its case."""
from __future__ import annotations

import sys

import numpy as np

import meshgen as mg


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=None):
    torch = torch_cuda()
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def problem_on_device(prob: mg.Problem):
    torch = torch_cuda()
    m = prob.mesh
    return dict(coords=dev(m.coords, torch.float64), cells=dev(m.cells.astype(np.int32)), degree=m.degree,
                T=dev(prob.T, torch.float64), f=None if prob.f is None else dev(prob.f, torch.float64),
                mask=dev(prob.mask.astype(np.uint8)))


def gpu_assemble(prob: mg.Problem, u_bc=None):
    import paper_1804_10060_amd as te
    d = problem_on_device(prob)
    say("assemble", prob.name, "N =", prob.mesh.n_nodes)
    A, b = te.assemble(d["coords"], d["cells"], d["degree"], prob.E, prob.nu, prob.alpha, prob.T_ref, d["T"],
                       f=d["f"], mask=d["mask"], u_bc=None if u_bc is None else dev(u_bc, torch_cuda().float64))
    return A, b, d


def oracle_bsr_to_device(A):
    """scipy BSR (3x3 blocks) -> te.Matrix on the device (for feeding the oracle's matrix to the GPU setup)."""
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    return te.Matrix(dev(A.indptr.astype(np.int64)), dev(A.indices.astype(np.int32)),
                     dev(A.data.astype(np.float64), torch.float64))


def matrix_to_host(A):
    return (A.row_ptr.cpu().numpy(), A.col_idx.cpu().numpy(), A.val.cpu().numpy())


def oracle_levels_aggregates(levels):
    return [lv.agg.astype(np.int32) for lv in levels[:-1]]
