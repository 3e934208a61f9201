"""Learned initial guess for PCG: data generation with the library's own
batched solver, training with the library's MPNN kernels (float32 forward,
backward and Adam on the GPU), and evaluation against the zero guess.

The network only proposes u0; it is scaled to its energy-optimal multiple
(amg_energy_scale, which falls back to the zero guess when the guess cannot
beat zero in the energy norm), and the solve still runs to the same true
relative residual, so accuracy never depends on the network.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

import meshgen as mg

from . import AMG, MPNN, assemble, assemble_load

S_U = 1.0e-3
H, L, F = 64, 4, 10


def init_params(seed: int = 0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases, in the
    parameter order of the C ABI (numpy default_rng(seed))."""
    rng = np.random.default_rng(seed)
    parts = []

    def u(fi, shape):
        a = 1.0 / np.sqrt(fi)
        return rng.uniform(-a, a, shape).ravel()

    parts += [u(F, (F, H)), np.zeros(H)]
    for _ in range(L):
        # W_s, W_n, W_g and the three directional weights, then b
        parts += [u(6 * H, (H, H)) for _ in range(6)] + [np.zeros(H)]
    parts += [u(H, (H, 3)), np.zeros(3)]
    return np.concatenate(parts).astype(np.float32)


@dataclasses.dataclass
class Dataset:
    T: object        # [S, N] float64 (device)
    f: object        # [S, 3] float64 (device) uniform body force per sample (zero rows = none)
    U: object        # [S, N, 3] float32 (device): solution / S_U
    iters: list
    solve_s: float


class Problem:
    """One P1 disc, its assembled operator, AMG hierarchy and MPNN graph."""

    def __init__(self, nr, nth, nz, max_nrhs=64, device="cuda:0", aggregation="mis2"):
        import torch
        self.prob = mg.disc_problem(nr, nth, nz, 1, seed=0)
        m = self.prob.mesh
        self.mesh = m
        dev = torch.device(device)
        self.dev = dev
        self.coords = torch.from_numpy(m.coords).to(dev)
        self.cells = torch.from_numpy(m.cells).to(dev)
        self.mask = torch.from_numpy(self.prob.mask).to(dev)
        T0 = torch.full((m.n_nodes,), self.prob.T_ref, dtype=torch.float64, device=dev)
        self.A, _ = assemble(self.coords, self.cells, 1, self.prob.E, self.prob.nu, self.prob.alpha,
                             self.prob.T_ref, T0, mask=self.mask)
        self.amg = AMG(self.A, self.coords, self.mask, max_nrhs=max_nrhs, aggregation=aggregation)
        self.net = MPNN(self.A, self.coords)

    def fields(self, seeds):
        """Temperature fields and uniform body forces of the load-case family."""
        m = self.mesh
        T = np.stack([mg.disc_temperature_bumps(m, s) for s in seeds])
        fv = np.zeros((len(seeds), 3))
        for i, s in enumerate(seeds):
            f = mg.body_force_case(m, s)
            if f is not None:
                fv[i] = f[0]
        return T, fv

    def loads(self, T, fv):
        """b [N, 3, k] for k load cases (device tensors T [k, N], fv [k, 3])."""
        import torch
        k = T.shape[0]
        f = fv[:, None, :].expand(k, self.mesh.n_nodes, 3).contiguous()
        return assemble_load(self.coords, self.cells, 1, self.prob.E, self.prob.nu, self.prob.alpha,
                             self.prob.T_ref, T, f=f, mask=self.mask)

    def generate(self, seeds, batch=64, log=print):
        """Solve every load case (float64, rtol 1e-8) in batches of `batch` columns."""
        import torch
        T_np, f_np = self.fields(seeds)
        T = torch.from_numpy(T_np).to(self.dev)
        fv = torch.from_numpy(f_np).to(self.dev)
        n = self.mesh.n_nodes
        U = torch.empty((len(seeds), n, 3), dtype=torch.float32, device=self.dev)
        iters = []
        t0 = time.perf_counter()
        for s0 in range(0, len(seeds), batch):
            s1 = min(len(seeds), s0 + batch)
            b = self.loads(T[s0:s1].contiguous(), fv[s0:s1].contiguous())
            u, rep = self.amg.solve(b)
            assert all(rep.converged), "training solve did not converge"
            U[s0:s1] = (u.permute(2, 0, 1) / S_U).float()
            iters += rep.iters
            log(f"  solved {s1}/{len(seeds)} (max {max(rep.iters)} it)")
        torch.cuda.synchronize()
        return Dataset(T, fv, U, iters, time.perf_counter() - t0)

    def features(self, T_row, f_vec):
        import torch
        f = None
        if float(f_vec.abs().max()) > 0:
            f = f_vec[None, :].expand(self.mesh.n_nodes, 3).contiguous()
        return self.net.features(T_row.contiguous(), self.prob.T_ref, self.mask, f)

    def train(self, data: Dataset, epochs=8, lr=1e-3, seed=0, log=print, loss="energy"):
        """Adam on the relative energy error of the energy-optimally scaled
        guess (the quantity the solve sees; loss="energy") or on the mean
        squared error (loss="mse")."""
        import torch
        params = torch.from_numpy(init_params(seed)).to(self.dev)
        m1 = torch.zeros_like(params)
        v1 = torch.zeros_like(params)
        S = data.T.shape[0]
        rng = np.random.default_rng(seed + 1)
        step = 0
        hist = []
        t0 = time.perf_counter()
        for ep in range(epochs):
            tot = 0.0
            for i in rng.permutation(S).tolist():
                X = self.features(data.T[i], data.f[i])
                self.net.forward(params, X, self.mask)
                if loss == "energy":
                    gy, lv = self.net.energy_grad(self.amg, data.U[i])
                    g = self.net.backward_from(params, gy)
                else:
                    g, lv = self.net.backward(params, data.U[i])
                step += 1
                lr_t = lr * (0.5 ** (ep // max(1, epochs // 4)))
                self.net.adam_step(params, g, m1, v1, step, lr=lr_t)
                tot += lv
            hist.append(tot / S)
            log(f"  epoch {ep}: mean loss {tot / S:.4e}")
        torch.cuda.synchronize()
        return params, hist, time.perf_counter() - t0

    def guess(self, params, T_row, f_vec):
        X = self.features(T_row, f_vec)
        self.net.forward(params, X, self.mask)
        return self.net.guess()

    def evaluate(self, params, data: Dataset, log=print):
        """Per test case: iterations and solve time from the scaled learned guess
        and from zero, both to true relres 1e-8 in float64, and the time of
        the guess itself (features, network, energy-optimal scaling)."""
        import torch
        res = []
        for i in range(data.T.shape[0]):
            b = self.loads(data.T[i:i + 1].contiguous(), data.f[i:i + 1].contiguous()).reshape(-1).contiguous()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u0 = self.guess(params, data.T[i], data.f[i])
            # energy-optimal multiple of the guess; gamma = 0 falls back to zero
            gamma = self.amg.energy_scale(b, u0)
            torch.cuda.synchronize()
            ms_inf = (time.perf_counter() - t0) * 1e3
            r0 = float(torch.linalg.norm(b - self.apply_A(u0)))
            uz, rz = self.amg.solve(b)
            ug, rg = self.amg.solve(b, u0=u0)
            err = float(torch.linalg.norm(ug - uz) / torch.linalg.norm(uz))
            e0 = float(torch.linalg.norm(u0 - uz) / torch.linalg.norm(uz))
            res.append({"iters_zero": rz.iters[0], "iters_guess": rg.iters[0], "ms_zero": rz.time_ms,
                        "ms_guess": rg.time_ms, "ms_inference": ms_inf, "gamma": gamma, "guess_used": gamma > 0,
                        "relres0": r0 / float(torch.linalg.norm(b)), "rel_err0": e0,
                        "relres_true_guess": rg.relres_true[0], "rel_diff": err})
        return res

    def apply_A(self, x):
        """A x with the library operator (level 0, float64)."""
        from . import TE_OP_A
        return self.amg.apply(0, TE_OP_A, x.contiguous())
