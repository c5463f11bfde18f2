"""Training and evaluation of the learned preconditioner.

Every numerical step runs in libq1mf: the Jacobi-PCG solves that generate
the training pairs (q1_pcg_trace), the pair arithmetic (error, residual and
smoothing step: q1_unet_pairs), the encoding, the network's forward and
backward passes, the loss and Adam.  This module only schedules them and keeps
the pairs in device memory (torch tensors as plain buffers, touched only by
copies).

Problem family: scalar Laplace on an n^3-element unit-spacing box,
k = exp(N(0, sigma^2)) iid per cell, u = 0 on the z = 0 face, right-hand side
U(-1, 1) on the free nodes.  Training fields use seeds 10000 + j, held-out
evaluation fields 90000 + j.

Pairs: along a Jacobi-PCG solve to a tight tolerance, x_k is recorded at a
spread of iterations; with the converged x*, the error e_k = x* - x_k and the
residual r_k = A e_k form an exact pair for the operator.  The network maps
the encoded r_k (unit RMS on the free nodes, plus the nodal log-coefficient
channel) to e_k scaled to unit RMS; flexible PCG is invariant to the scale of
the preconditioned residual, so the scale need not be learned.
"""
from __future__ import annotations

import math
import time

import numpy as np

import seeded_inputs as si

from . import (Q1_PC_JACOBI, UNet, UNetPrecond, q1_fpcg, q1_op_create, q1_pcg, q1_pcg_trace,
               q1_unet_pairs)

TRAIN_SEED0 = 10000
EVAL_SEED0 = 90000


def grid_for(n: int) -> int:
    """Network grid edge for an n-element mesh edge: n + 1 nodes rounded up to 4."""
    return (n + 1 + 3) // 4 * 4


class Problem:
    """Device-resident Laplace problem of the learned-preconditioner family."""

    def __init__(self, n: int, seed: int, sigma: float = 2.0):
        import torch
        self.n, self.seed = n, seed
        xyz, conn = si.box_mesh(n, n, n)
        k = si.field_lognormal(n ** 3, 0.0, sigma, seed)
        mask = si.face_mask(n, n, n, "z0")
        b = si.vec_uniform(xyz.shape[1], seed, si.STREAM_RHS)
        b[mask == 1] = 0.0
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        self.xyz, self.conn = dev(xyz), dev(conn.astype(np.int32))
        self.k = dev(k)
        self.coef = self.k.view(1, -1)
        self.mask = dev(mask.astype(np.uint8))
        self.b = dev(b)
        self.nn = xyz.shape[1]
        self.op = q1_op_create(1, 0, 0, self.xyz, self.conn, self.coef, self.mask)


def snapshot_iters(kmax: int, count: int) -> list[int]:
    """min(count, kmax) distinct iterations in [1, kmax]: half log-spaced, half
    evenly spaced, and where those coincide, further evenly spaced ones."""
    lo = np.unique(np.round(np.geomspace(1, max(kmax, 2), count // 2)).astype(int))
    hi = np.unique(np.linspace(1, kmax, count - count // 2).astype(int))
    chosen = set(int(v) for v in np.concatenate([lo, hi]) if 1 <= v <= kmax)
    rest = [v for v in range(1, kmax + 1) if v not in chosen]
    need = min(count - len(chosen), len(rest))
    if need > 0:  # spacing >= 1 between the picks, so they are distinct
        pick = np.round(np.linspace(0, len(rest) - 1, need)).astype(int)
        chosen.update(rest[i] for i in pick)
    return sorted(chosen)


class Field:
    """What training keeps of a harvested problem: its size, coefficients and mask
    (the network's coefficient channel and the encoding need nothing else)."""

    def __init__(self, P: Problem):
        self.n, self.k, self.mask = P.n, P.k, P.mask


def harvest(n: int, seeds, per_solve: int, rtol: float = 1e-10, sigma: float = 2.0,
            omega: float | None = 0.6, log=print):
    """Residual -> error pairs from Jacobi-PCG trajectories, written by the
    library (q1_unet_pairs) into preallocated FP32 banks on the device.  Returns
    a dict of the banks r, e ([npairs, nn]), the field index per pair and the
    fields (for the coefficient channel).  With omega, each pair is taken after
    one damped-Jacobi step, as the two-level preconditioner presents it to the
    network: e1 = e - omega D^-1 r and r1 = A e1."""
    import torch
    nn = (n + 1) ** 3
    cap = len(seeds) * per_solve
    rb = torch.empty((cap, nn), dtype=torch.float32, device="cuda")
    eb = torch.empty((cap, nn), dtype=torch.float32, device="cuda")
    fld = np.empty(cap, dtype=np.int64)
    fields, count = [], 0
    t0 = time.perf_counter()
    for j, seed in enumerate(seeds):
        P = Problem(n, seed, sigma)
        x = torch.empty_like(P.b)
        st = q1_pcg(P.op, Q1_PC_JACOBI, P.b, x, rtol, 100000)
        its = snapshot_iters(max(1, int(st["iters"] * 0.9)), per_solve)
        snaps = [torch.empty_like(P.b) for _ in its]
        q1_pcg_trace(P.op, Q1_PC_JACOBI, P.b, x, rtol, 100000, its, snaps)
        m = len(its)
        q1_unet_pairs(P.op, x, snaps, omega or 0.0, [eb[count + i] for i in range(m)],
                      [rb[count + i] for i in range(m)])
        fld[count:count + m] = j
        count += m
        fields.append(Field(P))
        P.op.destroy()
        if (j + 1) % 100 == 0:
            log(f"harvest: {count} pairs from {j + 1} solves ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    log(f"harvest: {count} pairs from {len(fields)} solves in {time.perf_counter() - t0:.2f} s")
    return {"r": rb[:count], "e": eb[:count], "field": fld[:count], "probs": fields}


class Trainer:
    """Adam on mini-batches of encoded pairs."""

    def __init__(self, net: UNet, data: dict, batch: int, seed: int = 0):
        import torch
        self.net, self.data, self.B = net, data, batch
        G = net.D * net.H * net.W
        self.inp = torch.zeros((batch, net.D, net.H, net.W, 8), dtype=torch.bfloat16, device="cuda")
        self.tgt = torch.zeros((batch, net.D, net.H, net.W), dtype=torch.float32, device="cuda")
        self.wgt = torch.zeros_like(self.tgt)
        self.out = torch.empty_like(self.tgt)
        self.dout = torch.empty_like(self.tgt)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.pcs = [UNetPrecond(net, p.n, p.n, p.n, p.k, p.mask) for p in data["probs"]]
        self.rng = np.random.default_rng(seed)
        self.step_no = 0
        self.G = G

    def _fill(self, idx):
        for s, i in enumerate(idx):
            pc = self.pcs[int(self.data["field"][i])]
            r = self.data["r"][i].double()
            e = self.data["e"][i].double()
            pc.encode(r, self.inp[s])
            pc.encode_target(e, self.tgt[s], self.wgt[s])

    def step(self, lr: float) -> None:
        idx = self.rng.integers(0, self.data["r"].shape[0], size=self.B)
        self._fill(idx)
        self.net.forward(self.inp, self.out, self.B)
        self.net.mse(self.out, self.tgt, self.wgt, self.dout, self.loss)
        self.net.backward(self.dout)
        self.step_no += 1
        self.net.adam_step(lr, self.step_no)

    def train(self, steps: int, lr: float = 1e-3, lr_min: float = 1e-5, log=print,
              log_every: int = 50):
        import torch
        hist = []
        t0 = time.perf_counter()
        for s in range(steps):
            lr_s = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * s / max(1, steps)))
            self.step(lr_s)
            if (s + 1) % log_every == 0 or s == 0 or s + 1 == steps:
                hist.append((s + 1, float(self.loss.item())))
                log(f"train step {s + 1}/{steps} loss {hist[-1][1]:.4f} "
                    f"({time.perf_counter() - t0:.1f} s)")
        torch.cuda.synchronize()
        return hist, time.perf_counter() - t0


VAL_SEED0 = 80000


def evaluate(net: UNet, n: int, seeds, rtol: float = 1e-8, sigma: float = 2.0,
             safeguard_m: int = 50, omega: float | None = 0.6, trunc_m: int = 1,
             periods=(1,), smoothing_baseline: bool = False, log=print):
    """Flexible CG with the network against Jacobi-PCG on held-out fields:
    iterations and wall time (every network inference included), for each
    schedule period p (the network on every p-th preconditioner call, the
    Jacobi step on the others).  omega: damping of the two-level form's Jacobi
    smoothing, None for z = N(r) (period 1 only).  smoothing_baseline: also run
    the same solver with the network's weights set to zero (the two-level form
    without its learned correction)."""
    import torch
    rows = []
    zero = torch.zeros(net.nparams, dtype=torch.float32, device="cuda") if smoothing_baseline else None
    for seed in seeds:
        P = Problem(n, seed, sigma)
        pc = UNetPrecond(net, n, n, n, P.k, P.mask)
        if omega is not None:
            pc.two_level(P.op, omega)
        x = torch.empty_like(P.b)
        q1_pcg(P.op, Q1_PC_JACOBI, P.b, x, rtol, 100000)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sj = q1_pcg(P.op, Q1_PC_JACOBI, P.b, x, rtol, 100000)
        tj = time.perf_counter() - t0
        row = {"seed": seed, "jacobi_iters": sj["iters"], "jacobi_s": tj,
               "jacobi_true_rel_res": sj["true_rel_res"], "periods": {}}
        for per in periods:
            pc.schedule(per)
            q1_fpcg(P.op, pc, P.b, x, rtol, 5, safeguard_m, trunc_m=trunc_m)  # warm-up
            torch.cuda.synchronize()
            pc.schedule(per)
            t0 = time.perf_counter()
            sn = q1_fpcg(P.op, pc, P.b, x, rtol, 20000, safeguard_m, trunc_m=trunc_m)
            tn = time.perf_counter() - t0
            r = {"nn_iters": sn["iters"], "nn_s": tn, "nn_true_rel_res": sn["true_rel_res"],
                 "nn_status": sn["status"], "nn_fallback_at": sn["fallback_at"]}
            if zero is not None:
                theta = net.get(0)
                net.set_params(zero)
                pc.schedule(per)
                s0 = q1_fpcg(P.op, pc, P.b, x, rtol, 20000, safeguard_m, trunc_m=trunc_m)
                net.set_params(theta)
                r["smoothing_iters"] = s0["iters"]
            row["periods"][per] = r
            log(f"eval seed {seed}: Jacobi-PCG {sj['iters']} it {tj * 1e3:.1f} ms | "
                f"NN-FCG period {per}: {sn['iters']} it {tn * 1e3:.1f} ms "
                f"(fallback at {sn['fallback_at']})")
        rows.append(row)
        pc.destroy()
        P.op.destroy()
    return rows


def choose_period(net: UNet, n: int, periods, nval: int = 2, trunc_m: int = 8, log=print) -> int:
    """The schedule period with the least mean wall time on validation fields
    (seeds 80000 + j, neither training nor held-out fields)."""
    rows = evaluate(net, n, [VAL_SEED0 + j for j in range(nval)], periods=periods,
                    trunc_m=trunc_m, log=log)
    mean = {p: sum(r["periods"][p]["nn_s"] for r in rows) / len(rows) for p in periods}
    return min(mean, key=mean.get)
