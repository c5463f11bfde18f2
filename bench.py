#!/usr/bin/env python3
"""Headline benchmark: GDOF/s per matrix-free apply.

Workload: scalar Laplace, trilinear hexahedra on an undistorted 128^3-element
grid (2,146,689 DOF), layered coefficient (one lognormal(0, 1.5) value per
4-cell z-layer times iid lognormal(0, 0.5) per cell), FP64, no boundary
condition.  Every element of the undistorted grid is a parallelepiped, so the
apply takes the exact constant-Jacobian (affine) element path; the jittered
grid (general hexahedra) is reported beside it.  A step is one y = A x apply
with all inputs resident in HBM.  The timed steps rotate over four resident
copies of the operator and its vectors (about 0.75 GB together, three times
the 256 MB MALL), so every apply streams its data from HBM; back-to-back
applies of one copy (warm, partly served from the MALL) and single applies
after a 1 GiB cache flush (cold) are reported beside it.

Prints one JSON line with the roofline of the apply (algorithmic bytes per
apply / event-timed apply duration against 8 TB/s) and the CPU oracle
(assembled CSR, OpenMP SpMV) timed on the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
ROTATE = 4  # resident copies the timed applies rotate over
# HBM bytes per apply measured with rocprofv3 FETCH_SIZE and WRITE_SIZE (each scaled by what
# the counter reads for a plain device copy of known size, see profiles/), keyed by the
# hash of the apply's kernel sources and the grid edge.  A kernel changed since its counters
# were taken hashes differently, so its traffic is reported as null.
KERNEL_SOURCES = ("paper_2308_09839_amd/csrc/q1_tile.hip", "paper_2308_09839_amd/csrc/q1_elem.hpp")
MEASURED_TRAFFIC: dict = {
    # 128^3, owner-computes tiles: FETCH_SIZE 49,158.7 KiB (x 2), WRITE_SIZE 16,786.6 KiB
    # (x 1) per apply
    ("04426c3e67b8fe9b", 128): 117.9e6,
}


def kernel_hash() -> str:
    """Hash of the apply's kernel sources without their line comments and blank
    lines (a comment edit leaves the kernels, and so their traffic, unchanged)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def upload(pr, dtype):
    import numpy as np
    import torch
    t = torch.float64 if dtype == 0 else torch.float32
    d = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=dt)
    mask = d(pr["mask"].astype(np.uint8)) if pr.get("mask") is not None else None
    return d(pr["xyz"], t), d(pr["conn"].astype(np.int32)), d(pr["coef"], t), mask


def time_applies(op, x, y, steps, warmup):
    """Back-to-back applies on the current stream; events bracket the K steps."""
    import torch
    st = torch.cuda.current_stream().cuda_stream
    for _ in range(warmup):
        op.apply(x, y, st)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        op.apply(x, y, st)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def time_rotating(copies, steps, warmup):
    """Applies rotating over resident copies (op, x, y) of the workload on the current
    stream; events on that stream bracket the K steps.  Returns ms per apply."""
    import torch
    st = torch.cuda.current_stream().cuda_stream
    R = len(copies)
    for i in range(warmup):
        op, x, y = copies[i % R]
        op.apply(x, y, st)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        op, x, y = copies[i % R]
        op.apply(x, y, st)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_each(fn, reps, warmup=10):
    """Median of `reps` calls of fn, each bracketed by its own events (launch-bound sizes)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def time_cold(op, x, y, reps, mode="write"):
    """Median of `reps` applies, each timed alone after touching a 1 GiB buffer, which evicts
    the operator's data from L2 and the MALL (256 MB): mode "write" fills it (the apply then
    also competes with the write-back of the dirty lines), mode "read" sums it (clean lines;
    the apply reads from HBM).  The events and the apply are queued behind the flush, not
    after a synchronisation: on an idle GPU the first event would also time the host's
    launch latency (Python, the binding and the runtime), which is no part of the apply."""
    import torch
    flush = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ts = []
    for i in range(reps):
        if mode == "write":
            flush.fill_(float(i))
        else:
            flush.sum()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        op.apply(x, y)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def cpu_baseline(n: int, seed: int):
    """The oracle as it stands on the whole headline workload: CSR assembly once
    (timed apart), then the OpenMP CSR SpMV timed with all host threads and with
    one; plus the oracle's Jacobi-PCG on the 16^3 jittered problem."""
    import numpy as np

    import oracle
    import seeded_inputs as si
    oracle.build(force=False)
    pr = si.problem_laplace_layered(n, seed)
    nn = pr["xyz"].shape[1]
    t0 = time.perf_counter()
    A = oracle.assemble(1, pr["xyz"], pr["conn"], pr["coef"])
    t_asm = time.perf_counter() - t0
    x = si.vec_uniform(nn, seed, si.STREAM_X)

    def spmv_time(min_s):
        A.matvec(x)
        reps, t0 = 0, time.perf_counter()
        while reps < 3 or time.perf_counter() - t0 < min_s:
            A.matvec(x)
            reps += 1
        return (time.perf_counter() - t0) / reps, reps

    threads = oracle.num_threads()
    t_all, reps = spmv_time(4.0)
    oracle.set_num_threads(1)
    t_one, reps1 = spmv_time(4.0)
    oracle.set_num_threads(threads)
    # the oracle's Jacobi-PCG on the 16^3 jittered problem, for the solve-time comparison
    prc, bc = cg16_problem(si)
    Ac = oracle.assemble(1, prc["xyz"], prc["conn"], prc["coef"], prc["mask"])
    t0 = time.perf_counter()
    refc = oracle.pcg(Ac, bc, rtol=1e-8)
    t_cg = time.perf_counter() - t0
    del A
    return dict(value=round(nn / t_all / 1e9, 4), unit="GDOF/s", cores=threads,
                kind="oracle", single_thread_value=round(nn / t_one / 1e9, 4),
                cg16_s=round(t_cg, 5), cg16_iters=refc.iters,
                sample=(f"the whole {n}^3 workload ({nn} DOF): CSR assembled once in "
                        f"{t_asm:.2f} s (not in the rate), OpenMP CSR SpMV timed over {reps} "
                        f"products on {threads} threads and {reps1} on one thread"),
                assembly_s=round(t_asm, 3), spmv_ms=round(t_all * 1e3, 3),
                spmv_single_thread_ms=round(t_one * 1e3, 3))


def bench_csr(q1, si, n, seed, args):
    """Same-GPU CSR SpMV of the assembled 128^3 operator (the matrix-based comparison)."""
    import torch
    pr = si.problem_laplace_layered(n, seed)
    nn = pr["xyz"].shape[1]
    op = q1.q1_op_create(1, 0, 0, *upload(pr, 0))
    t0 = time.perf_counter()
    csr = q1.q1_csr_create(op)
    t_asm = time.perf_counter() - t0
    x = torch.from_numpy(si.vec_uniform(nn, seed, si.STREAM_X)).to("cuda")
    y = torch.empty_like(x)
    ms, _ = time_applies(csr, x, y, args.steps, args.warmup)
    b, _ = csr.bytes()
    nnz = q1.q1_csr_info(csr)[1]
    torch.cuda.synchronize()
    csr.destroy()
    op.destroy()
    return {"csr_spmv_gdofs": round(nn / (ms * 1e-3) / 1e9, 3), "csr_spmv_ms": round(ms, 5),
            "csr_hbm_frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "csr_nnz": nnz,
            "csr_assembly_s": round(t_asm, 3)}


def cg16_problem(si):
    """16^3 jittered Laplace, k = exp(N(0,1)), Dirichlet on z=0, b ~ U(-1, 1) on free nodes."""
    s0 = si.seed_for(0)
    pr = si.problem_laplace_jittered(16, s0)
    b = si.vec_uniform(pr["xyz"].shape[1], s0, si.STREAM_RHS)
    b[pr["mask"] == 1] = 0.0
    return pr, b


def bench_cg16(q1, si, n, seed, args):
    """16^3 jittered Laplace (launch-latency bound): microseconds per apply (median of
    100 individually timed applies after 10 warm-up ones, and 100 applies back to back)
    and FP64 Jacobi-PCG to a 1e-8
    relative residual (wall time of the whole solve and per iteration) through the
    launch-per-kernel driver, the persistent batched kernel (one cooperative launch),
    and the fused single-workgroup kernel."""
    import torch
    pr, b = cg16_problem(si)
    bd = torch.from_numpy(b).to("cuda")
    xd = torch.empty_like(bd)
    res = {}
    op = q1.q1_op_create(1, 0, 0, *upload(pr, 0))
    yd = torch.empty_like(bd)
    res["cg16_apply_us"] = round(1e3 * time_each(lambda: op.apply(bd, yd), 100, 10), 2)
    # the same 100 applies queued back to back (one event pair): the device time per apply,
    # without the host's launch latency that each individually timed apply waits for
    ms_b2b, _ = time_applies(op, bd, yd, 100, 10)
    res["cg16_apply_us_back_to_back"] = round(1e3 * ms_b2b, 2)
    op.destroy()
    for tag, variant in (("", 0), ("_persistent", 3), ("_fused", 0)):
        op = q1.q1_op_create(1, 0, variant, *upload(pr, 0))
        if tag == "":
            solve = lambda: q1.q1_pcg(op, 1, bd, xd, 1e-8, 20000)
        elif tag == "_fused":
            solve = lambda: q1.q1_pcg_fused(op, 1, bd, xd, 1e-8, 20000)
        else:
            solve = lambda: q1.q1_batched_pcg([op], [[bd]], [[xd]], 1e-8, 20000)[0]
        solve()  # warm-up
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            st = solve()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        t = ts[len(ts) // 2]
        res[f"cg16{tag}_gpu_s"] = round(t, 6)
        res[f"cg16{tag}_iters"] = st["iters"]
        res[f"cg16{tag}_us_per_iter"] = round(1e6 * t / max(1, st["iters"]), 2)
        res[f"cg16{tag}_rel_res"] = st["rel_res"]
        op.destroy()
    torch.cuda.synchronize()
    return res


def bench_cg128(q1, si, n, seed, args):
    """The paper's CG studies on the 128^3 workload with Dirichlet u = 0 on z = 0:
    FP64 Jacobi-PCG throughput (N_dof x iterations / time) beside the apply alone, the
    per-iteration time split into apply, dot products and vector updates, and the two
    dot-product implementations (two-stage deterministic, single-pass atomic) over
    block counts."""
    import torch
    pr = si.problem_laplace_layered(n, seed)
    pr["mask"] = si.face_mask(n, n, n, "z0")
    nn = pr["xyz"].shape[1]
    op = q1.q1_op_create(1, 0, 0, *upload(pr, 0))
    b = si.vec_uniform(nn, seed, si.STREAM_RHS)
    b[pr["mask"] == 1] = 0.0
    bd = torch.from_numpy(b).to("cuda")
    xd = torch.empty_like(bd)
    yd = torch.empty_like(bd)
    res = {}
    ms_apply, _ = time_applies(op, bd, yd, 200, 50)
    q1.q1_pcg(op, 1, bd, xd, 0.0, 20)  # warm-up
    torch.cuda.synchronize()
    K = 400
    t0 = time.perf_counter()
    st = q1.q1_pcg(op, 1, bd, xd, 0.0, K)
    t_pcg = time.perf_counter() - t0
    us_iter = 1e6 * t_pcg / st["iters"]
    res["cg128_iters_timed"] = st["iters"]
    res["cg128_us_per_iter"] = round(us_iter, 2)
    res["cg128_gdofs"] = round(nn * st["iters"] / t_pcg / 1e9, 3)
    res["cg128_apply_us"] = round(1e3 * ms_apply, 2)
    res["cg128_apply_gdofs"] = round(nn / (ms_apply * 1e-3) / 1e9, 3)
    # dot products: the two implementations over block counts
    work = torch.empty(1024, dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    s_ = torch.cuda.current_stream().cuda_stream
    for name, variant in (("twostage", q1.Q1_DOT_TWO_STAGE), ("atomic", q1.Q1_DOT_ATOMIC)):
        for nb in (256, 1024):
            ms, _ = time_applies(_DotOp(q1, bd, yd, out, variant, nb, work), None, None, 500, 50)
            res[f"dot128_{name}_nb{nb}_us"] = round(1e3 * ms, 2)
            res[f"dot128_{name}_nb{nb}_gbs"] = round(2 * 8 * nn / (ms * 1e-3) / 1e9, 1)
    ms_dot, _ = time_applies(_DotOp(q1, bd, yd, out, q1.Q1_DOT_TWO_STAGE, 0, work), None, None,
                             500, 50)
    # per iteration: one apply that also forms the p.q partials (timed here without
    # them), the update (x, r, two dots) and the direction; the separate p.q dot the
    # apply replaces is timed beside them
    res["cg128_split_us"] = {"apply": round(1e3 * ms_apply, 2),
                             "update_direction_and_their_dots": round(
                                 us_iter - 1e3 * ms_apply, 2)}
    res["cg128_separate_dot_pq_us"] = round(1e3 * ms_dot, 2)
    op.destroy()
    torch.cuda.synchronize()
    return res


def bench_family(q1, si, n, seed, args):
    """The element families of the paper's conclusions: linear tetrahedra (the
    Kuhn split of the headline 128^3 grid, 12,582,912 tetrahedra, each with its
    hexahedron's coefficient), triquadratic hexahedra (a 64^3-element box,
    2,146,689 nodes, coefficient layered per 2 cells) and tricubic hexahedra
    (a 42^3-element box, 2,048,383 nodes, layered per cell): FP64 and FP32 applies of
    scalar Laplace, FP64 elasticity applies, and Jacobi-PCG to 1e-8 with
    Dirichlet u = 0 on z = 0."""
    import numpy as np
    import torch
    res = {}

    def up(a, dt=None):
        return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=dt)

    def make(elem, physics, dtype, xyz, conn, coef, mask=None):
        t = torch.float64 if dtype == 0 else torch.float32
        return q1.q1_op_create_elem(elem, physics, dtype, 0, up(xyz, t), up(conn.astype(np.int32)),
                                    up(coef, t), up(mask.astype(np.uint8)) if mask is not None
                                    else None)

    for elem, tag in ((q1.Q1_TET4, "tet"), (q1.Q1_HEX27, "q2"), (q1.Q1_HEX64, "q3")):
        if elem == q1.Q1_TET4:
            m = n
            xyz, conn = si.tet_mesh(m, m, m)
            k = np.repeat(si.field_layered(m, m, m, 4, 1.5, 0.5, seed), 6)[None]
            me = n // 2
            xyz_e, conn_e = si.tet_mesh(me, me, me)
            mask_e = si.face_mask(me, me, me, "z0")
        elif elem == q1.Q1_HEX27:
            m = n // 2
            xyz, conn = si.q2_box_mesh(m, m, m)
            k = si.field_layered(m, m, m, 2, 1.5, 0.5, seed)[None]
            me = n // 4
            xyz_e, conn_e = si.q2_box_mesh(me, me, me)
            mask_e = si.q2_face_mask(me, me, me, "z0")
        else:
            m = n // 3
            xyz, conn = si.q3_box_mesh(m, m, m)
            k = si.field_layered(m, m, m, 1, 1.5, 0.5, seed)[None]
            me = n // 6
            xyz_e, conn_e = si.q3_box_mesh(me, me, me)
            mask_e = si.q3_face_mask(me, me, me, "z0")
        nn = xyz.shape[1]
        for dt, dtag in ((0, "fp64"), (1, "fp32")):
            op = make(elem, 1, dt, xyz, conn, k)
            t = torch.float64 if dt == 0 else torch.float32
            x = up(si.vec_uniform(nn, seed, si.STREAM_X), t)
            y = torch.empty_like(x)
            ms, _ = time_applies(op, x, y, 200, 20)
            b, f = op.bytes()
            res[f"{tag}_laplace_{dtag}_gdofs"] = round(nn / (ms * 1e-3) / 1e9, 3)
            res[f"{tag}_laplace_{dtag}_us"] = round(1e3 * ms, 2)
            res[f"{tag}_laplace_{dtag}_hbm_frac"] = round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            if dt == 0:
                res[f"{tag}_laplace_fp64_flop_frac"] = round(f / (ms * 1e-3) / 1e12 / FP64_PEAK_TFS, 4)
                res[f"{tag}_laplace_n_elems"] = conn.shape[1]
                res[f"{tag}_laplace_n_dof"] = nn
            op.destroy()
        # elasticity apply and Jacobi-PCG on the smaller grid
        ne_e = conn_e.shape[1]
        E, nu = si.field_elastic(ne_e, seed)
        coef_e = np.stack(si.lame_from_E_nu(E, nu))
        op = make(elem, 3, 0, xyz_e, conn_e, coef_e, mask_e)
        nd = 3 * xyz_e.shape[1]
        x = up(si.vec_uniform(nd, seed, si.STREAM_X))
        y = torch.empty_like(x)
        ms, _ = time_applies(op, x, y, 200, 20)
        res[f"{tag}_elasticity_fp64_gdofs"] = round(nd / (ms * 1e-3) / 1e9, 3)
        res[f"{tag}_elasticity_n_dof"] = nd
        op.destroy()
        kp = si.field_lognormal(conn_e.shape[1], 0.0, 1.0, seed)[None]
        op = make(elem, 1, 0, xyz_e, conn_e, kp, mask_e)
        bb = si.vec_uniform(xyz_e.shape[1], seed, si.STREAM_RHS)
        bb[mask_e == 1] = 0.0
        bd = up(bb)
        xd = torch.empty_like(bd)
        q1.q1_pcg(op, 1, bd, xd, 1e-8, 5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = q1.q1_pcg(op, 1, bd, xd, 1e-8, 50000)
        tp = time.perf_counter() - t0
        res[f"{tag}_pcg_s"] = round(tp, 4)
        res[f"{tag}_pcg_iters"] = st["iters"]
        res[f"{tag}_pcg_true_rel_res"] = st["true_rel_res"]
        res[f"{tag}_pcg_n_dof"] = int(xyz_e.shape[1])
        op.destroy()
    torch.cuda.synchronize()
    return res


class _DotOp:
    """q1_dot behind the apply(x, y, stream) interface of the timing helpers."""

    def __init__(self, q1, a, b, out, variant, nb, work):
        self.q1, self.a, self.b, self.out, self.v, self.nb, self.w = q1, a, b, out, variant, nb, work

    def apply(self, _x, _y, stream=None):
        self.q1.q1_dot(self.a, self.b, self.out, self.v, self.nb, self.w, stream)


def bench_ir96(q1, si, n, seed, args):
    """96^3 elasticity, Dirichlet on z=0, random body force: FP64 Jacobi-PCG vs
    FP32-apply iterative refinement with FP64 residuals and vs mixed-precision
    PCG with reliable updates, all to 1e-10."""
    import torch
    s2 = si.seed_for(2)
    pr = si.problem_elasticity(96, s2)
    nn = pr["xyz"].shape[1]
    b = si.vec_uniform(3 * nn, s2, si.STREAM_RHS)
    b[si.dof_mask(pr["mask"], 3) == 1] = 0.0
    op64 = q1.q1_op_create(3, 0, 0, *upload(pr, 0))
    op32 = q1.q1_op_create(3, 1, 0, *upload(pr, 1))
    bd = torch.from_numpy(b).to("cuda")
    xd = torch.empty_like(bd)
    t0 = time.perf_counter()
    st64 = q1.q1_pcg(op64, 1, bd, xd, 1e-10, 50000)
    t64 = time.perf_counter() - t0
    t0 = time.perf_counter()
    sti = q1.q1_ir_solve(op64, op32, bd, xd, 1e-10, 1e-4)
    tir = time.perf_counter() - t0
    t0 = time.perf_counter()
    stm = q1.q1_mpcg(op64, op32, bd, xd, 1e-10, 0.1, 50000)
    tmp = time.perf_counter() - t0
    x32 = torch.empty(3 * nn, dtype=torch.float32, device="cuda")
    y32 = torch.empty_like(x32)
    ms32, _ = time_applies(op32, x32, y32, 50, 5)
    xx = torch.empty(3 * nn, dtype=torch.float64, device="cuda")
    yy = torch.empty_like(xx)
    ms64, _ = time_applies(op64, xx, yy, 50, 5)
    b64, f64 = op64.bytes()
    # the general-hexahedron instance: the same problem on the jittered grid
    prj = dict(pr)
    prj["xyz"], _ = si.box_mesh(96, 96, 96, 1.0, 0.1, s2)
    opj = q1.q1_op_create(3, 0, 0, *upload(prj, 0))
    msj, _ = time_applies(opj, xx, yy, 50, 5)
    opj.destroy()
    # partial assembly (scaled adjugate stored per point) against the matrix-free apply
    pa = {}
    for dt, tag, xv, yv in ((0, "fp64", xx, yy), (1, "fp32", x32, y32)):
        oppa = q1.q1_op_create(3, dt, 6, *upload(pr, dt))
        mspa, _ = time_applies(oppa, xv, yv, 50, 5)
        bpa, _ = oppa.bytes()
        pa[f"el96_pa_{tag}_gdofs"] = round(3 * nn / (mspa * 1e-3) / 1e9, 3)
        pa[f"el96_pa_{tag}_hbm_frac"] = round(bpa / (mspa * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        pa[f"el96_pa_{tag}_alg_bytes"] = bpa
        oppa.destroy()
    op64.destroy()
    op32.destroy()
    return {**pa, "el96_apply_fp64_hbm_frac": round(b64 / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "el96_jittered_fp64_gdofs": round(3 * nn / (msj * 1e-3) / 1e9, 3),
            "el96_jittered_fp64_flop_frac": round(f64 / (msj * 1e-3) / 1e12 / FP64_PEAK_TFS, 4),
            "el96_pcg64_s": round(t64, 4), "el96_pcg64_iters": st64["iters"],
            "el96_pcg64_status": st64["status"], "el96_pcg64_true_rel_res": st64["true_rel_res"],
            "el96_ir_s": round(tir, 4), "el96_ir_inner_iters": sti["iters"],
            "el96_ir_outer": sti["outer_iters"], "el96_ir_status": sti["status"],
            "el96_ir_rel_res": sti["rel_res"],
            "el96_mpcg_s": round(tmp, 4), "el96_mpcg_iters": stm["iters"],
            "el96_mpcg_refreshes": stm["outer_iters"], "el96_mpcg_status": stm["status"],
            "el96_mpcg_true_rel_res": stm["true_rel_res"],
            "el96_apply_fp64_gdofs": round(3 * nn / (ms64 * 1e-3) / 1e9, 3),
            "el96_apply_fp32_gdofs": round(3 * nn / (ms32 * 1e-3) / 1e9, 3)}


def bench_vlap96(q1, si, n, seed, args):
    """96^3 vector Laplace (3 DOF per node, k = exp(N(0,1)) iid, Dirichlet on z=0):
    FP64 and FP32 applies of the default variant, and FP64 Jacobi-PCG to 1e-8."""
    import torch
    s5 = si.seed_for(5)
    pr = si.problem_vlaplace(96, s5)
    nn = pr["xyz"].shape[1]
    res = {}
    for dt, tag in ((0, "fp64"), (1, "fp32")):
        op = q1.q1_op_create(2, dt, 0, *upload(pr, dt))
        t = torch.float64 if dt == 0 else torch.float32
        x = torch.from_numpy(si.vec_uniform(3 * nn, s5, si.STREAM_X)).to("cuda", dtype=t)
        y = torch.empty_like(x)
        ms, _ = time_applies(op, x, y, 100, 10)
        alg, _ = op.bytes()
        res[f"vlap96_apply_{tag}_gdofs"] = round(3 * nn / (ms * 1e-3) / 1e9, 3)
        res[f"vlap96_apply_{tag}_hbm_frac"] = round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        if dt == 0:
            b = si.vec_uniform(3 * nn, s5, si.STREAM_RHS)
            b[si.dof_mask(pr["mask"], 3) == 1] = 0.0
            bd = torch.from_numpy(b).to("cuda")
            xd = torch.empty_like(bd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = q1.q1_pcg(op, 1, bd, xd, 1e-8, 50000)
            res["vlap96_pcg64_s"] = round(time.perf_counter() - t0, 4)
            res["vlap96_pcg64_iters"] = st["iters"]
            res["vlap96_pcg64_true_rel_res"] = st["true_rel_res"]
        torch.cuda.synchronize()
        op.destroy()
    return res


def bench_batched(q1, si, n, seed, args):
    """32 scalar-Laplace problems with edges U{16..64}, k = exp(N(0,1)) iid,
    Dirichlet on z=0, 4 right-hand sides each: one persistent launch for all
    128 solves to 1e-8, against the same solves looped through q1_pcg."""
    import torch
    s3 = si.seed_for(3)
    sizes = si.batch_sizes(32, s3)
    ops, bd, xd, ndof = [], [], [], 0
    for i, m in enumerate(sizes):
        m = int(m)
        xyz, conn = si.box_mesh(m, m, m, 1.0, 0.0, s3 + 1000 * i)
        k = si.field_lognormal(m ** 3, 0.0, 1.0, s3 + 1000 * i)[None]
        mask = si.face_mask(m, m, m, "z0")
        pr = dict(xyz=xyz, conn=conn, coef=k, mask=mask)
        ops.append(q1.q1_op_create(1, 0, 3, *upload(pr, 0)))  # one-wave tiles
        nn = xyz.shape[1]
        ndof += nn
        row = []
        allb = si.vec_uniform(4 * nn, s3 + 2000 * i, si.STREAM_RHS)
        for c in range(4):
            b = allb[c * nn:(c + 1) * nn].copy()
            b[mask == 1] = 0.0
            row.append(torch.from_numpy(b).to("cuda"))
        bd.append(row)
        xd.append([torch.empty_like(b) for b in row])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = q1.q1_batched_pcg(ops, bd, xd, 1e-8, 20000)
    t_batched = time.perf_counter() - t0
    iters = sum(s_["iters"] for s_ in st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stm = q1.q1_batched_mpcg(ops, bd, xd, 1e-8, 20000, 0.1)
    t_mixed = time.perf_counter() - t0
    t0 = time.perf_counter()
    it_loop = 0
    for i in range(32):
        for c in range(4):
            it_loop += q1.q1_pcg(ops[i], 1, bd[i][c], xd[i][c], 1e-8, 20000)["iters"]
    t_loop = time.perf_counter() - t0
    torch.cuda.synchronize()
    for o in ops:
        o.destroy()
    return {"batched_s": round(t_batched, 4), "batched_kernel_s": round(st[0]["seconds"], 4),
            "batched_loop_pcg_s": round(t_loop, 4), "batched_total_iters": iters,
            "batched_loop_iters": it_loop, "batched_ndof_x4": 4 * ndof,
            "batched_all_converged": all(s_["status"] == 0 for s_ in st),
            "batched_gdofs": round(4 * ndof * iters / 128 / st[0]["seconds"] / 1e9, 3),
            "batched_mixed_s": round(t_mixed, 4),
            "batched_mixed_kernel_s": round(stm[0]["seconds"], 4),
            "batched_mixed_total_iters": sum(s_["iters"] for s_ in stm),
            "batched_mixed_refreshes": sum(s_["outer_iters"] for s_ in stm),
            "batched_mixed_all_converged": all(s_["status"] == 0 for s_ in stm),
            "batched_mixed_max_true_rel_res": max(s_["rel_res"] for s_ in stm)}


# the network's 3x3x3 convolutions: (real input channels, output channels, level);
# level l runs on the grid divided by 2^(l-1)
UNET_CONVS = [(2, 16, 1), (16, 16, 1), (16, 32, 2), (32, 32, 2), (32, 64, 3), (64, 64, 3),
              (96, 32, 2), (32, 32, 2), (48, 16, 1), (16, 16, 1)]


def unet_forward_flops(D: int, H: int, W: int) -> float:
    """Algorithmic FLOPs of one network forward on a D x H x W grid: 2 * 27 * Cin * Cout per
    voxel and convolution (real input channels), plus the 1x1 head."""
    f = 0.0
    for ci, co, lvl in UNET_CONVS:
        s = 2 ** (lvl - 1)
        f += 2.0 * 27 * ci * co * (D // s) * (H // s) * (W // s)
    return f + 2.0 * 16 * D * H * W


def bench_learned(q1, si, n, seed, args):
    """Learned preconditioner on 64^3 scalar Laplace, k = exp(N(0, 2^2)) iid,
    Dirichlet on z=0: harvest Jacobi-PCG trajectories, train the U-Net on the
    GPU (time reported separately), then flexible PCG with the two-level
    learned preconditioner against FP64 Jacobi-PCG to 1e-8 on held-out fields,
    every inference inside the timed solve."""
    import torch
    from paper_2308_09839_amd import learned as Lm
    n4 = 64
    G = Lm.grid_for(n4)
    B = 4
    net = q1.UNet(G, G, G, B, seed=si.seed_for(4))
    # forward / backward timing (HIP events on the current stream)
    inp = torch.zeros((B, G, G, G, 8), dtype=torch.bfloat16, device="cuda")
    out = torch.empty((B, G, G, G), dtype=torch.float32, device="cuda")
    res = {}
    for nb in (1, B):
        for _ in range(3):
            net.forward(inp, out, nb)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            net.forward(inp, out, nb)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        res[f"nn_forward_b{nb}_ms"] = round(ms, 4)
        res[f"nn_forward_b{nb}_tflops"] = round(nb * unet_forward_flops(G, G, G) / (ms * 1e-3) / 1e12, 2)
    dout = torch.zeros_like(out)
    net.forward(inp, out, B)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        net.forward(inp, out, B)
        net.backward(dout)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    res["nn_train_step_b4_ms"] = round(ms, 3)
    res["nn_train_step_b4_tflops"] = round(3 * B * unet_forward_flops(G, G, G) / (ms * 1e-3) / 1e12, 2)
    quiet = lambda m: log(m)
    data = Lm.harvest(n4, [Lm.TRAIN_SEED0 + j for j in range(args.nn_fields)], args.nn_per_field,
                      log=quiet)
    tr = Lm.Trainer(net, data, B, seed=1)
    hist, t_train = tr.train(args.nn_steps, lr=1e-3, log=quiet, log_every=500)
    periods = (1, 4, 16, 64)
    per = Lm.choose_period(net, n4, periods, nval=2, trunc_m=8, log=quiet)
    rows = Lm.evaluate(net, n4, [Lm.EVAL_SEED0 + j for j in range(args.nn_eval)], omega=0.6,
                       trunc_m=8, periods=sorted({1, per}), smoothing_baseline=True, log=quiet)
    # FCG(1) (the flexible PCG beta alone) against FCG(8), the network on every call
    rows1 = Lm.evaluate(net, n4, [Lm.EVAL_SEED0 + j for j in range(min(2, args.nn_eval))],
                        omega=0.6, trunc_m=1, periods=(1,), log=quiet)
    jt = sum(r["jacobi_s"] for r in rows) / len(rows)
    nt = sum(r["periods"][per]["nn_s"] for r in rows) / len(rows)
    n1 = sum(r["periods"][1]["nn_s"] for r in rows) / len(rows)
    res.update({"nn_pairs": int(data["r"].shape[0]), "nn_train_fields": args.nn_fields,
                "nn_train_steps": args.nn_steps,
                "nn_train_s": round(t_train, 2), "nn_loss_first": hist[0][1],
                "nn_loss_last": hist[-1][1], "nn_eval_fields": len(rows),
                "nn_schedule_period": per,
                "nn_eval_jacobi_iters": [r["jacobi_iters"] for r in rows],
                "nn_eval_fcg_iters": [r["periods"][per]["nn_iters"] for r in rows],
                "nn_eval_smoothing_only_iters": [r["periods"][per]["smoothing_iters"] for r in rows],
                "nn_eval_fcg_every_call_iters": [r["periods"][1]["nn_iters"] for r in rows],
                "nn_eval_jacobi_ms": [round(r["jacobi_s"] * 1e3, 2) for r in rows],
                "nn_eval_fcg_ms": [round(r["periods"][per]["nn_s"] * 1e3, 2) for r in rows],
                "nn_eval_fcg_every_call_ms": round(n1 * 1e3, 2),
                "nn_eval_fcg1_every_call_iters": [r["periods"][1]["nn_iters"] for r in rows1],
                "nn_eval_fcg1_every_call_ms": [round(r["periods"][1]["nn_s"] * 1e3, 2)
                                               for r in rows1],
                "nn_eval_fcg8_every_call_iters_same_fields":
                    [r["periods"][1]["nn_iters"] for r in rows[:len(rows1)]],
                "nn_eval_fcg_true_rel_res": max(r["periods"][per]["nn_true_rel_res"] for r in rows),
                "nn_eval_fallback_at": [r["periods"][per]["nn_fallback_at"] for r in rows],
                "nn_wall_speedup_vs_jacobi": round(jt / nt, 3)})
    del data
    torch.cuda.synchronize()
    net.destroy()
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    # 1000 timed applies (about 40 ms) after 200 untimed ones: a shorter warm-up
    # leaves the first timed applies before the GPU's clocks have settled
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=128, help="elements per edge")
    ap.add_argument("--variant", type=int, default=0, help="0 auto, 1 atomic, 3 LDS tile")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip FP32/jittered/cold extras")
    ap.add_argument("--only-extras", action="store_true",
                    help="skip the cold, variant, FP32 and jittered applies (run the headline "
                         "and the solver extras named by --extras only; for profiling a leg)")
    ap.add_argument("--extras", default="all",
                    help="comma-separated solver extras to run (csr, cg16, cg128, "
                         "cg_elasticity96, vlaplace96, family, learned64, batched32) or 'all'")
    ap.add_argument("--nn-fields", type=int, default=500, help="training fields of the learned leg")
    ap.add_argument("--nn-per-field", type=int, default=40, help="pairs per training field")
    ap.add_argument("--nn-steps", type=int, default=3000, help="Adam steps of the learned leg")
    ap.add_argument("--nn-eval", type=int, default=8, help="held-out fields of the learned leg")
    ap.add_argument("--copy-ref-mb", type=int, default=0,
                    help="also run one plain device copy of this many MB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the operator is single-device by design "
              "(multi-GPU sharding is described, not built); run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch

    import paper_2308_09839_amd as q1
    import seeded_inputs as si

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    seed = si.seed_for(1)
    n = args.n
    log(f"[bench] building {n}^3 layered-coefficient Laplace inputs")
    pr = si.problem_laplace_layered(n, seed)
    nn = pr["xyz"].shape[1]
    ndof = nn

    def make(pr_, dtype):
        xyz, conn, coef, mask = upload(pr_, dtype)
        op = q1.q1_op_create(1, dtype, args.variant, xyz, conn, coef, mask)
        t = torch.float64 if dtype == 0 else torch.float32
        x = torch.from_numpy(si.vec_uniform(nn, seed, si.STREAM_X)).to("cuda", dtype=t)
        y = torch.empty_like(x)
        return op, x, y

    if args.copy_ref_mb > 0:
        a = torch.ones(args.copy_ref_mb * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    copies = [make(pr, 0) for _ in range(ROTATE)]
    op, x, y = copies[0]
    info = op.info()
    alg_bytes, alg_flops = op.bytes()
    # untimed applies for about 60 ms first, so that the timed ones (and the warm-up the
    # command line asks for) run at settled clocks even when K and W are small
    for i in range(1500):
        c = copies[i % ROTATE]
        c[0].apply(c[1], c[2])
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} FP64 applies rotating over {ROTATE} copies "
        f"(variant {info['variant']})")
    ms = time_rotating(copies, args.steps, args.warmup)
    gdofs = ndof / (ms * 1e-3) / 1e9
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    extras = {}
    ms_warm, _ = time_applies(op, x, y, args.steps, args.warmup)
    extras["fp64_warm_gdofs"] = round(ndof / (ms_warm * 1e-3) / 1e9, 3)
    extras["fp64_warm_ms"] = round(ms_warm, 5)
    extras["fp64_warm_hbm_frac"] = round(alg_bytes / (ms_warm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    for c in copies[1:]:
        c[0].destroy()
    del copies
    if not args.no_extras and args.only_extras:
        op.destroy()
        del op, x, y
    elif not args.no_extras:
        log("[bench] cold (flushed) applies")
        ms_cold = time_cold(op, x, y, 100)
        extras["fp64_cold_write_flush_gdofs"] = round(ndof / (ms_cold * 1e-3) / 1e9, 3)
        extras["fp64_cold_write_flush_ms"] = round(ms_cold, 5)
        extras["fp64_cold_write_flush_hbm_frac"] = round(
            alg_bytes / (ms_cold * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        ms_cold_r = time_cold(op, x, y, 100, "read")
        extras["fp64_cold_read_flush_gdofs"] = round(ndof / (ms_cold_r * 1e-3) / 1e9, 3)
        extras["fp64_cold_read_flush_ms"] = round(ms_cold_r, 5)
        extras["fp64_cold_read_flush_hbm_frac"] = round(alg_bytes / (ms_cold_r * 1e-3) / 1e9 /
                                                        HBM_PEAK_GBS, 4)
        for v in (1, 2, 3, 5, 6):
            if v == info["variant"]:
                continue
            opv = q1.q1_op_create(1, 0, v, *upload(pr, 0))
            msv, _ = time_applies(opv, x, y, args.steps, args.warmup)
            extras[f"fp64_variant{v}_gdofs"] = round(ndof / (msv * 1e-3) / 1e9, 3)
            if v == 6:  # partial assembly: its own (Table 3) bytes
                bv, _ = opv.bytes()
                extras["fp64_pa_hbm_frac"] = round(bv / (msv * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                extras["fp64_pa_alg_bytes"] = bv
            opv.destroy()
        op.destroy()
        del op, x, y
        log("[bench] FP32 applies")
        copies = [make(pr, 1) for _ in range(ROTATE)]
        ms32 = time_rotating(copies, args.steps, args.warmup)
        b32, _ = copies[0][0].bytes()
        extras["fp32_gdofs"] = round(ndof / (ms32 * 1e-3) / 1e9, 3)
        extras["fp32_ms"] = round(ms32, 5)
        extras["fp32_hbm_frac"] = round(b32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        ms32w, _ = time_applies(*copies[0], args.steps, args.warmup)
        extras["fp32_warm_gdofs"] = round(ndof / (ms32w * 1e-3) / 1e9, 3)
        for c in copies:
            c[0].destroy()
        del copies
        log("[bench] jittered (general-hexahedron) FP64 applies")
        prj = dict(pr)
        prj["xyz"], _ = si.box_mesh(n, n, n, 1.0, 0.1, seed)
        copies = [make(prj, 0) for _ in range(ROTATE)]
        msj = time_rotating(copies, args.steps, args.warmup)
        extras["fp64_jittered_gdofs"] = round(ndof / (msj * 1e-3) / 1e9, 3)
        extras["fp64_jittered_ms"] = round(msj, 5)
        extras["fp64_jittered_flop_frac"] = round(alg_flops / (msj * 1e-3) / 1e12 / FP64_PEAK_TFS, 4)
        extras["fp64_jittered_hbm_frac"] = round(alg_bytes / (msj * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        for c in copies:
            c[0].destroy()
        del copies
    else:
        op.destroy()
    if not args.no_extras:
        torch.cuda.synchronize()
        for name, fn in (("csr", bench_csr), ("cg16", bench_cg16), ("cg128", bench_cg128),
                         ("cg_elasticity96", bench_ir96), ("vlaplace96", bench_vlap96),
                         ("family", bench_family), ("learned64", bench_learned),
                         ("batched32", bench_batched)):
            if args.extras != "all" and name not in args.extras.split(","):
                continue
            try:
                log(f"[bench] {name}")
                extras.update(fn(q1, si, n, seed, args))
            except Exception as exc:  # an extra must not take down the headline line
                log(f"[bench] {name} failed: {exc!r}")
                extras[f"{name}_error"] = repr(exc)
            torch.cuda.synchronize()
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(n, seed)
    torch.cuda.synchronize()
    traffic = MEASURED_TRAFFIC.get((kernel_hash(), n)) if info["variant"] == 5 else None
    # the library takes owner-computes tiles for this workload (a box lattice of
    # parallelepipeds with n a multiple of 16) unless Q1_OWNER_TILE=0
    owner = info["variant"] == 5 and n % 16 == 0 and os.environ.get("Q1_OWNER_TILE") != "0"
    kernel = ("k_apply_owner (one kernel per apply)" if owner
              else "k_apply_block + k_halo_sum (one apply)")
    out = {
        "metric": "GDOF/s per matrix-free apply",
        "value": round(gdofs, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"scalar Laplace Q1, {n}^3 undistorted hexahedra "
                               f"({ndof} DOF; every element a parallelepiped, so the exact "
                               "constant-Jacobian element path), layered lognormal "
                               "coefficient, FP64 matrix-free apply (owner-computes tiles: "
                               "each workgroup writes the 16x8x4 nodes it owns); the timed "
                               "applies rotate "
                               f"over {ROTATE} resident copies so each streams from HBM",
                   "n_elems": n ** 3, "n_dof": ndof, "variant": info["variant"],
                   "element_path": "parallelepiped"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": kernel,
                     "algorithmic_bytes_per_apply": alg_bytes,
                     "warm_frac": extras.get("fp64_warm_hbm_frac"),
                     "cold_frac_read_flush": extras.get("fp64_cold_read_flush_hbm_frac"),
                     "cold_frac_write_flush": extras.get("fp64_cold_write_flush_hbm_frac")},
        "cpu_baseline": cpu,
        "extra": extras,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
