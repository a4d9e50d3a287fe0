"""Throughput of the block-based spectral hot path on one MI355X.

Headline workload (batched uneven blocks): 1,024 independent submeshes, each a
seeded Delaunay-triangulated disk of U{500..5000} vertices (2.82M vertices in
all), combinatorial Laplacian, tracked width p_b = min(320, n_b), kept pairs
up to c_max = 256, cold seeded starts (the library's MI_RANDOM generator),
FP32 slabs with FP64 Gram sums and FP64 small solves; all blocks in one wave.

One step = eigenspace tracking of every block (one HIP graph replay of the
wave's launches) + the choice of c per block for the calibrated NMSVE target
(Section 5, Eq. 16) + projection of the xyz coordinates onto the first c_b
Ritz vectors + reconstruction.  The Laplacians (combinatorial, and the 1/d
one of the NMSVE's GL operator) are built once, outside the step, and timed
separately.  A seeded sample of blocks is checked against the FP64 oracle
before the timed region (principal angle <= 1e-5).

A secondary line covers the static block sequence (displaced level-7
icosphere, 100 blocks warm-started along a BFS order of the blocks, c = 100,
p = 192) and the extras measured on it (merge, codec, quality, dynamic walk,
R^z); a third covers the 1M-vertex precision workload with FP32 and with
BF16 working slabs.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--no-secondary] [--no-precision] [--only-precision]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the static block sequence and its extras")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 1M-vertex FP32 / BF16 precision leg")
    ap.add_argument("--only-precision", action="store_true",
                    help="run the 1M-vertex precision leg alone (for profilers)")
    ap.add_argument("--cpu-sample-blocks", type=int, default=60)
    ap.add_argument("--parity-blocks", type=int, default=8,
                    help="sampled disks checked against the oracle before timing")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + a few steps only (for profilers)")
    ap.add_argument("--traffic-calib", action="store_true",
                    help="first copy 256 MiB once (a plain copy kernel of known size: "
                         "the scale of the HBM byte counters)")
    return ap.parse_args()


def merge_run(mis, ctx, W, dev, reps):
    """Degree-weighted merge of overlapped submeshes (Section 6.1, Alg. 3) on
    the same level-7 icosphere cut into 100 parts extended by 15 % to equal
    size, with the block coordinates standing in for the reconstructions.
    Timed with events around `reps` calls after a first call that builds the
    occurrence table.  Algorithmic bytes: per occurrence the coordinates
    (12 B), two row pointers (8 B) and the occurrence entry (8 B); per vertex
    the occurrence offset (8 B) and the output (12 B)."""
    import torch
    t0 = time.time()
    bs = W.icosphere_overlapped(level=7, n_blocks=100, c=100, p=192, overlap=0.15)
    fl = W.flatten(bs)
    blocks = mis.Blocks(bs.n, p=fl["p"], ld=fl["ld"], pred=bs.pred)
    prims = torch.from_numpy(np.ascontiguousarray(fl["prims"].reshape(-1))).to(dev)
    coords = torch.from_numpy(np.ascontiguousarray(fl["coords"].reshape(-1))).to(dev)
    gid = np.concatenate(bs.global_ids).astype(np.int32)
    L = mis.build_laplacian(ctx, blocks, fl["prim_off"], prims, 3, coords, mis.MI_W_COMBINATORIAL)
    Xout = torch.empty(bs.n_global * 3, dtype=torch.float32, device=dev)
    mis.merge_overlapped(ctx, blocks, gid, bs.n_global, L, coords, Xout)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        mis.merge_overlapped(ctx, blocks, gid, bs.n_global, L, coords, Xout)
    e1.record()
    torch.cuda.synchronize()
    call_ms = e0.elapsed_time(e1) / reps  # includes the host side of each call
    # the kernel alone: the library's event timer brackets each launch
    ctx.set_timing(True)
    for _ in range(reps):
        mis.merge_overlapped(ctx, blocks, gid, bs.n_global, L, coords, Xout)
    torch.cuda.synchronize()
    kt_ms, kt_n = ctx.kernel_times()["merge"]
    ctx.set_timing(False)
    ms = kt_ms / max(kt_n, 1)
    nocc, nv = int(gid.size), int(bs.n_global)
    nbytes = 28 * nocc + 20 * nv
    exact = bool(torch.equal(Xout.view(-1, 3).cpu(),
                             torch.from_numpy(bs.extra["verts_global"].astype(np.float32))))
    return {"workload": "icosphere7_100parts_overlap15", "vertices": nv, "occurrences": nocc,
            "n_d": int(bs.extra["n_d"]), "kernel_ms": ms, "call_ms": call_ms,
            "vertices_per_s": nv / (ms * 1e-3),
            "bytes_per_launch": nbytes, "achieved_GBps": nbytes / (ms * 1e-3) / 1e9,
            "frac_hbm": nbytes / (ms * 1e-3) / 1e9 / 8000.0, "equal_inputs_exact": exact,
            "setup_s": gen_s}


def doi_run(mis, ctx, blocks, L, coords, V0, dev, reps):
    """The dynamic walk of Alg. 2 on the step's blocks (not part of the step):
    start sizes 80, band [0.045, 0.065] of the Eq. 6 residual, c_max 190,
    at most 60 iterations per block; the same filter as the step.  Time per
    walk (eager launches) and the sizes it reaches."""
    import torch
    prm = mis.OiParams(precision=mis.MI_FP32, warm=mis.MI_WARM_PRED, m=10, passes=2, m0=10,
                       passes0=2, adapt=1, a_mode=mis.MI_A_WEYL, a_value=1.0)
    c0 = torch.full((blocks.n_blocks,), 80, dtype=torch.int32, device=dev)
    args = (ctx, blocks, L, prm, coords, c0, 0.045, 0.065, 190, 60)
    r = mis.doi_track(*args, V0=V0)  # plan
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        r = mis.doi_track(*args, V0=V0)
    e1.record()
    torch.cuda.synchronize()
    c = r.c.cpu().numpy()
    its = r.iters.cpu().numpy()
    return {"workload": "icosphere7_100blocks, c0=80, band [0.045, 0.065], c_max=190, t_max=60",
            "walk_ms": e0.elapsed_time(e1) / reps, "iters_mean": float(its.mean()),
            "iters_max": int(its.max()), "c_mean": float(c.mean()), "c_min": int(c.min()),
            "c_max": int(c.max()), "status_nonzero": int((r.status.cpu().numpy() != 0).sum())}


def rz_run(mis, ctx, blocks, L, V0, dev, reps):
    """The step's tracking with the paper's operator R^z = (L + 1e-3 I)^-1
    (z = 1, 60 conjugate-gradient iterations per solve, one solve per
    iteration, T = 3 / 5 as in the step) in place of the Chebyshev filter:
    time per tracking call and the largest Ritz residual of the kept pairs
    relative to the block's largest kept Ritz value (the library's own
    measure)."""
    import torch
    prm = mis.OiParams(precision=mis.MI_FP32, warm=mis.MI_WARM_PRED, T=3, T0=5, m=1, m0=1,
                       passes=1, passes0=1, adapt=0, op=mis.MI_OP_RZ, z=1, cg_iters=60,
                       delta=1e-3)
    V = torch.empty(int(blocks.u_off[-1]), dtype=torch.float32, device=dev)
    ritz = torch.zeros(int(blocks.t_off[-1]), dtype=torch.float64, device=dev)
    st = torch.zeros(blocks.n_blocks, dtype=torch.int32, device=dev)
    mis.oi_track(ctx, blocks, L, prm, V0=V0, V=V, ritz=ritz, status=st)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        mis.oi_track(ctx, blocks, L, prm, V0=V0, V=V, ritz=ritz, status=st)
    e1.record()
    torch.cuda.synchronize()
    res = mis.ritz_residuals(ctx, blocks, L, V, ritz).cpu().numpy()
    th = ritz.cpu().numpy()
    worst = 0.0
    for b in range(blocks.n_blocks):
        t0 = int(blocks.t_off[b])
        worst = max(worst, float(res[t0:t0 + 100].max() / max(th[t0 + 99], 1e-30)))
    return {"workload": "icosphere7_100blocks_c100, R^z with z=1, delta=1e-3, 60 CG iterations",
            "ms_per_step": e0.elapsed_time(e1) / reps, "max_rel_ritz_residual_c100": worst,
            "status_nonzero": int((st.cpu().numpy() != 0).sum())}


def quality_run(mis, ctx, bs, blocks, L, coords, Xr, Xq, dev, reps):
    """Section 8 quality of the step's reconstruction on the whole mesh: the
    blocks' reconstructions placed at their mesh vertices (the merge, with
    one occurrence per vertex for disjoint blocks), then NMSVE in dB and the
    mean face-normal angle, for the FP32 coefficients and their 12-bit codes."""
    import torch
    gid = np.concatenate(bs.global_ids).astype(np.int32)
    nv = int(bs.n_global)
    Xg = mis.merge_overlapped(ctx, blocks, gid, nv, L, coords)  # the original mesh
    Xm = mis.merge_overlapped(ctx, blocks, gid, nv, L, Xr)
    Xmq = mis.merge_overlapped(ctx, blocks, gid, nv, L, Xq)
    faces = torch.from_numpy(np.ascontiguousarray(
        bs.extra["faces_global"].astype(np.int32).reshape(-1))).to(dev)
    Lm = mis.mesh_laplacian(ctx, nv, faces)
    q32 = mis.mesh_quality(ctx, nv, Lm.row_ptr, Lm.col, faces, Xg, Xm)
    q12 = mis.mesh_quality(ctx, nv, Lm.row_ptr, Lm.col, faces, Xg, Xmq)
    ctx.set_timing(True)
    for _ in range(reps):
        mis.mesh_quality(ctx, nv, Lm.row_ptr, Lm.col, faces, Xg, Xm, out=q32)
    torch.cuda.synchronize()
    k_ms, k_n = ctx.kernel_times()["quality"]
    ctx.set_timing(False)
    a = dict(zip(mis.QUALITY_FIELDS, q32.cpu().numpy().tolist()))
    b = dict(zip(mis.QUALITY_FIELDS, q12.cpu().numpy().tolist()))
    return {"workload": "icosphere7 whole mesh, c=100 per block", "vertices": nv,
            "faces": int(faces.numel() // 3), "nmsve": a["nmsve"], "nmsve_db": a["nmsve_db"],
            "theta_deg": a["theta_deg"], "nmsve_db_12bit": b["nmsve_db"],
            "theta_deg_12bit": b["theta_deg"], "kernel_ms": k_ms / max(k_n, 1)}


SEED = 181002719          # master seed of the seeded start
# the fewest iterations meeting 1e-5 on all 1,024 disks against the oracle
# (worst angle 5.4e-6; degree 13 per pass leaves three disks above 1e-4)
C3_T0, C3_M0, C3_PASSES0 = 5, 12, 2
G_MIN = 1e-3              # relative gap the choice of c snaps to
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden")


def c3_target():
    """Calibrated NMSVE target of the disks (median of the oracle's NMSVE(c =
    128) over the seeded sample; the literal 1e-4 is met by no block)."""
    with open(os.path.join(GOLDEN, "c3_calibrated_target.txt")) as f:
        for line in f:
            if line.startswith("target "):
                return float(line.split()[1])
    raise RuntimeError("no target in c3_calibrated_target.txt")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def c3_oracle(bs, blocks, ids, target, V, Xr, c_gpu):
    """The FP64 oracle's whole method on the blocks ids (dense eigh of the p+1
    lowest pairs, the NMSVE curve for c = 1..c_max by explicit
    reconstructions, the choice of c, projection and reconstruction), timed;
    and the GPU step's result on the same blocks against it: principal angles
    at c_max and at the GPU's c, the reconstruction at the GPU's c, and
    whether both sides chose the same c."""
    from oracle import laplacian as lap
    from oracle import metrics as met
    from oracle import spectral as S
    Vh = None if V is None else V
    t, nv, rows = 0.0, 0, []
    for b in ids:
        b = int(b)
        n, pb, cm = int(blocks.n[b]), int(blocks.p[b]), int(bs.c[b])
        X = bs.coords[b].astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        e = lap.canonical_edges(bs.faces[b], n)
        lam, U = S.eigh_lowest(lap.laplacian_dense(n, e, np.ones(len(e))), pb + 1)
        curve = met.nmsve_curve_sparse(U, X, e, X, cm)
        co = met.choose_c(curve, lam, target, G_MIN)
        Xo = S.encode_decode(U[:, :co], X)
        t += time.perf_counter() - t0
        nv += n
        if Vh is None:
            continue
        ld = int(blocks.ld[b])
        Vb = Vh[int(blocks.u_off[b]):int(blocks.u_off[b + 1])].view(n, ld).double().cpu().numpy()
        cg = int(c_gpu[b])
        v0 = int(blocks.v_off[b])
        Xg = Xr[3 * v0:3 * (v0 + n)].view(n, 3).double().cpu().numpy()
        Xo_g = S.encode_decode(U[:, :cg], X)
        # a cut inside a near-tie cluster (relative gap below 1e-3) is checked
        # at the cluster's end: the subspace up to the tie is not determined
        # by FP32 data (the choice of c snaps cuts below c_max off near-ties)
        cut = cm
        while cut < pb - 1 and (lam[cut] - lam[cut - 1]) < 1e-3 * lam[cut]:
            cut += 1
        cut_c = cut if cg == cm else cg
        rows.append({"block": b, "n": n, "c_gpu": cg, "c_oracle": co,
                     "sin_angle_cmax": S.sin_theta_max(U[:, :cut], Vb[:, :cut]),
                     "cut_cmax": cut,
                     "sin_angle_c": S.sin_theta_max(U[:, :cut_c], Vb[:, :cut_c]),
                     "recon_rel_err": S.rel_error(Xg, Xo_g),
                     "gap_c": float(lam[cg] - lam[cg - 1]) if cg < lam.size else None,
                     "nmsve_oracle_at_c": float(curve[cg - 1])})
        del Xo
    return t, nv, rows


def c3_headline(args):
    import torch

    import paper_1810_02719_amd as mis
    from synth import workloads as W

    t0 = time.time()
    bs = W.disk_blocks()
    fl = W.flatten(bs)
    dev = "cuda:0"
    nb = bs.n_blocks
    blocks = mis.Blocks(bs.n, p=fl["p"], ld=fl["ld"])  # independent blocks: one wave
    prims = torch.from_numpy(np.ascontiguousarray(fl["prims"].reshape(-1))).to(dev)
    coords = torch.from_numpy(np.ascontiguousarray(fl["coords"].reshape(-1))).to(dev)
    gen_s = time.time() - t0
    target = c3_target()

    ctx = mis.Context(0)
    torch.cuda.synchronize()
    tl = time.time()
    L = mis.build_laplacian(ctx, blocks, fl["prim_off"], prims, 3, coords, mis.MI_W_COMBINATORIAL)
    GL = mis.build_laplacian(ctx, blocks, fl["prim_off"], prims, 3, coords, mis.MI_W_INV_DIST)
    torch.cuda.synchronize()
    lap_ms = (time.time() - tl) * 1e3

    prm = mis.OiParams(precision=mis.MI_FP32, warm=mis.MI_RANDOM, seed=SEED, T0=C3_T0, m0=C3_M0,
                       passes0=C3_PASSES0, adapt=1, a_mode=mis.MI_A_WEYL, a_value=1.0, autotune=1)
    V = torch.empty(int(blocks.u_off[-1]), dtype=torch.float32, device=dev)
    ritz = torch.zeros(int(blocks.t_off[-1]), dtype=torch.float64, device=dev)
    status = torch.zeros(nb, dtype=torch.int32, device=dev)
    cmax = torch.from_numpy(np.asarray(bs.c, np.int32)).to(dev)
    c = torch.empty(nb, dtype=torch.int32, device=dev)
    metric = torch.zeros(int(blocks.t_off[-1]), dtype=torch.float64, device=dev)
    E = torch.empty(int(blocks.t_off[-1]) * 3, dtype=torch.float32, device=dev)
    Xr = torch.empty(int(blocks.v_off[-1]) * 3, dtype=torch.float32, device=dev)

    def step(blk=blocks, lap=L, gl=GL, per_block=False, Vv=V, rz=ritz, st=status, cc=c,
             cm=cmax, mt=metric, ee=E, xr=Xr):
        mis.oi_track(ctx, blk, lap, prm, V=Vv, ritz=rz, status=st, per_block=per_block)
        mis.choose_c(ctx, blk, cm, target, G_MIN, Vv, rz, coords, gl, c_out=cc, metric=mt)
        mis.project(ctx, blk, cc, Vv, coords, E=ee)
        mis.reconstruct(ctx, blk, cc, Vv, ee, Xr=xr)

    if args.traffic_calib:
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tp = time.time()
    step()  # plan (autotuned launch shapes) and graph capture
    torch.cuda.synchronize()
    plan_s = time.time() - tp
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # a seeded sample of blocks against the oracle before the timed region;
    # the oracle's work on it is the CPU baseline
    parity, cpu = None, None
    if not args.profile_only:
        ids = W.sample_blocks(bs.n, k=max(args.parity_blocks - 2, 1))
        c_gpu = c.cpu().numpy()
        t_all, nv_all, rows = c3_oracle(bs, blocks, ids, target, V, Xr, c_gpu)
        worst = max(r["sin_angle_c"] for r in rows)
        parity = {"blocks": len(rows), "sin_angle_c_max": worst,
                  "sin_angle_cmax_max": max(r["sin_angle_cmax"] for r in rows),
                  "recon_rel_err_max": max(r["recon_rel_err"] for r in rows),
                  "c_agree": int(sum(r["c_gpu"] == r["c_oracle"] for r in rows)),
                  "per_block": rows}
        if worst > 1e-5 or parity["recon_rel_err_max"] > 1e-5:
            raise RuntimeError(f"sampled blocks miss the 1e-5 bar: {parity}")
        if not args.no_cpu_baseline:
            from threadpoolctl import threadpool_info, threadpool_limits
            threads = max([i.get("num_threads", 1) for i in threadpool_info()
                           if i.get("internal_api") in ("openblas", "mkl", "blis")] or [1])
            small = sorted(ids, key=lambda b: int(bs.n[b]))[:2]
            with threadpool_limits(limits=1):
                t_one, nv_one, _ = c3_oracle(bs, blocks, small, target, None, None, None)
            cpu = {"value": nv_all / t_all, "unit": "vertices/s", "cores": int(threads),
                   "kind": "oracle", "cpu_model": cpu_model(),
                   "sample": f"{len(ids)} of {nb} disks (seeded, incl. the smallest and the "
                             f"largest; {nv_all} vertices): FP64 eigh of the p+1 lowest pairs, "
                             f"NMSVE curve c = 1..256, choice of c, projection, reconstruction; "
                             f"{t_all:.1f} s",
                   "one_core": {"value": nv_one / t_one, "unit": "vertices/s", "cores": 1,
                                "sample": f"the 2 smallest of those disks ({nv_one} "
                                          f"vertices), {t_one:.1f} s"}}

    chk0 = float(V.double().abs().sum())
    K = 2 if args.profile_only else args.steps
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(K):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / K
    nverts = int(blocks.v_off[-1])
    value = nverts / (ms * 1e-3)
    same = float(V.double().abs().sum()) == chk0  # the timed steps reproduce the checked result
    st = status.cpu().numpy()
    c_used = c.cpu().numpy()

    # one more step with every launch bracketed by HIP events on the
    # library's stream (eager launches): per-class durations for the roofline
    ctx.set_timing(True)
    step()
    torch.cuda.synchronize()
    ktimes = ctx.kernel_times()
    ctx.set_timing(False)
    step()  # back to graph replay
    torch.cuda.synchronize()
    shapes = [list(t) for t in ctx.tuning()]  # before other plans replace this one

    # the same kernels block after block (no wave, no graph) on the first 64
    # disks, and the batched path on the same 64
    per_block = None
    if not args.profile_only:
        k = 64
        sub = mis.Blocks(bs.n[:k], p=fl["p"][:k], ld=fl["ld"][:k])
        Ls = mis.Laplacian(L.row_ptr, L.col, L.val, L.edges, L.edge_w, L.nnz_off[:k + 1],
                           L.edge_off[:k + 1], L.mode)
        GLs = mis.Laplacian(GL.row_ptr, GL.col, GL.val, GL.edges, GL.edge_w, GL.nnz_off[:k + 1],
                            GL.edge_off[:k + 1], GL.mode)
        nvk = int(sub.v_off[-1])
        kw = dict(blk=sub, lap=Ls, gl=GLs, Vv=torch.empty(int(sub.u_off[-1]), dtype=torch.float32,
                                                           device=dev),
                  rz=torch.zeros(int(sub.t_off[-1]), dtype=torch.float64, device=dev),
                  st=torch.zeros(k, dtype=torch.int32, device=dev), cc=c[:k].clone(),
                  cm=cmax[:k].clone(), mt=torch.zeros(int(sub.t_off[-1]), dtype=torch.float64,
                                                      device=dev),
                  ee=torch.empty(int(sub.t_off[-1]) * 3, dtype=torch.float32, device=dev),
                  xr=torch.empty(nvk * 3, dtype=torch.float32, device=dev))
        res = {}
        for pb in (True, False):
            step(per_block=pb, **kw)  # plan
            torch.cuda.synchronize()
            tq = time.time()
            step(per_block=pb, **kw)
            torch.cuda.synchronize()
            res[pb] = (time.time() - tq) * 1e3
        per_block = {"blocks": k, "vertices": nvk, "per_block_ms": res[True],
                     "per_block_value": nvk / (res[True] * 1e-3), "batched_ms": res[False],
                     "batched_value": nvk / (res[False] * 1e-3), "unit": "vertices/s"}

    # the same step with every filter pass as one persistent launch over a
    # block work queue (workgroups claim whole disks, largest first, and run
    # the pass's m Chebyshev steps with workgroup barriers)
    persistent = None
    if not args.profile_only:
        V_graph = V.clone()
        prm.persistent = 1
        try:
            step()  # plan and graph capture
            torch.cuda.synchronize()
            ev0.record()
            for _ in range(K):
                step()
            ev1.record()
            torch.cuda.synchronize()
            ms_p = ev0.elapsed_time(ev1) / K
            equal = bool(torch.equal(V, V_graph))
            ctx.set_timing(True)
            step()
            torch.cuda.synchronize()
            kp = ctx.kernel_times()
            ctx.set_timing(False)
        finally:
            prm.persistent = 0
        del V_graph
        n64 = np.asarray(blocks.n, np.int64)
        nnz = np.diff(np.asarray(L.nnz_off, np.int64))
        csr_b = int(((n64 + 1) * 4 + nnz * 8).sum())
        slab_b = int((n64 * np.asarray(blocks.ld, np.int64) * 4).sum())
        pass_b = C3_M0 * (csr_b + 2 * slab_b) + (C3_M0 - 1) * slab_b
        pms, pn = kp["cheb_pass"]
        persistent = {"ms_per_step": ms_p, "value": nverts / (ms_p * 1e-3), "unit": "vertices/s",
                      "graph_ms_per_step": ms, "bit_equal_to_graph": equal,
                      "pass_launches": pn, "pass_avg_ms": pms / max(pn, 1),
                      "pass_bytes": pass_b,
                      "pass_achieved_GBs": pass_b / (pms / max(pn, 1) * 1e-3) / 1e9,
                      "step_launches_same_work_ms": C3_M0 * ktimes["spmm"][0] / ktimes["spmm"][1],
                      "spmm_launches_left": kp["spmm"][1]}
    out = {
        "metric": "submesh vertices/sec (OI + project/recon) at principal angle <=1e-5 vs FP64 oracle",
        "value": value,
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "disks1024_uneven_500_5000_p320_cmax256_fp32", "vertices": nverts,
                   "blocks": nb, "p_max": int(np.max(fl["p"])), "c_max": int(np.max(bs.c)),
                   "T": C3_T0, "m": C3_M0, "passes": C3_PASSES0, "start": "seeded (MI_RANDOM)",
                   "nmsve_target": target, "g_min": G_MIN,
                   "c_chosen_mean": float(c_used.mean()), "c_chosen_min": int(c_used.min()),
                   "c_chosen_max": int(c_used.max())},
        "roofline": roofline(ktimes, bs, blocks, L, prm, tag="disks", c_arr=c_used),
        "roofline_spmm": roofline(ktimes, bs, blocks, L, prm, "spmm", tag="disks"),
        "roofline_gram": roofline(ktimes, bs, blocks, L, prm, "gram", tag="disks"),
        "roofline_rowmul": roofline(ktimes, bs, blocks, L, prm, "rowmul", tag="disks"),
        "roofline_chol": roofline(ktimes, bs, blocks, L, prm, "chol", tag="disks"),
        "roofline_eig_reduce": roofline(ktimes, bs, blocks, L, prm, "eig_reduce", tag="disks"),
        "roofline_project": roofline(ktimes, bs, blocks, L, prm, "project", c_arr=c_used,
                                     tag="disks"),
        "roofline_reconstruct": roofline(ktimes, bs, blocks, L, prm, "reconstruct", c_arr=c_used,
                                         tag="disks"),
        "kernels": {k: {"ms": round(v[0], 4), "launches": v[1]} for k, v in ktimes.items() if v[1]},
        "launch_shapes": shapes,
        "build_laplacian_ms": lap_ms,
        "plan_and_capture_s": plan_s,
        "per_block_baseline": per_block,
        "persistent_queue": persistent,
        "sample_parity": parity,
        "timed_steps_reproduce_checked_result": same,
        "block_status_nonzero": int((st != 0).sum()),
        "input_gen_s": gen_s,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    ctx.close()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the workload is one GPU's share and no "
              "multi-GPU path is built.", file=sys.stderr)
        return 2
    if args.only_precision:
        print(json.dumps({"precision": c4_precision(args)}))
        return 0
    out = c3_headline(args)
    if not args.no_secondary and not args.profile_only:
        out["secondary"] = c2_secondary(args)
    if not args.no_precision and not args.profile_only:
        out["precision"] = c4_precision(args)
    print(json.dumps(out))
    return 0


def c4_precision(args):
    """The 1M-vertex precision workload: a displaced geodesic sphere of
    998,562 vertices in 100 blocks of about 10k vertices, c = 200, p = 256,
    one wave of independent blocks from seeded starts (12 iterations of two
    degree-10 passes), tracked once with FP32 slabs and once with BF16
    working slabs (MI_BF16_IN).  Per precision: the tracking's time (the mean
    of 3 graph replays after the plan), the SpMM's event-timed launches and
    their roofline at the slab's element size, and the smallest and the
    median block against the FP64 oracle (principal angle at c, and the
    reconstruction error)."""
    import torch

    import paper_1810_02719_amd as mis
    from oracle import laplacian as lap
    from oracle import spectral as S
    from synth import workloads as W
    dev = "cuda:0"
    t0 = time.time()
    bs = W.geodesic_blocks()
    fl = W.flatten(bs)
    blocks = mis.Blocks(bs.n, p=fl["p"], ld=fl["ld"])  # independent blocks: one wave
    prims = torch.from_numpy(np.ascontiguousarray(fl["prims"].reshape(-1))).to(dev)
    coords = torch.from_numpy(np.ascontiguousarray(fl["coords"].reshape(-1))).to(dev)
    gen_s = time.time() - t0
    ctx = mis.Context(0)
    L = mis.build_laplacian(ctx, blocks, fl["prim_off"], prims, 3, coords, mis.MI_W_COMBINATORIAL)
    c = torch.from_numpy(np.asarray(bs.c, np.int32)).to(dev)
    n = np.asarray(blocks.n)
    nverts = int(blocks.v_off[-1])
    if args.traffic_calib and args.only_precision:
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ids = [int(np.argmin(n)), int(np.argsort(n)[n.size // 2])]  # smallest and median block
    orc = {}
    if not args.profile_only:
        for b in ids:
            e = lap.canonical_edges(bs.faces[b], int(n[b]))
            lam, U = S.eigh_lowest(lap.laplacian_dense(int(n[b]), e, np.ones(len(e))),
                                   int(bs.p[b]) + 1)
            orc[b] = U
    out = {"workload": "geodesic316_998562v_100blocks_c200_p256", "vertices": nverts,
           "blocks": int(blocks.n_blocks), "T": 12, "m": 10, "passes": 2, "input_gen_s": gen_s}
    for name, prec, es in (("fp32", mis.MI_FP32, 4), ("bf16", mis.MI_BF16_IN, 2)):
        prm = mis.OiParams(precision=prec, warm=mis.MI_RANDOM, seed=SEED, T0=12, m0=10,
                           passes0=2, adapt=1, a_mode=mis.MI_A_WEYL, a_value=1.0, autotune=1)
        V = torch.empty(int(blocks.u_off[-1]), dtype=torch.float32, device=dev)
        ritz = torch.zeros(int(blocks.t_off[-1]), dtype=torch.float64, device=dev)
        status = torch.zeros(blocks.n_blocks, dtype=torch.int32, device=dev)
        mis.oi_track(ctx, blocks, L, prm, V=V, ritz=ritz, status=status)  # plan and capture
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        reps = 1 if args.profile_only else 3
        ev0.record()
        for _ in range(reps):
            mis.oi_track(ctx, blocks, L, prm, V=V, ritz=ritz, status=status)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        ctx.set_timing(True)
        mis.oi_track(ctx, blocks, L, prm, V=V, ritz=ritz, status=status)
        torch.cuda.synchronize()
        kt = ctx.kernel_times()
        ctx.set_timing(False)
        mis.oi_track(ctx, blocks, L, prm, V=V, ritz=ritz, status=status)  # graph replay again
        torch.cuda.synchronize()
        rec = {"ms_per_tracking": ms, "vertices_per_s": nverts / (ms * 1e-3),
               "block_status_nonzero": int((status.cpu().numpy() != 0).sum()),
               "launch_shapes": [list(t) for t in ctx.tuning()],
               "roofline_spmm": roofline(kt, bs, blocks, L, prm, "spmm", tag="sphere1m_" + name,
                                         es=es, levels=np.zeros(len(n), np.int64))}
        if orc:
            Xr = mis.reconstruct(ctx, blocks, c, V, mis.project(ctx, blocks, c, V, coords))
            torch.cuda.synchronize()
            Vh = V.double().cpu().numpy()
            Xh = Xr.double().cpu().numpy().reshape(-1, 3)
            rows = []
            for b in ids:
                nb, ld, cb = int(n[b]), int(blocks.ld[b]), int(bs.c[b])
                Vb = Vh[int(blocks.u_off[b]):int(blocks.u_off[b + 1])].reshape(nb, ld)
                X = bs.coords[b].astype(np.float32).astype(np.float64)
                v0 = int(blocks.v_off[b])
                rows.append({"block": b, "n": nb,
                             "sin_angle": S.sin_theta_max(orc[b][:, :cb], Vb[:, :cb]),
                             "recon_rel_err": S.rel_error(Xh[v0:v0 + nb],
                                                          S.encode_decode(orc[b][:, :cb], X))})
            rec["sample_parity"] = rows
        out[name] = rec
    ctx.close()
    return out


def c2_secondary(args):
    """The static block sequence (level-7 icosphere, 100 warm-started blocks,
    c = 100, p = 192, 5 BFS levels from 3 first blocks) with its extras."""
    import torch

    import paper_1810_02719_amd as mis
    from synth import workloads as W

    t0 = time.time()
    bs = W.icosphere_blocks(level=7, n_blocks=100, c=100, p=192, n_roots=N_ROOTS)
    fl = W.flatten(bs)
    dev = "cuda:0"
    blocks = mis.Blocks(bs.n, p=fl["p"], ld=fl["ld"], pred=bs.pred)
    prims = torch.from_numpy(np.ascontiguousarray(fl["prims"].reshape(-1))).to(dev)
    coords = torch.from_numpy(np.ascontiguousarray(fl["coords"].reshape(-1))).to(dev)
    V0 = np.zeros(int(blocks.u_off[-1]), np.float32)
    starts = W.random_starts(bs)
    for b in range(bs.n_blocks):
        if bs.pred[b] < 0:
            n, ld = int(blocks.n[b]), int(blocks.ld[b])
            V0[int(blocks.u_off[b]):int(blocks.u_off[b + 1])].reshape(n, ld)[:, :192] = starts[b]
    V0 = torch.from_numpy(V0).to(dev)
    gen_s = time.time() - t0

    ctx = mis.Context(0)
    # Laplacian build (reported separately)
    torch.cuda.synchronize()
    tl = time.time()
    L = mis.build_laplacian(ctx, blocks, fl["prim_off"], prims, 3, coords, mis.MI_W_COMBINATORIAL)
    torch.cuda.synchronize()
    lap_ms = (time.time() - tl) * 1e3

    prm = mis.OiParams(precision=mis.MI_FP32, warm=mis.MI_WARM_PRED, T=3, m=10, passes=2, T0=5,
                       m0=10, passes0=2, adapt=1, max_sweeps=12, a_mode=mis.MI_A_WEYL, a_value=1.0,
                       autotune=1)
    V = torch.empty(int(blocks.u_off[-1]), dtype=torch.float32, device=dev)
    ritz = torch.zeros(int(blocks.t_off[-1]), dtype=torch.float64, device=dev)
    status = torch.zeros(blocks.n_blocks, dtype=torch.int32, device=dev)
    c = torch.full((blocks.n_blocks,), 100, dtype=torch.int32, device=dev)
    E = torch.empty(int(blocks.t_off[-1]) * 3, dtype=torch.float32, device=dev)
    Xr = torch.empty(int(blocks.v_off[-1]) * 3, dtype=torch.float32, device=dev)

    def step():
        mis.oi_track(ctx, blocks, L, prm, V0=V0, V=V, ritz=ritz, status=status)
        mis.project(ctx, blocks, c, V, coords, E=E)
        mis.reconstruct(ctx, blocks, c, V, E, Xr=Xr)

    if args.traffic_calib:
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    K = 2 if args.profile_only else args.steps
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for i in range(K):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / K
    nverts = int(blocks.v_off[-1])
    value = nverts / (ms * 1e-3)
    st = status.cpu().numpy()

    # one more step with every kernel launch bracketed by HIP events on the
    # library's stream (eager launches): per-class durations for the roofline
    ctx.set_timing(True)
    step()
    torch.cuda.synchronize()
    ktimes = ctx.kernel_times()
    ctx.set_timing(False)
    step()  # back to graph replay
    torch.cuda.synchronize()
    shapes = [list(t) for t in ctx.tuning()]  # before other plans replace this one

    per_block_ms = None
    if not args.profile_only:
        per_block_ms = per_block_run(mis, ctx, blocks, L, prm, V0, V, ritz, status, c, coords, E, Xr)
        step()  # restore the batched result (the per-block run used the same output slab)
        torch.cuda.synchronize()

    merge = merge_run(mis, ctx, W, dev, reps=5 if args.profile_only else 50)

    # codec (Section 8): 12-bit uniform quantisation of this step's feature
    # vectors, the rate, and the change of the reconstruction it causes
    qb = 12
    mis.quantize(ctx, blocks, c, E, qb)
    ctx.set_timing(True)
    for _ in range(5 if args.profile_only else 20):
        _, _, Eq = mis.quantize(ctx, blocks, c, E, qb)
    torch.cuda.synchronize()
    q_ms, q_n = ctx.kernel_times()["quantize"]
    ctx.set_timing(False)
    Xq = mis.reconstruct(ctx, blocks, c, V, Eq)
    torch.cuda.synchronize()
    codec = {"qbits": qb, "bpv": 3.0 * qb * float(c.sum().item()) / nverts,
             "kernel_ms": q_ms / max(q_n, 1),
             "recon_rel_change": float((Xq - Xr).double().norm() / Xr.double().norm())}
    quality = quality_run(mis, ctx, bs, blocks, L, coords, Xr, Xq, dev,
                          reps=5 if args.profile_only else 50)
    doi = None if args.profile_only else doi_run(mis, ctx, blocks, L, coords, V0, dev, reps=3)
    rz = None if args.profile_only else rz_run(mis, ctx, blocks, L, V0, dev, reps=3)

    out = {
        "value": value,
        "unit": "vertices/s",
        "steps": K,
        "ms_per_step": ms,
        "config": {"workload": "icosphere7_100blocks_c100_T3_fp32", "vertices": nverts,
                   "blocks": int(blocks.n_blocks), "c": 100, "p": 192, "T": 3, "m": 10,
                   "passes": 2, "first_blocks": int((bs.pred < 0).sum()), "T_first": 5,
                   "m_first": 10, "passes_first": 2, "waves": int(bs.level.max() + 1)},
        "per_block_baseline": None if per_block_ms is None else
        {"value": nverts / (per_block_ms * 1e-3), "unit": "vertices/s", "ms": per_block_ms},
        "roofline": roofline(ktimes, bs, blocks, L, prm),
        "roofline_spmm": roofline(ktimes, bs, blocks, L, prm, "spmm"),
        "roofline_chol": roofline(ktimes, bs, blocks, L, prm, "chol"),
        "roofline_gram": roofline(ktimes, bs, blocks, L, prm, "gram"),
        "roofline_project": roofline(ktimes, bs, blocks, L, prm, "project"),
        "roofline_reconstruct": roofline(ktimes, bs, blocks, L, prm, "reconstruct"),
        "kernels": {k: {"ms": round(v[0], 4), "launches": v[1]} for k, v in ktimes.items() if v[1]},
        "launch_shapes": shapes,
        "build_laplacian_ms": lap_ms,
        "merge": merge,
        "codec": codec,
        "quality": quality,
        "doi": doi,
        "rz": rz,
        "block_status_nonzero": int((st != 0).sum()),
        "input_gen_s": gen_s,
    }

    if not args.no_cpu_baseline and not args.profile_only:
        out["cpu_baseline"], out["sample_parity"] = cpu_baseline(bs, blocks, V, Xr, args)
    ctx.close()
    return out


N_ROOTS = 3  # first blocks (cold starts); the rest are warm-started
CALIB_BYTES = 256 << 20
HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "paper_1810_02719_amd", "csrc")
TRAFFIC = {
    ("spmm", "disks"): (os.path.join(HERE, "profiles", "spmm_disks1024_traffic.json"),
                        os.path.join(CSRC, "dense.hip")),
    ("spmm", "sphere1m_fp32"): (os.path.join(HERE, "profiles", "spmm_sphere1m_fp32_traffic.json"),
                                os.path.join(CSRC, "dense.hip")),
    ("spmm", "sphere1m_bf16"): (os.path.join(HERE, "profiles", "spmm_sphere1m_bf16_traffic.json"),
                                os.path.join(CSRC, "dense.hip")),
}
MI_RANDOM = 2  # seeded start mode of mi_oi_params.warm


def measured_traffic(kind, alg_bytes_per_launch, tag="icosphere"):
    """HBM bytes per launch of a kernel class ("spmm", "chol", "gram") of a
    workload ("icosphere", "disks") from the committed rocprofv3 counter
    passes (FETCH_SIZE and WRITE_SIZE, scaled by the same counters of a copy
    of known size), or None when there is none, the kernel source changed
    since, or the launches no longer have the size they had then."""
    import hashlib
    if (kind, tag) not in TRAFFIC:
        return None
    path, source = TRAFFIC[(kind, tag)]
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(source, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != sha:
        return None
    ref = rec.get("algorithmic_bytes_per_launch")
    if not ref or abs(ref - alg_bytes_per_launch) > 0.01 * ref:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector and MFMA (dense)


FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix


def roofline(ktimes, bs, blocks, L, prm, dom=None, c_arr=None, tag="icosphere", es=4,
             levels=None):
    """Roofline of a kernel class of the step (default: the dominant one, the
    largest event-timed total).  The algorithmic bytes or flops of one step's
    launches of that class (the method's own traffic, not what the caches
    make of it) over the event-timed total.  c_arr: the kept sizes the step
    used (default: the block set's c); levels: the dependency level of
    every block as tracked (default: the block set's; all zero when the
    blocks run as independent blocks in one wave)."""
    if dom is None:
        dom = max(ktimes, key=lambda k: ktimes[k][0])
    ms, launches = ktimes[dom]
    levels = np.asarray(bs.level if levels is None else levels)
    n = np.asarray(blocks.n, np.int64)
    ld = np.asarray(blocks.ld, np.int64)
    p = np.asarray(blocks.p, np.int64)
    nnz = np.diff(np.asarray(L.nnz_off, np.int64))
    # es: bytes per slab element (4 for FP32, 2 for BF16 working slabs)
    out = {"kernel": dom, "launches": launches, "avg_us": 1e3 * ms / max(launches, 1),
           "traffic": None}
    if dom == "spmm":
        # per launch over a wave: CSR (row_ptr, col, val) once, the input
        # block once, the previous iterate (all but the first step of a
        # pass) and the output
        tot = 0
        for lvl in np.unique(levels):
            sel = levels == lvl
            T, m, passes = (prm.T0, prm.m0, prm.passes0) if lvl == 0 else (prm.T, prm.m, prm.passes)
            csr = int(((n[sel] + 1) * 4 + nnz[sel] * 8).sum())
            slab = int((n[sel] * ld[sel] * es).sum())
            per_pass = m * (csr + 2 * slab) + (m - 1) * slab
            # W = L X once per iteration for the adaptive bound, and for the
            # Rayleigh-Ritz step
            n_w = (T - 1) * (1 if prm.adapt else 0) + 1
            tot += T * passes * per_pass + n_w * (csr + 2 * slab)
        out.update(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS, bytes_per_step=tot,
                   bytes_per_launch=tot / max(launches, 1))
        out["achieved"] = tot / (ms * 1e-3) / 1e9
        out["traffic"] = measured_traffic("spmm", tot / max(launches, 1), tag)
    elif dom == "chol":
        # Cholesky (p^3/3) and triangular inverse (p^3/3) of every block's
        # Gram, for each of the step's Cholesky-QRs.  Bytes: the Gram's upper
        # triangle read (FP64), R^-1 written in full (FP64, ld x ld) and, for
        # all but the Rayleigh-Ritz factorisation, its FP32 copy
        tot, byt = 0, 0
        for lvl in np.unique(levels):
            sel = levels == lvl
            T, passes = (prm.T0, prm.passes0) if lvl == 0 else (prm.T, prm.passes)
            start = lvl > 0 or prm.warm == MI_RANDOM  # a Cholesky-QR of the start basis
            nchol = T * passes + 1 + (1 if start else 0)
            tot += nchol * int((2 * p[sel].astype(np.float64) ** 3 / 3).sum())
            pp, ll = p[sel].astype(np.int64), ld[sel].astype(np.int64)
            byt += int((nchol * 8 * pp * (pp + 1) // 2 + (nchol - 1) * 12 * ll * ll
                        + 8 * ll * ll).sum())
        out.update(bound="alu", unit="TFLOP/s", peak=FP64_PEAK_TFLOPS, flops_per_step=tot,
                   bytes_per_launch=byt / max(launches, 1))
        out["achieved"] = tot / (ms * 1e-3) / 1e12
        out["traffic"] = measured_traffic("chol", byt / max(launches, 1), tag)
    elif dom == "eig_reduce":
        # Householder tridiagonalisation of every block's p x p Rayleigh-Ritz
        # matrix (4 p^3 / 3 flops), one per block and step
        tot = int((4.0 * p.astype(np.float64) ** 3 / 3).sum())
        out.update(bound="alu", unit="TFLOP/s", peak=FP64_PEAK_TFLOPS, flops_per_step=tot)
        out["achieved"] = tot / (ms * 1e-3) / 1e12
    elif dom == "gram":
        # Y^T Y over the rows (upper triangle incl. the diagonal, FP64 MFMA):
        # n p (p + 1) flops; the Rayleigh-Ritz product is dual (Y^T Y, Y^T W),
        # every other one (each Cholesky-QR) single
        tot, byt = 0, 0
        for lvl in np.unique(levels):
            sel = levels == lvl
            T, passes = (prm.T0, prm.passes0) if lvl == 0 else (prm.T, prm.passes)
            start = lvl > 0 or prm.warm == MI_RANDOM
            single = T * passes + (1 if start else 0)
            per = (n[sel] * p[sel] * (p[sel] + 1)).astype(np.float64).sum()
            tot += (single + 2) * per
            slab = float((n[sel] * ld[sel] * es).sum())
            byt += (single + 2) * slab  # one read of each operand slab
        out.update(bound="mfma", unit="TFLOP/s", peak=FP64_PEAK_TFLOPS, flops_per_step=tot,
                   bytes_per_launch=byt / max(launches, 1))
        out["achieved"] = tot / (ms * 1e-3) / 1e12
        out["traffic"] = measured_traffic("gram", byt / max(launches, 1), tag)
    elif dom == "rowmul":
        # Y S on the FP32 MFMA: the Rayleigh-Ritz rotation (S = R^-1 Z, full:
        # 2 n p ld flops) and the Cholesky-QRs (S = R^-1, upper triangular:
        # n p (p + 1) flops, column j summing j + 1 products)
        tot = 0
        for lvl in np.unique(levels):
            sel = levels == lvl
            T, passes = (prm.T0, prm.passes0) if lvl == 0 else (prm.T, prm.passes)
            start = lvl > 0 or prm.warm == MI_RANDOM
            ntri = T * passes + (1 if start else 0) + 1
            nn, pp, ll = (x[sel].astype(np.float64) for x in (n, p, ld))
            tot += float((2 * nn * pp * ll).sum()) + ntri * float((nn * pp * (pp + 1)).sum())
        out.update(bound="mfma", unit="TFLOP/s", peak=FP32_MFMA_PEAK_TFLOPS, flops_per_step=tot)
        out["achieved"] = tot / (ms * 1e-3) / 1e12
    elif dom in ("project", "reconstruct"):
        # per row: the first c_b entries of the basis row (FP32) and the
        # row's coordinates (project: read; reconstruct: written)
        c = np.asarray(bs.c if c_arr is None else c_arr, np.int64)
        tot = int((n * (es * c + 12)).sum())
        out.update(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS, bytes_per_step=tot,
                   bytes_per_launch=tot / max(launches, 1))
        out["achieved"] = tot / (ms * 1e-3) / 1e9
    elif dom == "jacobi_sweep":
        # sweeps run until convergence: the work is data dependent; count the
        # minimum, one full sweep per block and Rayleigh-Ritz (3 q^2 (q-1)
        # flops: every rotation updates two rows of the packed matrix)
        q = (p + 1) // 2 * 2
        tot = int((3.0 * q ** 2 * (q - 1)).sum())
        out.update(bound="alu", unit="TFLOP/s", peak=FP64_PEAK_TFLOPS, flops_per_step_min=tot)
        out["achieved"] = tot / (ms * 1e-3) / 1e12
    else:
        out.update(bound=None, unit=None, peak=None, achieved=None)
    out["frac"] = None if out["achieved"] is None else out["achieved"] / out["peak"]
    return out


def per_block_run(mis, ctx, blocks, L, prm, V0, V, ritz, status, c, coords, E, Xr):
    """The same kernels launched block after block (no waves, no graph): the
    plain sequential schedule of the paper's block loop, for comparison."""
    import torch
    for it in range(2):  # first call builds the plan
        torch.cuda.synchronize()
        t = time.time()
        mis.oi_track(ctx, blocks, L, prm, V0=V0, V=V, ritz=torch.zeros_like(ritz),
                     status=torch.zeros_like(status), per_block=True)
        mis.project(ctx, blocks, c, V, coords, E=E)
        mis.reconstruct(ctx, blocks, c, V, E, Xr=Xr)
        torch.cuda.synchronize()
    return (time.time() - t) * 1e3


def cpu_baseline(bs, blocks, V, Xr, args):
    """The FP64 oracle (dense eigh + projection + reconstruction) on a bounded
    sample of the same blocks, timed on the host; the oracle's subspaces of the
    sampled blocks also give the GPU result's principal angles."""
    from threadpoolctl import threadpool_info

    from oracle import laplacian as lap
    from oracle import spectral as S
    order = [int(b) for b in bs.order[:args.cpu_sample_blocks]]
    Vh = V.double().cpu().numpy()
    Xh = Xr.double().cpu().numpy().reshape(-1, 3)
    angles, recs = [], []
    t = 0.0
    nv = 0
    for b in order:
        n = int(blocks.n[b])
        X = bs.coords[b].astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        e = lap.canonical_edges(bs.faces[b], n)
        Lb = lap.laplacian_dense(n, e, np.ones(len(e)))
        lam, U = S.eigh_lowest(Lb)
        Xo = S.encode_decode(U[:, :100], X)
        t += time.perf_counter() - t0
        nv += n
        ld = int(blocks.ld[b])
        Vg = Vh[int(blocks.u_off[b]):int(blocks.u_off[b + 1])].reshape(n, ld)[:, :100]
        angles.append(S.sin_theta_max(U[:, :100], Vg))
        v0 = int(blocks.v_off[b])
        recs.append(S.rel_error(Xh[v0:v0 + n], Xo))
    threads = max([i.get("num_threads", 1) for i in threadpool_info()
                   if i.get("internal_api") in ("openblas", "mkl", "blis")] or [1])
    base = {"value": nv / t, "unit": "vertices/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(order)} of {bs.n_blocks} blocks (first in BFS order, {nv} vertices): "
                      f"dense FP64 eigh + projection + reconstruction, {t:.1f} s"}
    par = {"blocks": len(order), "sin_angle_max": float(max(angles)),
           "sin_angle_median": float(np.median(angles)),
           "recon_rel_err_max": float(max(recs))}
    return base, par


if __name__ == "__main__":
    sys.exit(main())
