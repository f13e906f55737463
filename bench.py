#!/usr/bin/env python3
"""Throughput of the octree GIMP assembly hot path on one GPU.

One step = one pass of the whole hot path over the workload's points:
  point-to-cell (Morton keys, radix sort, leaf search) + state gather into sorted order,
  fused assembly (basis, kinematics, Hencky/von Mises return, consistent tangent, per-leaf
  reduction, scatter into f_int and CSR K) + residual and its FP64 norm,
  adjoint assembly (dL/dE, dL/dnu, dL/dsigma_y, dL/dV_n per point).
`value` = points / wall time of one step (FP64 primary run); the FP32-tangent run is
reported beside it. Inputs are resident in HBM before the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "material points/s for residual+tangent assembly (FP64 vs FP32) + adjoint cost"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_VEC_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_VEC_TFLOPS = 157.3   # packed FP32 (the library is built without packed FP32 ops)

# Algorithmic cost of one point with an 8-node stencil (flops; FMA = 2):
# basis 100, kinematics (H, grad_x S, dF^-1) 330, b_tr 90, symmetric 3x3 eigen 400,
# return map 50, spatial tangent 3000, T_b = a.g_b 1296, upper-triangle K blocks 1944,
# force 144.
FLOPS_PER_POINT = 100 + 330 + 90 + 400 + 50 + 3000 + 1296 + 1944 + 144
# Algorithmic HBM bytes of one assembly launch: per point read x, l (48), V_n, J_n (16),
# b_n (48), E, nu, sy (24) and write sigma (48) = 184 B; plus K values written once
# (nnz x 8 or 4) and u read + f_int written once (3 n_node x 16).
BYTES_PER_POINT = 184


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("assemble.hip", "point_math.h", "geom.h", "internal.h"):
        h.update((ROOT / "paper_2606_09275_amd" / "csrc" / f).read_bytes())
    return h.hexdigest()


def measured_traffic(workload_name, prim):
    """HBM bytes per launch of the FP64 assembly kernel from the committed rocprofv3 counter
    runs (FETCH_SIZE x2 + WRITE_SIZE, calibrated on a plain copy); None when the kernel
    sources changed since the counters were taken or no run exists for this workload."""
    p = ROOT / "profiles" / f"assemble_fast_traffic_{workload_name.split('_')[0]}.json"
    if prim != "f64" or not p.exists():
        return None
    d = json.loads(p.read_text())
    if d.get("source_sha256") != kernel_source_hash() or not d.get("workload", "").startswith(workload_name[:2]):
        return None
    return float(d["hbm_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--cpu-sample", type=int, default=1000000, help="points in the oracle CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["f64", "f32k"], default=None, help="time one precision only")
    ap.add_argument("--calib-copy", action="store_true", help="run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--jitter", type=int, default=None,
                    help="move the points by the seeded jitter k (domains over several leaves: the general path)")
    ap.add_argument("--no-c4", action="store_true", help="skip the largest workload's protocol in the output")
    return ap.parse_args()


def calib_copy():
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_read": n * 8, "calib_copy_bytes_written": n * 8, "launches": 3}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is a "
              "design note (contiguous Morton ranges per GPU with one halo exchange of interface rows), "
              "not a measured path.", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads as W
    from paper_2606_09275_amd.mesh import Mesh

    if args.calib_copy:
        calib_copy()
        return
    torch.cuda.set_device(0)
    w = W.get(args.workload)
    t0 = time.time()
    m0 = Mesh(w.crit())
    lv = m0.arrays()["leaf"].cpu().numpy()
    del m0
    ps = W.make_points(w, lv[:, :3], lv[:, 3])
    if args.jitter is not None:
        ps = W.jitter_points(w, ps, args.jitter)
    st = W.make_state(w, ps)
    log(f"[bench] workload {w.name}: {ps.n} points, {lv.shape[0]} leaves ({time.time() - t0:.1f}s)")
    x_dev = torch.from_numpy(ps.x).cuda()
    l_dev = torch.from_numpy(ps.l).cuda()
    if "prev_x_s" in w.extra:
        # moving tool: the mesh of the previous tool position exists first; the timed build
        # below is the re-adaptation to the current position with the same points
        b = list(w.body)
        dx = float(w.extra["prev_x_s"]) - b[0]
        prev = dict(w.crit(), body=tuple([b[0] + dx, b[1] + dx] + b[2:] + [0.0] * (8 - len(b))))
        pm = Mesh(prev, x_dev, l_dev)
        del pm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh = Mesh(w.crit(), x_dev, l_dev)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    info = mesh.info
    rp = mesh.arrays()["row_ptr"]
    max_deg = int(((rp[1::3] - rp[:-1:3]) // 3).max().item()) if info["n_node"] else 0
    log(f"[bench] octree_build {build_ms:.1f} ms: nodes {info['n_node']} hanging {info['n_hang']} "
        f"nnz {info['nnz']} straddle {info['n_straddle']} widest row {max_deg} nodes")
    nodes = mesh.arrays()["node_ijk"].cpu().numpy()
    u = torch.from_numpy(W.make_u(w, nodes)).cuda()
    lam = torch.from_numpy(W.make_lambda(w, nodes)).cuda()
    dirichlet = torch.from_numpy(W.dirichlet_dofs(nodes)).cuda()
    n = ps.n
    # original-order state packed as one [ncomp, n] device array; sorted-order views of a copy
    keys = [("x", 3), ("l", 3), ("vol", 1), ("mass", 1), ("Jn", 1), ("bn", 6), ("E", 1), ("nu", 1), ("sy", 1)]
    packed = torch.cat([torch.from_numpy(np.asarray(st[k], np.float64).reshape(c, n)) for k, c in keys]).cuda()
    sorted_buf = torch.empty_like(packed)
    views, r = {}, 0
    for k, c in keys:
        v = sorted_buf[r:r + c]
        views[k] = v.reshape(-1) if c == 1 else v
        r += c
    views["g"] = (0.0, 0.0, -9.81)
    perm_buf = torch.empty(n, dtype=torch.int64, device="cuda")
    leaf_buf = torch.empty(n, dtype=torch.int32, device="cuda")
    # f_ext is constant over the Newton iterations of a step: computed once, outside the timing
    mesh.permute(packed, None, out=sorted_buf)
    f_ext = mesh.external_force(views)
    torch.cuda.synchronize()

    def step(prec, outs, ev=None):
        mesh.point_sort(x_dev, perm_buf, leaf_buf)
        mesh.permute(packed, perm_buf, out=sorted_buf)
        if ev is not None:
            ev[0].record()
        mesh.assemble(views, u, prec, f_ext=f_ext, dirichlet=dirichlet, out=outs["asm"])
        if ev is not None:
            ev[1].record()
        mesh.adjoint(views, u, lam, prec, out=outs["adj"])
        if ev is not None:
            ev[2].record()

    results = {}
    precs = [args.only] if args.only else ["f64", "f32k"]
    for prec in precs:
        outs = {"asm": {}, "adj": {}}
        for _ in range(args.warmup):
            step(prec, outs)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        mesh.kernel_timing(1)
        mesh.kernel_timing(-1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            evs[k][3].record()
            step(prec, outs, ev=evs[k])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = mesh.kernel_timing(0)
        ms = (t1 - t0) * 1e3 / args.steps
        step_ms = np.array([e[3].elapsed_time(e[2]) for e in evs])
        sort_ms = float(np.mean([e[3].elapsed_time(e[0]) for e in evs]))
        asm_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
        adj_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
        k_asm = kt[0] / max(kt[1], 1)
        k_adj = kt[2] / max(kt[3], 1)
        k_gat = kt[4] / max(kt[5], 1)
        rn = float(outs["asm"]["rnorm"].item())
        results[prec] = dict(ms_per_step=ms, value=n / (ms * 1e-3), sort_ms=sort_ms, assemble_ms=asm_ms,
                             adjoint_ms=adj_ms, assemble_kernel_ms=k_asm, adjoint_kernel_ms=k_adj,
                             gather_kernel_ms=k_gat,
                             assembly_points_per_s=n / (asm_ms * 1e-3), adjoint_points_per_s=n / (adj_ms * 1e-3),
                             adjoint_over_assembly=adj_ms / asm_ms, rnorm=rn,
                             step_ms_p10=float(np.percentile(step_ms, 10)),
                             step_ms_p50=float(np.percentile(step_ms, 50)),
                             step_ms_p90=float(np.percentile(step_ms, 90)))
        log(f"[bench] {prec}: step {ms:.3f} ms ({n / ms / 1e3:.3e} pts/s) | sort+gather {sort_ms:.3f} "
            f"assemble {asm_ms:.3f} (kernel {k_asm:.3f} + gather {k_gat:.3f}) adjoint {adj_ms:.3f} (kernel {k_adj:.3f}) ms")

    prim = "f64" if "f64" in results else precs[0]
    R = results[prim]
    n_fast = n - info["n_straddle"]

    def roofline_of(prec, r):
        """ALU roofline of the fused kernel (algorithmic flops of its points over its own
        average launch time) and the HBM roofline of the assembly's two kernels (the fused
        kernel reads the state and writes sigma and the segment sums; the row gather writes K
        and f_int): algorithmic bytes over the sum of their average launch times."""
        kb = 8 if prec == "f64" else 4
        alg_flops = FLOPS_PER_POINT * n_fast
        alg_bytes = BYTES_PER_POINT * n + info["nnz"] * kb + 3 * info["n_node"] * 16
        kt_s = r["assemble_kernel_ms"] * 1e-3
        kg_s = (r["assemble_kernel_ms"] + r["gather_kernel_ms"]) * 1e-3
        peak = PEAK_FP64_VEC_TFLOPS if prec == "f64" else PEAK_FP32_VEC_TFLOPS
        rf = {"bound": "alu", "kernel": "k_assemble_fast<%s, false>" % ("double" if prec == "f64" else "float"),
              "achieved": alg_flops / kt_s / 1e12, "peak": peak, "unit": "TFLOP/s",
              "frac": alg_flops / kt_s / 1e12 / peak, "traffic": measured_traffic(w.name, prec),
              "flops_per_point": FLOPS_PER_POINT, "points_per_launch": n_fast,
              "kernel_ms": r["assemble_kernel_ms"],
              "hbm": {"kernels": "k_assemble_fast + k_gather", "achieved": alg_bytes / kg_s / 1e9,
                      "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": alg_bytes / kg_s / 1e9 / PEAK_HBM_GBS,
                      "bytes_per_launch": alg_bytes, "kernels_ms": kg_s * 1e3}}
        if prec != "f64":
            # the library is built without packed FP32 instructions: its own ceiling is the
            # unpacked FP32 rate, equal to the FP64 one
            rf["frac_of_unpacked_fp32"] = alg_flops / kt_s / 1e12 / PEAK_FP64_VEC_TFLOPS
        return rf

    roofline = roofline_of(prim, R)
    out = {
        "metric": METRIC, "value": R["value"], "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": R["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prim == "f64" else "f32",
        "data": "synthetic (seeded octree workload; no experimental data)",
        "config": {"workload": f"{w.name}: {w.note}", "n_points": n, "n_leaf": info["n_leaf"],
                   "n_node": info["n_node"], "n_hang": info["n_hang"], "nnz": info["nnz"],
                   "n_straddle": info["n_straddle"],
                   "step": "point sort + state gather + assemble (f_int, K, sigma, residual norm) + adjoint"},
        "phases_ms": {k: R[k] for k in ("sort_ms", "assemble_ms", "adjoint_ms", "assemble_kernel_ms",
                                        "gather_kernel_ms", "adjoint_kernel_ms", "step_ms_p10",
                                        "step_ms_p50", "step_ms_p90")},
        "setup_ms": {"octree_build": build_ms},
        "assembly_points_per_s": R["assembly_points_per_s"], "adjoint_points_per_s": R["adjoint_points_per_s"],
        "adjoint_over_assembly": R["adjoint_over_assembly"],
        "roofline": roofline,
    }
    if "f32k" in results and prim != "f32k":
        out["fp32k"] = {k: results["f32k"][k] for k in ("value", "ms_per_step", "assembly_points_per_s",
                                                         "adjoint_points_per_s", "assemble_kernel_ms",
                                                         "gather_kernel_ms", "adjoint_kernel_ms")}
        out["fp32k"]["speedup_assembly_vs_fp64"] = results["f32k"]["assembly_points_per_s"] / R["assembly_points_per_s"]
        out["fp32k"]["roofline"] = roofline_of("f32k", results["f32k"])
    if not args.only:
        out["dynamic"] = dynamic_assembly(mesh, w, ps, views, u, f_ext, dirichlet, n)
        out["solve"] = newton_solve(mesh, views, u, f_ext, dirichlet, info)
        out["ghost"] = ghost_stabilisation(w, x_dev, l_dev, views, u, f_ext, dirichlet, R["assemble_ms"])
        out["gimp_split"] = gimp_split(mesh, w)
    out["state_gather_runs_ms"] = gather_runs(mesh, packed, sorted_buf)
    if not args.only and w.name.startswith("c2") and args.jitter is None:
        out["supplementary"] = supplementary(w)
        if not args.no_c4:
            out["supplementary"]["c4"] = c4_protocol()
    if "prev_x_s" in w.extra:
        out["protocol"] = tool_protocol(mesh, w, nodes, views, x_dev, perm_buf, leaf_buf, packed, sorted_buf,
                                        f_ext, dirichlet, lam)
    if not args.no_cpu_baseline:
        out["cpu_baseline"], errs = cpu_baseline(w, ps, st, nodes, args.cpu_sample)
        out.setdefault("fp32k", {})["err"] = errs["f32k"]
        out["fp64_err"] = errs["f64"]
    print(json.dumps(out), flush=True)


def dynamic_assembly(mesh, w, ps, views, u, f_ext, dirichlet, n, reps=10, dt=1e-3):
    """The Newmark (gamma = 1, beta = 1/2) dynamic assembly on the sorted state: mean ms of the
    call and of its fused kernel, per precision (same u, point velocities N(0, 0.1^2))."""
    import torch
    import workloads as W
    vel = torch.from_numpy(W.make_velocity(w, ps)).cuda()  # order does not matter for timing
    res = {}
    for prec in ("f64", "f32k"):
        outs = {}
        mesh.assemble_dynamic(views, u, vel, dt, prec, f_ext=f_ext, dirichlet=dirichlet, out=outs)
        torch.cuda.synchronize()
        mesh.kernel_timing(1)
        mesh.kernel_timing(-1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            mesh.assemble_dynamic(views, u, vel, dt, prec, f_ext=f_ext, dirichlet=dirichlet, out=outs)
        e1.record()
        torch.cuda.synchronize()
        kt = mesh.kernel_timing(0)
        ms = e0.elapsed_time(e1) / reps
        res[prec] = {"assembly_ms": ms, "assemble_kernel_ms": kt[0] / max(kt[1], 1),
                     "gather_kernel_ms": kt[4] / max(kt[5], 1), "assembly_points_per_s": n / (ms * 1e-3)}
    log(f"[bench] dynamic assembly: f64 {res['f64']['assembly_ms']:.3f} ms (kernel "
        f"{res['f64']['assemble_kernel_ms']:.3f}), f32k {res['f32k']['assembly_ms']:.3f} ms")
    return res


def ghost_stabilisation(w, x_dev, l_dev, views, u, f_ext, dirichlet, plain_ms, reps=10):
    """The FP64 assembly on the same points with the ghost penalty of Section 4 (mesh built with
    ghost faces): build time, face count, pattern growth, and mean ms of the assembly (HIP
    events over reps calls) against the plain assembly's."""
    import torch
    from paper_2606_09275_amd.mesh import Mesh
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gm = Mesh(w.crit(), x_dev, l_dev, ghost=True)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    outs = {}
    for _ in range(2):
        gm.assemble(views, u, "f64", f_ext=f_ext, dirichlet=dirichlet, out=outs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        gm.assemble(views, u, "f64", f_ext=f_ext, dirichlet=dirichlet, out=outs)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    res = {"n_ghost_face": gm.info["n_ghost_face"], "nnz": gm.info["nnz"], "octree_build_ms": build_ms,
           "assemble_ms": ms, "plain_assemble_ms": plain_ms, "overhead_ms": ms - plain_ms}
    log(f"[bench] ghost: {res['n_ghost_face']} faces, nnz {res['nnz']}, build {build_ms:.1f} ms, "
        f"assemble {ms:.3f} ms (plain {plain_ms:.3f} ms)")
    del gm
    return res


def supplementary(w_main, reps=5):
    """Assembly throughput (FP64 and FP32K, mean of reps calls with HIP events, inputs sorted
    and resident) of the other configurations: the sphere workload with full and with partial
    yielding, and the jittered variant of the main workload (domains over several leaves run
    the general path with atomics)."""
    import torch
    import workloads as W
    from paper_2606_09275_amd.mesh import Mesh
    res = {}
    cases = [("c1", W.get("c1"), None), ("c1b", W.get("c1b"), None), (w_main.name.split("_")[0] + "_jittered", w_main, 0)]
    for tag, w, jit in cases:
        m0 = Mesh(w.crit())
        lv = m0.arrays()["leaf"].cpu().numpy()
        del m0
        ps = W.make_points(w, lv[:, :3], lv[:, 3])
        if jit is not None:
            ps = W.jitter_points(w, ps, jit)
        st = W.make_state(w, ps)
        m = Mesh(w.crit(), torch.from_numpy(ps.x).cuda(), torch.from_numpy(ps.l).cuda())
        nodes = m.arrays()["node_ijk"].cpu().numpy()
        u = torch.from_numpy(W.make_u(w, nodes)).cuda()
        s = m.sorted_state(st)
        r = {"points": ps.n, "n_straddle": m.info["n_straddle"], "nnz": m.info["nnz"],
             "sigma_y": w.sy, "yield_fraction": yield_fraction(m, s, u)}
        for prec in ("f64", "f32k"):
            outs = {}
            m.assemble(s, u, prec, out=outs)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                m.assemble(s, u, prec, out=outs)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            r[f"assemble_{prec}_ms"] = ms
            r[f"assembly_{prec}_points_per_s"] = ps.n / (ms * 1e-3)
        log(f"[bench] {tag}: {ps.n} points ({r['n_straddle']} straddling, {r['yield_fraction']:.3f} yielding), "
            f"assembly FP64 "
            f"{r['assemble_f64_ms']:.3f} ms ({r['assembly_f64_points_per_s']:.3e} pts/s), FP32K "
            f"{r['assemble_f32k_ms']:.3f} ms")
        res[tag] = r
        del m, s, outs
    return res


def yield_fraction(m, s, u):
    """Fraction of the points whose returned stress lies on the yield surface: one FP64
    assembly with the committed history, tau = J sigma with J = det F_new, and the von Mises
    stress sqrt(3 J2) of tau against sigma_y (relative slack 1e-9)."""
    import torch
    o = m.assemble(s, u, "f64", want_K=False, want_residual=False, commit=True)
    F = o["F_new"]
    J = (F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
         F[2] * (F[3] * F[7] - F[4] * F[6]))
    tau = o["sigma"] * J
    d = tau.clone()
    d[:3] -= tau[:3].mean(0)
    q = torch.sqrt(1.5 * (d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + 2 * (d[3] ** 2 + d[4] ** 2 + d[5] ** 2)))
    sy = s["sy"]
    return float((torch.isfinite(sy) & (q >= sy * (1 - 1e-9))).double().mean().item())


def c4_protocol(reps=3):
    """The largest single-GPU workload (moving box tool, about 30 M points in a never-coarsened
    trail): mesh at the previous tool position, then the timed re-adaptation (octree_build at
    the current position with the same points), re-sort and state gather, ten assemblies with
    the FP32 tangent (FP64 f_int; displacement k of the step's Newton iterations), one FP32K
    adjoint, and the FP64 step (sort + gather + assembly + adjoint, mean of reps)."""
    import torch
    import workloads as W
    from paper_2606_09275_amd.mesh import Mesh
    w = W.get("c4")
    t0 = time.time()
    m0 = Mesh(w.crit())
    lv = m0.arrays()["leaf"].cpu().numpy()
    del m0
    ps = W.make_points(w, lv[:, :3], lv[:, 3])
    st = W.make_state(w, ps)
    n = ps.n
    log(f"[bench] c4: {n} points generated ({time.time() - t0:.1f}s)")
    x_dev = torch.from_numpy(ps.x).cuda()
    l_dev = torch.from_numpy(ps.l).cuda()
    b = list(w.body)
    dx = float(w.extra["prev_x_s"]) - b[0]
    prev = dict(w.crit(), body=tuple([b[0] + dx, b[1] + dx] + b[2:] + [0.0] * (8 - len(b))))
    pm = Mesh(prev, x_dev, l_dev)
    del pm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh = Mesh(w.crit(), x_dev, l_dev)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    info = mesh.info
    nodes = mesh.arrays()["node_ijk"].cpu().numpy()
    keys = [("x", 3), ("l", 3), ("vol", 1), ("mass", 1), ("Jn", 1), ("bn", 6), ("E", 1), ("nu", 1), ("sy", 1)]
    packed = torch.cat([torch.from_numpy(np.asarray(st[k], np.float64).reshape(c, n)) for k, c in keys]).cuda()
    del st
    sorted_buf = torch.empty_like(packed)
    views, r = {}, 0
    for k, c in keys:
        v = sorted_buf[r:r + c]
        views[k] = v.reshape(-1) if c == 1 else v
        r += c
    views["g"] = (0.0, 0.0, -9.81)
    perm_buf = torch.empty(n, dtype=torch.int64, device="cuda")
    leaf_buf = torch.empty(n, dtype=torch.int32, device="cuda")
    dirichlet = torch.from_numpy(W.dirichlet_dofs(nodes)).cuda()
    lam = torch.from_numpy(W.make_lambda(w, nodes)).cuda()
    mesh.permute(packed, None, out=sorted_buf)
    f_ext = mesh.external_force(views)
    prot = tool_protocol(mesh, w, nodes, views, x_dev, perm_buf, leaf_buf, packed, sorted_buf, f_ext, dirichlet, lam)
    u = torch.from_numpy(W.make_u(w, nodes)).cuda()
    outs, adj = {}, {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def step():
        mesh.point_sort(x_dev, perm_buf, leaf_buf)
        mesh.permute(packed, perm_buf, out=sorted_buf)
        mesh.assemble(views, u, "f64", f_ext=f_ext, dirichlet=dirichlet, out=outs)
        mesh.adjoint(views, u, lam, "f64", out=adj)

    step()
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        step()
    ev[1].record()
    torch.cuda.synchronize()
    step_ms = ev[0].elapsed_time(ev[1]) / reps
    res = {"points": n, "n_leaf": info["n_leaf"], "n_node": info["n_node"], "nnz": info["nnz"],
           "readapt_octree_build_ms": build_ms, **prot, "fp64_step_ms": step_ms,
           "fp64_step_points_per_s": n / (step_ms * 1e-3),
           "assembly_f32k_points_per_s": n / (prot["assembly_f32k_ms"] * 1e-3)}
    log(f"[bench] c4: re-adapt {build_ms:.1f} ms, re-sort {prot['resort_ms']:.2f} ms, FP32K assembly "
        f"{prot['assembly_f32k_ms']:.2f} ms x 10, adjoint {prot['adjoint_f32k_ms']:.2f} ms, FP64 step {step_ms:.2f} ms")
    del mesh, packed, sorted_buf, views, outs, adj
    torch.cuda.empty_cache()
    return res


def gather_runs(mesh, packed, sorted_buf, reps=10):
    """State gather of the same 18 components when the point order is one run (points already
    in sorted order, as between time steps when few points change leaves): mean ms."""
    import torch
    ident = torch.arange(packed.shape[1], dtype=torch.int64, device="cuda")
    mesh.permute(packed, ident, out=sorted_buf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        mesh.permute(packed, ident, out=sorted_buf)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    mesh.permute(packed, None, out=sorted_buf)  # restore the sorted state
    torch.cuda.synchronize()
    log(f"[bench] state gather of an order made of runs: {ms:.3f} ms")
    return ms


def gimp_split(mesh, w, reps=5):
    """GIMP refinement (Section 5) on the mesh: points laid out one level coarser than the
    leaves (2 per axis in each parent cell) with the full state, reference positions and
    velocities; mean ms of the criterion and of the split (HIP events over reps calls), and the
    split's HBM rate from the bytes it must move (8 bytes x 33 fields read per input point and
    written per output point, plus the flags)."""
    import dataclasses
    import torch
    import workloads as W
    lv = mesh.arrays()["leaf"].cpu().numpy()
    par = lv.copy()
    s = np.left_shift(1, w.lvl_max - (lv[:, 3] - 1))
    par[:, :3] = (lv[:, :3] // s[:, None]) * s[:, None]
    par[:, 3] = lv[:, 3] - 1
    par = np.unique(par[par[:, 3] >= w.lvl_base], axis=0)
    w2 = dataclasses.replace(w, ppa=lambda lev: 2)
    pc = W.make_points(w2, par[:, :3], par[:, 3])
    st = W.make_state(w2, pc)
    dev = {k: torch.from_numpy(np.ascontiguousarray(st[k], np.float64)).cuda()
           for k in ("x", "l", "vol", "mass", "Jn", "bn", "Fn", "E", "nu", "sy")}
    X = dev["x"].clone()
    v = torch.zeros_like(X)
    props = {"E": (float(w.E), 0.0, 0.0, 0.0)}
    flags, cnt = mesh.split_mark(dev["x"], dev["l"])
    mesh.split_apply(dev, flags, cnt, X=X, v=v, props=props)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e[0].record()
    for _ in range(reps):
        flags, cnt = mesh.split_mark(dev["x"], dev["l"], out=flags)
    e[1].record()
    for _ in range(reps):
        o = mesh.split_apply(dev, flags, cnt, X=X, v=v, props=props)
    e[2].record()
    torch.cuda.synchronize()
    n = pc.n
    n_out = n + 7 * cnt
    mark_ms = e[0].elapsed_time(e[1]) / reps
    apply_ms = e[1].elapsed_time(e[2]) / reps
    nbytes = 33 * 8 * (n + n_out) + n
    res = {"points": n, "split": cnt, "points_out": n_out, "mark_ms": mark_ms, "apply_ms": apply_ms,
           "mark_points_per_s": n / (mark_ms * 1e-3), "apply_bytes": nbytes,
           "apply_GBps": nbytes / (apply_ms * 1e-3) / 1e9, "apply_hbm_frac": nbytes / (apply_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    log(f"[bench] GIMP split: {cnt} of {n} points -> {n_out}; criterion {mark_ms:.3f} ms, split {apply_ms:.3f} ms "
        f"({res['apply_GBps']:.0f} GB/s)")
    del o
    return res


def newton_solve(mesh, views, u, f_ext, dirichlet, info, iters=100, spmv_reps=20):
    """Linear solve of the first Newton step of a body-force load step (u = 0, elastic response
    from an unstrained start, right-hand side f_ext) with Jacobi-preconditioned CG over the free
    DOFs, on the same mesh and points (the tangent at the randomly strained plastic state of
    this workload is not positive definite, which ends CG early): ms per CG iteration over a
    fixed iteration count, iterations to a 1e-6 relative residual (at most 4000), and the SpMV
    kernel alone against the HBM roofline (bytes: K values, one column index per entry of a
    node's first row, x and y)."""
    import torch
    res = {}
    # elastic response from an unstrained start (F_n = I): a positive definite tangent
    bn0 = torch.zeros_like(views["bn"])
    bn0[:3] = 1.0
    el = dict(views, sy=torch.full_like(views["sy"], float("inf")), bn=bn0, Jn=torch.ones_like(views["Jn"]))
    u0 = torch.zeros_like(u)  # first Newton iteration of a step: the load is the body force
    for prec, tb in (("f64", 8), ("f32k", 4)):
        outs = {}
        mesh.assemble(el, u0, prec, f_ext=f_ext, dirichlet=dirichlet, out=outs)
        K = outs["K"]
        b = -outs["r"]
        mesh.solve_cg(K, b, dirichlet, rtol=0.0, max_iter=16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, it, rel = mesh.solve_cg(K, b, dirichlet, rtol=0.0, max_iter=iters)
        torch.cuda.synchronize()
        ms_it = (time.perf_counter() - t0) * 1e3 / max(it, 1)
        t0 = time.perf_counter()
        _, it6, rel6 = mesh.solve_cg(K, b, dirichlet, rtol=1e-6, max_iter=4000)
        torch.cuda.synchronize()
        solve_ms = (time.perf_counter() - t0) * 1e3
        y = torch.empty_like(b)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        mesh.spmv(K, x, out=y)
        e0.record()
        for _ in range(spmv_reps):
            mesh.spmv(K, x, out=y)
        e1.record()
        torch.cuda.synchronize()
        spmv_ms = e0.elapsed_time(e1) / spmv_reps
        nnz, ndof = info["nnz"], info["n_dof"]
        byts = nnz * tb + (nnz // 3) * 4 + ndof * 8 * 2 + (ndof + 1) * 8
        res[prec] = {"cg_iteration_ms": ms_it, "iterations_timed": it, "iterations_to_1e-6": it6,
                     "relres_final": rel6, "solve_to_1e-6_ms": solve_ms, "spmv_ms": spmv_ms,
                     "spmv_gbs": byts / (spmv_ms * 1e-3) / 1e9, "spmv_bytes": byts,
                     "spmv_hbm_frac": byts / (spmv_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
        log(f"[bench] solve {prec}: {ms_it:.3f} ms per CG iteration ({it} timed); to 1e-6: {it6} iterations, "
            f"{solve_ms:.1f} ms (relres {rel6:.1e}); SpMV {spmv_ms:.3f} ms = {res[prec]['spmv_gbs']:.0f} GB/s")
        res[prec]["gmres"] = gmres_solves(mesh, K, b, dirichlet, views, u, f_ext, prec)
    return res


def gmres_solves(mesh, K, b, dirichlet, views, u, f_ext, prec, restart=30, max_iter=3000):
    """Restarted GMRES (Jacobi preconditioner on the right) on the elastic tangent above (ms per
    Arnoldi step over two full cycles, steps and time to a 1e-6 true relative residual) and on
    the tangent at this workload's strained state and displacement, which is not positive
    definite: CG stops there, GMRES is timed to 1e-6 (at most max_iter steps)."""
    import torch
    mesh.solve_gmres(K, b, dirichlet, rtol=0.0, restart=restart, max_iter=restart)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, it, _ = mesh.solve_gmres(K, b, dirichlet, rtol=0.0, restart=restart, max_iter=2 * restart)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / max(it, 1)
    t0 = time.perf_counter()
    _, it6, rel6 = mesh.solve_gmres(K, b, dirichlet, rtol=1e-6, restart=restart, max_iter=max_iter)
    torch.cuda.synchronize()
    el_ms = (time.perf_counter() - t0) * 1e3
    outs = {}
    mesh.assemble(views, u, prec, f_ext=f_ext, dirichlet=dirichlet, out=outs)
    Kp, bp = outs["K"], -outs["r"]
    _, itc, relc = mesh.solve_cg(Kp, bp, dirichlet, rtol=1e-6, max_iter=max_iter)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, itp, relp = mesh.solve_gmres(Kp, bp, dirichlet, rtol=1e-6, restart=restart, max_iter=max_iter)
    torch.cuda.synchronize()
    pl_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] gmres({restart}) {prec}: {ms_step:.3f} ms per Arnoldi step; elastic to 1e-6: {it6} steps "
        f"{el_ms:.1f} ms (relres {rel6:.1e}); strained tangent: CG stops after {itc} (relres {relc:.1e}), "
        f"GMRES {itp} steps {pl_ms:.1f} ms (relres {relp:.1e})")
    return {"restart": restart, "step_ms": ms_step, "elastic_steps_to_1e-6": it6, "elastic_relres": rel6,
            "elastic_solve_ms": el_ms, "strained_cg_iterations": itc, "strained_cg_relres": relc,
            "strained_steps": itp, "strained_relres": relp, "strained_solve_ms": pl_ms}


def tool_protocol(mesh, w, nodes, views, x_dev, perm_buf, leaf_buf, packed, sorted_buf, f_ext, dirichlet, lam):
    """Moving-tool protocol after re-adaptation: re-sort of the points, then the Newton
    iterations of one step (10 assemblies with FP32 tangent and FP64 f_int, displacement k
    drawn with seed (seed_u, 1, k)) and one adjoint; mean milliseconds of each."""
    import torch
    import workloads as W
    us = [torch.from_numpy(W.make_u(w, nodes, k=k)).cuda() for k in range(10)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    outs = {}
    mesh.assemble(views, us[0], "f32k", f_ext=f_ext, dirichlet=dirichlet, out=outs)
    torch.cuda.synchronize()
    ev[0].record()
    mesh.point_sort(x_dev, perm_buf, leaf_buf)
    mesh.permute(packed, perm_buf, out=sorted_buf)
    ev[1].record()
    for k in range(10):
        mesh.assemble(views, us[k], "f32k", f_ext=f_ext, dirichlet=dirichlet, out=outs)
    ev[2].record()
    mesh.adjoint(views, us[-1], lam, "f32k")
    ev[3].record()
    torch.cuda.synchronize()
    return {"resort_ms": ev[0].elapsed_time(ev[1]), "assembly_f32k_ms": ev[1].elapsed_time(ev[2]) / 10,
            "adjoint_f32k_ms": ev[2].elapsed_time(ev[3]), "iterations": 10}


def cpu_baseline(w, ps, st, nodes, sample):
    """The FP64 oracle on a bounded sample of the same workload (every k-th point, on a mesh of
    the same octree): assembly (f_int, K, sigma) + adjoint on one thread, the oracle as
    written, which is `value`; the assembly again on all the host threads the process may use
    (per-thread sums added in a fixed order), reported beside it. The oracle's results on the
    sample are also the reference of the per-result errors of the library's FP64 and FP32
    tangent paths, run on a library mesh of the same sample points (precision_errors)."""
    import workloads as W
    from oracle.oracle import OracleMesh, residual
    k = max(1, ps.n // sample)
    idx = np.arange(0, ps.n, k)
    o = OracleMesh(w.crit())
    o.set_points(ps.x[:, idx], ps.l[:, idx])
    ss = {key: (v[..., idx] if isinstance(v, np.ndarray) else v) for key, v in st.items()}
    u = W.make_u(w, nodes)
    lam = W.make_lambda(w, nodes)
    t0 = time.perf_counter()
    ref = o.assemble(ss, u)
    t1 = time.perf_counter()
    o.adjoint(ss, u, lam)
    t2 = time.perf_counter()
    threads = max(1, min(int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0)),
                         len(os.sched_getaffinity(0))))
    t3 = time.perf_counter()
    par = o.assemble_threads(ss, u, threads)
    t4 = time.perf_counter()
    agree = float(np.abs(par["K"] - ref["K"]).max() / np.abs(ref["K"]).max())
    log(f"[bench] cpu oracle: {idx.size} points, assemble {t1 - t0:.2f}s adjoint {t2 - t1:.2f}s (1 thread); "
        f"assemble on {threads} threads {t4 - t3:.2f}s (K agrees to {agree:.1e})")
    fe = o.external_force(dict(ss, g=(0.0, 0.0, -9.81)))
    d = W.dirichlet_dofs(nodes)
    r_ref, rn_ref = residual(ref["f_int"], fe, d)
    errs = precision_errors(w, ps, idx, ss, u, d, o, ref, r_ref, rn_ref)
    base = {"value": idx.size / (t2 - t0), "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"every {k}-th point of the workload ({idx.size} points), FP64 assembly of f_int, K, sigma "
                      f"({t1 - t0:.1f}s) + adjoint ({t2 - t1:.1f}s), single thread",
            "assembly_points_per_s": idx.size / (t1 - t0), "cpu": _cpu_name(), "host_threads": os.cpu_count(),
            "all_cores": {"value": idx.size / (t4 - t3), "unit": "points/s (assembly of f_int, K, sigma)",
                          "cores": threads, "kind": "oracle, points cut into one contiguous range per thread",
                          "cpu": _cpu_name(), "max_rel_diff_K_vs_one_thread": agree}}
    return base, errs


def precision_errors(w, ps, idx, ss, u, d, o, ref, r_ref, rn_ref):
    """Per-result error of the library's FP64 and FP32-tangent assemblies against the FP64
    oracle on the CPU baseline's sample: the same points on a library mesh of the same
    octree (its CSR pattern equals the oracle's bit for bit), the same state, displacement,
    body force and fixed base. Normwise max|diff| / max|ref| for f_int, K, sigma and r;
    relative error of the residual norm."""
    import torch
    import workloads as W
    from paper_2606_09275_amd.mesh import Mesh
    m = Mesh(w.crit(), torch.from_numpy(np.ascontiguousarray(ps.x[:, idx])).cuda(),
             torch.from_numpy(np.ascontiguousarray(ps.l[:, idx])).cuda())
    perm = m.arrays()["perm"].cpu().numpy()
    s = m.sorted_state(dict(ss, g=(0.0, 0.0, -9.81)))
    fe = m.external_force(s)
    ud = torch.from_numpy(u).cuda()
    dd = torch.from_numpy(d).cuda()

    def rel(a, b):
        return float(np.abs(np.asarray(a, np.float64) - b).max() / np.abs(b).max())

    res = {}
    for prec in ("f64", "f32k"):
        out = m.assemble(s, ud, prec, f_ext=fe, dirichlet=dd)
        torch.cuda.synchronize()
        res[prec] = {"f_int": rel(out["f_int"].cpu().numpy(), ref["f_int"]),
                     "K": rel(out["K"].cpu().numpy(), ref["K"]),
                     "sigma": rel(out["sigma"].cpu().numpy(), ref["sigma"][:, perm]),
                     "r": rel(out["r"].cpu().numpy(), r_ref),
                     "rnorm": abs(float(out["rnorm"].item()) - rn_ref) / rn_ref,
                     "points": int(idx.size), "yield_fraction_oracle": float(ref["plastic"].mean()),
                     "reference": "FP64 oracle on the CPU baseline's sample"}
        log(f"[bench] {prec} errors vs oracle: " + " ".join(f"{k}={res[prec][k]:.2e}" for k in
                                                           ("f_int", "K", "sigma", "r", "rnorm")))
    del m
    return res


def _cpu_name():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
