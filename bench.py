"""Benchmark of the matrix-free P1 apply on one MI355X.

One step = one apply_stencil (y = A x, a single fused launch: interior rows
of the macro plus its macro-boundary/Dirichlet rows) on the 2D workload:
one macro triangle under a seeded random affine map, refinement level 14
(134,242,305 DoFs, 1.07 GB per FP64 vector), x ~ U[-1,1) from the keyed
generator.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line.  value = unique DoFs per second (GDoF/s) of the whole
job.  roofline: algorithmic bytes (16 B/DoF: x read once, y written once)
per launch / average launch time (HIP events on the launch stream), against
the 8 TB/s HBM3E peak.  cpu_baseline: the oracle's CSR row loop on the host
cores for a bounded sample.  extra: the FP32 apply, the 3D 6-tet cube apply,
the fused 2D P2 apply (vertex and edge DoFs, level 13: the same 134,242,305
DoFs), the variable-coefficient apply (weights formed on the fly from a nodal
coefficient, level 14), the library's streaming copy (the measured-copy
denominator of the roofline), and the mixed-precision vs FP64 V-cycle solve
with its algorithmic bytes per iteration and fraction of HBM peak.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_DOF_APPLY = {"f64": 16, "f32": 8}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_apply2d_l14.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2305_15116_amd", "csrc", "stencil_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bench_apply(P, torch, co, ce, L, dtype, steps, warmup, seed, p2=False):
    """Times the P1 apply of level L, or (p2=True) the P2 apply of level L,
    whose vectors have the layout of level L + 1."""
    Lv = L + 1 if p2 else L
    m = P.create_macro_mesh(co, ce, Lv)
    s, u = P.mesh_num_dofs(m, Lv)
    x = torch.empty(s, dtype=dtype, device="cuda")
    P.mesh_fill_random(m, Lv, seed, x)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    apply = P.apply_p2 if p2 else P.apply_stencil
    for _ in range(warmup):
        apply(m, L, x, y, stream)
    torch.cuda.synchronize()
    # whole timed region: `steps` back-to-back applies
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        apply(m, L, x, y, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    # each launch bracketed by its own events, for the per-launch average and median
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        apply(m, L, x, y, stream)
        b.record(stream)
    torch.cuda.synchronize()
    per = sorted(a.elapsed_time(b) for a, b in ev)
    del x, y
    P.destroy_macro_mesh(m)
    return {"storage": s, "unique": u, "ms_per_step": total_ms / steps, "launch_avg_ms": sum(per) / len(per),
            "launch_median_ms": per[len(per) // 2]}


def _launch_times(torch, stream, call, steps, warmup):
    """Average and median of `steps` launches of call(stream), each bracketed
    by its own HIP events on that stream."""
    for _ in range(warmup):
        call(stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        call(stream)
        b.record(stream)
    torch.cuda.synchronize()
    per = sorted(a.elapsed_time(b) for a, b in ev)
    return {"launch_avg_ms": sum(per) / len(per), "launch_median_ms": per[len(per) // 2]}


def bench_varcoef(P, torch, co, ce, L, dtype, steps, warmup):
    """Per-launch HIP-event times of apply_varcoef (k in [0.5, 2.5) from the
    keyed generator)."""
    m = P.create_macro_mesh(co, ce, L)
    s, u = P.mesh_num_dofs(m, L)
    x = torch.empty(s, dtype=dtype, device="cuda")
    k = torch.empty_like(x)
    P.mesh_fill_random(m, L, 3, x)
    P.mesh_fill_random(m, L, 4, k)
    k += 1.5
    y = torch.empty_like(x)
    r = _launch_times(torch, torch.cuda.current_stream(), lambda st: P.apply_varcoef(m, L, k, x, y, st), steps, warmup)
    del x, y, k
    P.destroy_macro_mesh(m)
    return {"storage": s, "unique": u, **r}


def bench_blended(P, torch, co, ce, L, steps, warmup):
    """Per-launch HIP-event times of apply_blended (FP64; every macro's bubble
    vector (0.45, -0.3), which keeps the mapped micro triangles valid)."""
    m = P.create_macro_mesh(co, ce, L)
    s, u = P.mesh_num_dofs(m, L)
    x = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 3, x)
    y = torch.empty_like(x)
    d = torch.tensor([[0.45, -0.3]] * len(ce), dtype=torch.float64, device="cuda")
    r = _launch_times(torch, torch.cuda.current_stream(), lambda st: P.apply_blended(m, L, d, x, y, st), steps, warmup)
    del x, y
    P.destroy_macro_mesh(m)
    return {"storage": s, "unique": u, **r}


def copy_bandwidth(P, torch, nbytes=1 << 30, reps=20):
    """Read + write GB/s of the library's streaming copy (device_copy: 16-byte
    loads, non-temporal 16-byte stores) and of torch's copy_, both over 1 GiB,
    each launch timed with HIP events on the launch stream."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    stream = torch.cuda.current_stream()
    out = {}
    for name, call in (("device_copy", lambda st: P.device_copy(b, a, st)), ("torch_copy", lambda st: b.copy_(a))):
        r = _launch_times(torch, stream, call, reps, 3)
        out[name] = 2 * nbytes / (r["launch_avg_ms"] * 1e-3) / 1e9
    del a, b
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def _time_oracle(om, budget_s, single_reps):
    """Median seconds of the oracle's CSR row loop on all host threads (reps
    fitted to budget_s) and on one thread."""
    nnz = om._native(True)
    nthreads = os.cpu_count() or 1
    t, used = om.time_spmv(nthreads, 2, 3)
    per = float(sorted(t)[len(t) // 2])
    reps = max(5, min(400, int(budget_s / max(per, 1e-6))))
    t, used = om.time_spmv(nthreads, 0, reps)
    med = float(sorted(t)[len(t) // 2])
    t1, _ = om.time_spmv(1, 1, single_reps)
    med1 = float(sorted(t1)[len(t1) // 2])
    csr_bytes = om.n * 8 * 2 + nnz * 16 + (om.n + 1) * 8  # x, y, values + column indices, row pointers
    return med, med1, reps, int(used), nnz, csr_bytes


def cpu_baseline(W, budget_s=20.0):
    """The oracle's CSR row loop on all host cores for a bounded sample of the
    same workload: the same affine triangle at level 13 (33.6M DoFs, a CSR of
    about 3.8 GB, far beyond the host caches)."""
    from oracle.oracle import OracleMesh
    co, ce = W.affine_triangle(2)
    L = 13
    t0 = time.time()
    om = OracleMesh(co, ce, L)
    om._native(True)
    t_build = time.time() - t0
    med, med1, reps, used, nnz, csr_bytes = _time_oracle(om, budget_s, 3)
    out = {"value": om.n / med / 1e9, "unit": "GDoF/s", "cores": used, "kind": "oracle",
           "sample": f"same affine triangle at level {L} ({om.n} DoFs, {nnz} CSR entries, {csr_bytes / 1e9:.2f} GB "
                     f"moved per product): CSR row loop y = A x, median of {reps} reps on {used} threads; CSR "
                     f"assembly ({t_build:.1f} s) excluded",
           "csr_GBps": csr_bytes / med / 1e9, "single_thread_GDoF_s": om.n / med1 / 1e9, "cpu_model": _cpu_model(),
           "nproc": os.cpu_count()}
    del om
    return out


def cpu_oracle_cube(W, L=8, reps=100):
    """The oracle on the 3D benchmark mesh (6-tet cube, level 8: 16,974,593
    unique DoFs, 15-entry rows): CSR row loop, median of `reps` products on
    all host threads and of 5 on one thread."""
    from oracle.oracle import OracleMesh
    t0 = time.time()
    om = OracleMesh(*W.kuhn_cube(), L)
    om._native(True)
    t_build = time.time() - t0
    med, med1, _, used, nnz, csr_bytes = _time_oracle(om, 1e9, 5)
    nthreads = os.cpu_count() or 1
    t, used = om.time_spmv(nthreads, 3, reps)
    med = float(sorted(t)[len(t) // 2])
    out = {"GDoF_s": om.n / med / 1e9, "single_thread_GDoF_s": om.n / med1 / 1e9, "threads": int(used),
           "reps": reps, "csr_GBps": csr_bytes / med / 1e9, "nnz": nnz, "assembly_s": t_build,
           "cpu_model": _cpu_model(), "nproc": os.cpu_count()}
    del om
    return out


def traffic_for(kernel_hash):
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != kernel_hash:
        return None
    return d.get("bytes_per_launch")


def solve_bytes(P, m, L, mode, iters, lc=2):
    """Algorithmic HBM bytes of one vcycle_solve with V(2,2) cycles: every
    vector a kernel of the solve must read or write, once (interface and
    coarse-solve traffic excluded).  Per V-cycle level l above the coarse
    level (storage S_l, precision e bytes: 8 FP64, 4 FP32 cycles): first
    sweep from zero 2e, second sweep 3e, residual 3e, restriction e + e S_{l-1}/S_l,
    prolongation e S_{l-1}/S_l + 2e, two post-sweeps 6e.  Outer step per fine
    DoF: refinement x += e and r = b - A x (FP64 48, mixed 56 with the
    scaled cast); CG r.z, direction, A p with p.Ap, x/r update (FP64 104,
    mixed 100: r.z and the direction read the FP32 cycle output, 4 bytes
    less each, and the update also writes the next FP32 preconditioner
    input, 4; the first input's cast, 12, is set-up);
    MINRES A z with z.Az 16, the Lanczos
    recurrence 32, v.z 16 (mixed: the scaled cast 12 and z formed in FP64,
    20), the direction recurrence 32 and x += c eta w 24 (FP64 120, mixed
    136).  Set-up: norm of b and the first residual (32), plus one
    recomputed residual (24) at Krylov termination; MINRES also clears three
    vectors (24) and applies the preconditioner once before its first
    iteration (one cycle and v.z)."""
    S = [P.mesh_num_dofs(m, l)[0] for l in range(L + 1)]
    e = 4 if mode & 1 else 8
    cycle = sum((17 * e + 2 * e * S[l - 1] / S[l]) * S[l] for l in range(lc + 1, L + 1))
    outer = {0: 48, 1: 56, 2: 104, 3: 100, 4: 120, 5: 136}[mode] * S[L]
    setup = (32 + (24 if mode & 6 else 0) + (12 if mode == 3 else 0)) * S[L]
    if mode & 4:
        setup += cycle + (24 + (32 if mode & 1 else 16)) * S[L]
    return {"per_iteration": cycle + outer, "per_iteration_B_per_dof": (cycle + outer) / S[L],
            "per_solve": setup + iters * (cycle + outer)}


def solve_bench(P, torch, W, L=8, repeats=10, modes=(0, 1, 2, 3, 4, 5)):
    co, ce = W.kuhn_cube()
    m = P.create_macro_mesh(co, ce, L)
    s, _ = P.mesh_num_dofs(m, L)
    # b = lumped load of f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z): on this mesh the
    # lumped mass is h^3 at every DoF; built here from the DoF coordinates.
    v, w = P.mesh_dof_keys(m, L)
    import numpy as np
    N = 1 << L
    xyz = np.zeros((s, 3))
    for k in range(4):
        ok = v[:, k] >= 0
        xyz[ok] += (w[ok, k:k + 1] / N) * co[v[ok, k]]
    h = 1.0 / N
    f = 3 * np.pi ** 2 * np.prod(np.sin(np.pi * xyz), axis=1)
    b = torch.as_tensor(h ** 3 * f, device="cuda")
    out = {}
    names = {0: "fp64", 1: "mixed", 2: "fp64_pcg", 3: "mixed_pcg", 4: "fp64_minres", 5: "mixed_minres"}
    for mode in modes:
        ws = torch.empty(P.mesh_workspace_bytes(m, L, mode), dtype=torch.uint8, device="cuda")
        x = torch.zeros(s, dtype=torch.float64, device="cuda")
        rc, it, rel, sec = P.vcycle_solve(m, L, b, x, ws, mode=mode, rtol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            x.zero_()
            rc, it, rel, sec = P.vcycle_solve(m, L, b, x, ws, mode=mode, rtol=1e-10)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / repeats
        us = np.prod(np.sin(np.pi * xyz), axis=1)
        uh = us * (np.pi ** 2 * h ** 2 / 4) / np.sin(np.pi * h / 2) ** 2
        xs = x.cpu().numpy()
        err = float(np.abs(xs - uh).max())
        err_cont = float(np.abs(xs - us).max())
        by = solve_bytes(P, m, L, mode, it)
        out[names[mode]] = {"mode": mode, "status": rc, "iters": it, "rel_res": rel, "ms_per_solve": dt * 1e3,
                            "ms_per_iteration": dt * 1e3 / max(it, 1), "solves_per_s": 1.0 / dt,
                            "algorithmic_B_per_dof_per_iteration": round(by["per_iteration_B_per_dof"], 1),
                            "algorithmic_GB_per_solve": by["per_solve"] / 1e9,
                            "achieved_GBps": by["per_solve"] / dt / 1e9,
                            "frac_of_hbm_peak": by["per_solve"] / dt / 1e9 / HBM_PEAK_GBS,
                            "max_err_vs_discrete_solution": err, "max_err_vs_continuous_solution": err_cont}
        del ws
    P.destroy_macro_mesh(m)
    return out


def serve_bench(torch, variant, n, util=0.75, budget_gib=None, calib_n=40, servers="both"):
    """Serving workload: Poisson arrivals of solve requests (2D strips of 1-64
    triangles, 3D rows of 1-64 Kuhn tets, seeded affine maps, tol 1e-8).
    capped: 3D levels 5-8 and an arrival rate set to `util` of the plain
    server's measured capacity; full: levels 5-11 at 200 requests/s."""
    from paper_2305_15116_amd import loadgen, serving
    # device memory the server may commit to requests (HBM is 288 GB; the
    # allocator's cache and the meshes' metadata need the rest)
    budget_gib = budget_gib or (200.0 if variant == "capped" else 160.0)
    budget = int(budget_gib * 2 ** 30)
    levels3 = (5, 8) if variant == "capped" else (5, 11)
    out = {"variant": variant, "n": n, "budget_GiB": budget_gib}
    if variant == "capped":
        out["deviation"] = ("not the stated serving workload: 3D levels 5-8 instead of 5-11, and an arrival rate of "
                            f"{util:.0%} of the plain server's measured capacity instead of 200 requests/s, whose "
                            "offered load (3D levels 9-11 with up to 64 tets) exceeds one GPU; --serve full runs "
                            "the stated workload")
    if variant == "capped":
        sample = loadgen.requests(n=calib_n, rate=1.0, levels3=levels3, seed_arrival=16, seed_req=17)
        srv = serving.Server(budget, batched=False, keep_solutions=False)
        t0 = time.perf_counter()
        futs = [srv.submit(r.dim, r.coords, r.cells, r.level, r.rhs_seed, r.tol) for r in sample]
        infos = [f.result()[1] for f in futs]
        srv.close()
        svc = (max(i["t_done"] for i in infos) - t0) / calib_n
        rate = util / svc
        out["calibration"] = {"requests": calib_n, "plain_service_ms": svc * 1e3, "target_utilisation": util}
    else:
        rate = 200.0
    out["rate_req_per_s"] = rate
    reqs = loadgen.requests(n=n, rate=rate, levels3=levels3)
    which = {"both": (False, True), "plain": (False,), "batched": (True,)}[servers]
    for name, batched in (("plain_fp64_fifo", False), ("batched_mixed", True)):
        if batched not in which:
            continue
        log(f"serving {variant}: {name}, {n} requests at {rate:.1f}/s")
        srv = serving.Server(budget, batched=batched, keep_solutions=False)
        out.setdefault("solver_modes", {})[name] = srv.mode
        futs, t0, _ = loadgen.replay(srv, reqs)
        import concurrent.futures as cf
        pending = set(futs)
        while pending:  # progress lines while the backlog drains
            _, pending = cf.wait(pending, timeout=20.0)
            log(f"  {len(futs) - len(pending)}/{len(futs)} requests finished")
        infos, rejected, status = [], 0, {}
        for f in futs:
            try:
                x, info = f.result()
            except Exception:
                rejected += 1
                continue
            infos.append(info)
            status[info["status"]] = status.get(info["status"], 0) + 1
        srv.close()
        t1 = max([i["t_done"] for i in infos], default=t0)
        st = serving.latency_stats(infos, t0, t1)
        st.update({"rejected": srv.rejected, "failed_to_prepare": srv.failed, "status_counts": {str(k): v for k, v in status.items()},
                   "offered_req_per_s": rate, "achieved_req_per_s": len(infos) / max(t1 - t0, 1e-9),
                   "busy_frac_per_lane": [b / max(t1 - t0, 1e-9) for b in srv.lane_busy_s],
                   "mean_iters": float(np.mean([i["iters"] for i in infos])) if infos else None})
        out[name] = st
        log(f"serving {variant} {name}: " + json.dumps(st))
    if "p50_ms" in out.get("plain_fp64_fifo", {}) and "p50_ms" in out.get("batched_mixed", {}):
        out["p50_speedup"] = out["plain_fp64_fifo"]["p50_ms"] / out["batched_mixed"]["p50_ms"]
        out["p99_speedup"] = out["plain_fp64_fifo"]["p99_ms"] / out["batched_mixed"]["p99_ms"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-extra", action="store_true")
    ap.add_argument("--skip-solve", action="store_true", help="leave the V-cycle solve out of the extras")
    ap.add_argument("--serve", choices=["none", "capped", "full"], default="capped",
                    help="serving workload in the extras (full: 2000 requests at 200/s, levels 5-11)")
    ap.add_argument("--serve-n", type=int, default=None, help="requests of the serving run")
    ap.add_argument("--serve-servers", choices=["both", "plain", "batched"], default="both",
                    help="which servers the serving run measures")
    ap.add_argument("--solve-only", type=int, choices=[0, 1, 2, 3, 4, 5], default=None,
                    help="only run the cube level-8 solve of this mode three times (for kernel traces)")
    ap.add_argument("--cpu-cube", action="store_true",
                    help="also time the oracle on the 3D benchmark mesh (cube level 8, 100 products; assembly takes minutes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of 1 GiB (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the macro-parallel multi-GPU path is not built "
              "(every GPU box here has one GPU); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2305_15116_amd as P
    from paper_2305_15116_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    P.lib()

    if args.solve_only is not None:
        print(json.dumps({"solve_cube_l8": solve_bench(P, torch, W, repeats=3, modes=(args.solve_only,))}), flush=True)
        return
    co, ce = W.affine_triangle(2)
    L = 14
    log(f"apply 2D level {L} fp64: {args.warmup} warmup + {args.steps} timed")
    r64 = bench_apply(P, torch, co, ce, L, torch.float64, args.steps, args.warmup, 3)
    gdofs = r64["unique"] / (r64["ms_per_step"] * 1e-3) / 1e9
    bytes_launch = BYTES_PER_DOF_APPLY["f64"] * r64["unique"]
    achieved = bytes_launch / (r64["launch_avg_ms"] * 1e-3) / 1e9
    khash = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(khash),
                "kernel": "stencil_kernel<double,2,apply>", "algorithmic_bytes_per_launch": bytes_launch,
                "launch_avg_ms": r64["launch_avg_ms"], "launch_median_ms": r64["launch_median_ms"]}
    extra = {}
    if args.copy_calibration:
        # one library streaming copy (stream_copy_kernel) of exactly 1 GiB read and 1 GiB written:
        # its FETCH_SIZE / WRITE_SIZE readings calibrate the counters of the other kernels
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        P.device_copy(b, a)
        torch.cuda.synchronize()
        extra["copy_calibration_bytes"] = {"read": a.numel() * 8, "write": b.numel() * 8}
        del a, b
    if not args.skip_extra:
        log("apply 2D level 14 fp32")
        r32 = bench_apply(P, torch, co, ce, L, torch.float32, args.steps, args.warmup, 3)
        extra["apply2d_l14_fp32"] = {"GDoF_s": r32["unique"] / (r32["launch_avg_ms"] * 1e-3) / 1e9,
                                     "GB_s": 8 * r32["unique"] / (r32["launch_avg_ms"] * 1e-3) / 1e9,
                                     "launch_avg_ms": r32["launch_avg_ms"]}
        log("apply 2D reference triangle level 8 fp64 (L2-resident)")
        r1 = bench_apply(P, torch, *W.unit_triangle(), 8, torch.float64, args.steps, args.warmup, 1)
        extra["apply2d_unit_l8_fp64"] = {"us_per_apply": r1["launch_avg_ms"] * 1e3, "dofs": r1["unique"]}
        for L3, order in ((8, "canonical"), (8, "random"), (9, "canonical")):
            log(f"apply 3D cube level {L3} fp64 ({order} vertex order)")
            mesh = W.kuhn_cube() if order == "canonical" else W.kuhn_cube("random", 5)
            r3 = bench_apply(P, torch, *mesh, L3, torch.float64, args.steps, args.warmup, 4)
            key = f"apply3d_cube_l{L3}_fp64" + ("" if order == "canonical" else "_random_order")
            extra[key] = {
                "GDoF_s": r3["unique"] / (r3["launch_avg_ms"] * 1e-3) / 1e9,
                "GB_s_storage": 16 * r3["storage"] / (r3["launch_avg_ms"] * 1e-3) / 1e9,
                "launch_avg_ms": r3["launch_avg_ms"], "storage": r3["storage"], "unique": r3["unique"]}
        for dt, bpd in ((torch.float64, 16), (torch.float32, 8)):
            tag = "fp64" if dt == torch.float64 else "fp32"
            log(f"P2 apply 2D level 13 {tag} (vertex and edge DoFs, one fused pass)")
            rp = bench_apply(P, torch, co, ce, 13, dt, args.steps, args.warmup, 3, p2=True)
            extra[f"apply2d_p2_l13_{tag}"] = {
                "GDoF_s": rp["unique"] / (rp["launch_avg_ms"] * 1e-3) / 1e9,
                "GB_s": bpd * rp["unique"] / (rp["launch_avg_ms"] * 1e-3) / 1e9,
                "launch_avg_ms": rp["launch_avg_ms"], "dofs": rp["unique"],
                "algorithmic_B_per_dof": bpd, "paper_four_kernel_B_per_dof": 2 * bpd}
        for dt, bpd in ((torch.float64, 24), (torch.float32, 12)):
            tag = "fp64" if dt == torch.float64 else "fp32"
            log(f"variable-coefficient apply 2D level 14 {tag} (weights formed on the fly)")
            rv = bench_varcoef(P, torch, co, ce, 14, dt, args.steps, args.warmup)
            extra[f"apply2d_varcoef_l14_{tag}"] = {
                "GDoF_s": rv["unique"] / (rv["launch_avg_ms"] * 1e-3) / 1e9,
                "GB_s": bpd * rv["unique"] / (rv["launch_avg_ms"] * 1e-3) / 1e9,
                "launch_avg_ms": rv["launch_avg_ms"], "dofs": rv["unique"], "algorithmic_B_per_dof": bpd}
        for dt, bpd in ((torch.float64, 24), (torch.float32, 12)):
            tag = "fp64" if dt == torch.float64 else "fp32"
            log(f"variable-coefficient apply 3D cube level 8 {tag} (weights formed on the fly)")
            rv = bench_varcoef(P, torch, *W.kuhn_cube(), 8, dt, args.steps, args.warmup)
            extra[f"apply3d_varcoef_cube_l8_{tag}"] = {
                "GDoF_s": rv["unique"] / (rv["launch_avg_ms"] * 1e-3) / 1e9,
                "GB_s_storage": bpd * rv["storage"] / (rv["launch_avg_ms"] * 1e-3) / 1e9,
                "launch_avg_ms": rv["launch_avg_ms"], "storage": rv["storage"], "unique": rv["unique"],
                "algorithmic_B_per_dof": bpd}
        log("blended (non-affine) apply 2D level 14 fp64 (element matrices formed on the fly)")
        rb = bench_blended(P, torch, co, ce, 14, args.steps, args.warmup)
        extra["apply2d_blended_l14_fp64"] = {
            "GDoF_s": rb["unique"] / (rb["launch_avg_ms"] * 1e-3) / 1e9,
            "GB_s": 16 * rb["unique"] / (rb["launch_avg_ms"] * 1e-3) / 1e9,
            "launch_avg_ms": rb["launch_avg_ms"], "dofs": rb["unique"], "algorithmic_B_per_dof": 16}
        log("device copy reference")
        cbw = copy_bandwidth(P, torch)
        extra["device_copy_GBps"] = cbw["device_copy"]
        extra["torch_copy_GBps"] = cbw["torch_copy"]
        extra["apply2d_frac_of_copy"] = achieved / cbw["device_copy"]
        roofline["measured_copy_GBps"] = round(cbw["device_copy"], 1)
        roofline["frac_of_measured_copy"] = round(achieved / cbw["device_copy"], 4)
        if not args.skip_solve:
            log("solve: mixed vs fp64, cube level 8")
            extra["solve_cube_l8"] = solve_bench(P, torch, W)

    if args.serve != "none":
        n = args.serve_n or (200 if args.serve == "capped" else 2000)
        extra[f"serving_{args.serve}"] = serve_bench(torch, args.serve, n, servers=args.serve_servers)
    cpu = None
    if not args.skip_cpu:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(W)
        if args.cpu_cube:
            log("oracle timing on the cube, level 8")
            extra["cpu_oracle_cube_l8"] = cpu_oracle_cube(W)
    line = {
        "metric": "stencil-apply GDoF/s & % HBM peak; batched-solve p50/p99 latency vs plain",
        "value": round(gdofs, 3), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D FP64 apply, one macro triangle under a seeded affine map (cond <= 10), level 14",
                   "dofs": r64["unique"], "level": L, "macros": 1},
        "roofline": roofline, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
