#!/usr/bin/env python
"""Benchmark of the nonlinear Poisson-Boltzmann FEM-BEM hot path on one MI355X.

One step = one complete solve of the large RNA-like workload (81920 triangles
per interface, 2949120 shell tets, 120 helix + 400 partial charges, kappa =
0.125) in its mixed-precision form: device setup from the resident mesh
(geometry, FEM values, Coulomb load, dense Laplace and Yukawa Galerkin
operators with FP32 evaluation of the regular pairs, FP64 touching-panel
integrals, FP32 storage), the linear solve, cubic-start Newton with the
self-adjusted relaxation factor, GMRES with an FP32 Krylov basis inside FP64
iterative refinement, and the energy.  The host-side mesh topology and the
mesh upload happen before the timed region (inputs resident in HBM).

Prints one JSON line: PB solves/s of that path (`value`), the FP64 path on
the same workload and the relative energy / surface-potential error between
them, coupled-operator GFLOP/s, step latency p50/p99, the roofline of the
dense GEMV (the dominant kernel) from HIP events, the CPU oracle baseline, and
further legs (the RNA-like 20k-triangle workload's variants, batched and
served solves).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per dense apply (k_bgemv + k_bgemv_fin, both interfaces) at the
# 80k-triangle size from two rocprofv3 --pmc runs (FETCH_SIZE x 2: the
# counter reads 0.5 x the bytes of a plain device copy; WRITE_SIZE x 1), valid
# for the row routines whose source hash is recorded with them; see
# profiles/gemv_rna80k_hbm_counters.md.
GEMV_TRAFFIC = {
    "rna80k_f32": {"src_sha256_16": "9066d2ee5bfca69e",
                   "bytes": 9868269.03 * 2048 + 207677.50 * 1024 + 157896.09 * 2048 + 1235.06 * 1024},
    "rna80k_f64": {"src_sha256_16": "9066d2ee5bfca69e",
                   "bytes": 19708630.60 * 2048 + 210751.00 * 1024 + 157896.09 * 2048 + 1235.06 * 1024},
}


def gemv_traffic_key(cfg, elem):
    return {1: "rna20k", 2: "rna80k"}.get(cfg, f"config{cfg}") + ("_f64" if elem == 8 else "_f32")
# algorithmic flops per quadrature-point pair of the regular tiles, counting
# add/mul/rsqrt/exp as 1 and FMA as 2: Laplace V and K 37, Yukawa 46
FLOPS_QP = {"laplace": 37, "yukawa": 46}
# the same for the matrix-free apply's k_mf_pot (one potential pair per
# quadrature pair): 3 sub, 5 for r^2, rsqrt, 2 mul r^-3, 2 FMA for the two
# strength sums = 15, plus the per-target-point normal distance and FP64
# accumulation (11 flops over the 6 source points) = 17; Yukawa forms the
# double-layer factor as e r^-1 r^-1 (r^-1 + kappa) instead of r^-3: r = r^2
# r^-1, the exponent (2 mul), exp, e r^-1, then add + 2 mul, in place of the
# 2 mul of r^-3 = +6
MF_FLOPS_QP = {"laplace": 17, "yukawa": 23}
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def gemv_source_hash():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2511_21713_amd", "csrc", "gemv_rows.hpp")).read()
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def regular_pairs(tri):
    """Ordered triangle pairs of one surface that share no vertex (the pairs
    the regular 6 x 6 rule integrates)."""
    import numpy as np
    import scipy.sparse as sp
    nt = tri.shape[0]
    T = sp.csr_matrix((np.ones(3 * nt), (np.repeat(np.arange(nt), 3), tri.ravel())))
    return nt * nt - (T @ T.T).nnz


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def gemv_bytes(nm, ns, elem, sym=False):
    # algorithmic bytes of one dense apply: both [K'|V'] operators (n x 2n),
    # their packed FP64 inputs (2n) and FP64 outputs (n).  With the symmetric
    # use of the stored single layer (square-tile assembly) only K' and the
    # lower triangle of V' with its diagonal are read (the sparse Delta rows,
    # ~0.1 % of the bytes, are left out)
    if sym:
        return sum(n * n * elem + n * (n + 1) // 2 * elem + 2 * n * 8 + n * 8 for n in (nm, ns))
    return sum(n * 2 * n * elem + 2 * n * 8 + n * 8 for n in (nm, ns))


def fem_nnz(prob):
    """Nonzeros of the FEM block rows: node pairs sharing a tet, plus the
    coupling columns of each interface node (its surface 1-ring)."""
    import scipy.sparse as sp
    nn = prob.nodes.shape[0]
    T = prob.tets
    r = np.repeat(T, 4, axis=1).ravel()
    c = np.tile(T, (1, 4)).ravel()
    nnz = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(nn, nn)).tocsr().nnz
    for tri in (prob.tri_m, prob.tri_s):
        r = np.repeat(tri, 3, axis=1).ravel()
        c = np.tile(tri, (1, 3)).ravel()
        nnz += sp.coo_matrix((np.ones(r.size), (r, c)), shape=(nn, nn)).tocsr().nnz
    return nnz


def spmv_bytes(nnz, nn, n, elem):
    # algorithmic bytes of one FEM SpMV launch: values and 32-bit columns of
    # the nonzeros, the FP64 input vector (all unknowns) once, FP64 output rows
    return nnz * (elem + 4) + n * 8 + nn * 8


def apply_flops(nm, ns, nnz):
    return 2 * (nm * 2 * nm + ns * 2 * ns) + 2 * nnz


def run_leg(pb, torch, prob, precision, steps, warmup, opts, label, bem_mode=None, potential=True, time_energy=False):
    ctx = pb.Context(0)
    g = pb.Problem.from_inputs(ctx, prob, precision=precision)
    if bem_mode is not None:
        g.set_bem_mode(bem_mode)
    t0 = time.perf_counter()
    g.setup()
    progress(f"{label}: first setup (topology + upload + assembly) {time.perf_counter() - t0:.2f} s, "
             f"device bytes {g.hbm() / 1e9:.2f} GB")
    for w in range(warmup):
        g.reset_operators()
        r = g.solve(**opts)
        progress(f"{label}: warmup {w}: total {r['total']:.6f} kcal/mol, newton {r['newton_iters']}, "
                 f"gmres {r['gmres_iters_total']}, status {r['status']}, {r['t_setup_s'] + r['t_solve_s']:.3f} s")
    g.timing_enable(True)
    g.timing(0, reset=True)
    lat, res = [], None
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        g.reset_operators()
        res = g.solve(**opts)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        progress(f"{label}: step {k}: {lat[-1]:.3f} s (setup {res['t_setup_s']:.3f}, solve {res['t_solve_s']:.3f}), "
                 f"newton {res['newton_iters']}, gmres {res['gmres_iters_total']}, total {res['total']:.8f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    tm = {name: g.timing(i) for i, name in enumerate(["apply", "gemv", "spmv", "assembly", "singular", "precond"])}
    # Batched GMRES launches its kernels for every iteration of the batch; an
    # instance between cycles or already converged returns at once.  Per-launch
    # figures below divide the summed time by the launches that did work.
    real = res["applies"] * steps
    for name in ("apply", "gemv", "spmv"):
        ms, cnt = tm[name]
        tm[name] = (ms * cnt / real if real else 0.0, real)
    g.timing_enable(False)
    u_m = None
    if potential:
        # one more solve outside the timed region for the potential on Gamma_m
        phi = torch.zeros(2 * g.n, dtype=torch.float64, device="cuda")
        g.solve(phi_out=phi, **opts)
        torch.cuda.synchronize()
        if time_energy:  # the energy entry point alone (two-field form: with the lambda_m recovery)
            te = []
            for _ in range(3):
                t0 = time.perf_counter()
                g.energy(phi[:g.n], phi[g.n:])
                torch.cuda.synchronize()
                te.append(time.perf_counter() - t0)
            energy_ms = 1e3 * min(te)
        phi = phi.cpu().numpy()
        u_m = (phi[:g.n] + phi[g.n:])[np.unique(prob.tri_m)]
    tiles = {"laplace_gamma_m": list(g.tile_shape(0)), "yukawa_gamma_s": list(g.tile_shape(1))}
    out = dict(elapsed=elapsed, lat=lat, res=res, timing=tm, n=g.n, n_m=g.n_m, n_s=g.n_s, hbm=g.hbm(), u_m=u_m,
               tiles=tiles, steps=steps)
    if potential and time_energy:
        out["energy_ms"] = energy_ms
    g.close()
    ctx.close()
    return out


def batch_leg(pb, torch, count, steps, precision):
    """Batched workload: `count` instances of the sphere-type and RNA-type
    generators (triangles log-uniform over 320..38720, 4..60 helix charges,
    kappa ~ U(0.03, 0.33)) solved by one pbfb_solve_batch per step, setup
    included (operators reset before each step)."""
    import pbgen
    t0 = time.perf_counter()
    probs = [pbgen.batch_instance(3, i) for i in range(count)]
    progress(f"batch: generated {count} instances in {time.perf_counter() - t0:.1f} s "
             f"({sum(p.tri_m.shape[0] for p in probs)} triangles per interface in total)")
    ctx = pb.Context(0)
    gs = [pb.Problem.from_inputs(ctx, p, precision=precision) for p in probs]
    code, res = pb.solve_batch(ctx, gs)  # warm-up: topology, uploads, first assembly
    walls, lat = [], []
    for k in range(steps):
        for g in gs:
            g.reset_operators()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        code, res = pb.solve_batch(ctx, gs)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - ts)
        lat += [r["t_setup_s"] + r["t_solve_s"] for r in res]
        if code != 0:
            raise RuntimeError(f"batched solve failed with status {code}: {pb.last_error()}")
        progress(f"batch: step {k}: {walls[-1]:.3f} s for {count} solves, status {code}, "
                 f"newton {[r['newton_iters'] for r in res][:8]}...")
    for g in gs:
        g.close()
    ctx.close()
    wall = sum(walls) / len(walls)
    return {"instances": count, "precision": "mixed" if precision == pb.MIXED else "fp64", "wall_s": wall,
            "value": count / wall, "unit": "PB solves/s",
            "completion_s": {"p50": percentile(lat, 0.5), "p99": percentile(lat, 0.99)},
            "status": code}


def _serve_instance(args):
    import pbgen
    return pbgen.serve_instance(args[0], n_hi=args[1])


def serve_requests(count, nmax):
    """The serving stream's requests, generated on the host before any GPU
    work (a long stream is generated by a pool of forked workers)."""
    t0 = time.perf_counter()
    work = [(i, nmax) for i in range(count)]
    if count > 64:
        import multiprocessing as mp
        probs = []
        with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
            for p in pool.imap(_serve_instance, work, chunksize=4):
                probs.append(p)
                if len(probs) % 250 == 0:
                    progress(f"serve: {len(probs)} of {count} requests generated")
    else:
        probs = [_serve_instance(w) for w in work]
    tris = sorted(p.tri_m.shape[0] for p in probs)
    progress(f"serve: generated {count} requests in {time.perf_counter() - t0:.1f} s, triangles per interface "
             f"{tris[0]}..{tris[-1]} (median {tris[len(tris) // 2]})")
    return probs


def serve_leg(pb, torch, probs, nmax, precision, loads=(0.5, 0.8, 1.0), seed=0, budget=None, slots=16):
    """Serving workload: the requests `probs` (RNA-like generator with its
    partial charges, triangles log-uniform over 320..20 n_max^2, random kappa)
    arriving as a Poisson process at `load` x the measured service rate,
    submitted to a continuous-batching server with an HBM budget that binds
    (requests wait for admission); latency = submit to completion, admission
    wait = submit to admission.  The service rate is the mean solo solve time
    of every fifth request (of about 40 evenly spaced ones in a long stream;
    setup included).  Default budget: 1.1 x the largest request's footprint
    (steady + setup workspace, taken over the 8 largest meshes), so that a
    large request waits for the running ones and the budget binds."""
    import numpy as np

    count = len(probs)
    ctx = pb.Context(0)
    if budget is None:
        # the footprint grows with the mesh: the largest requests set the budget
        big = sorted(probs, key=lambda p: (p.tri_m.shape[0], p.tets.shape[0]))[-8:]
        fps = []
        for p in big:
            g = pb.Problem.from_inputs(ctx, p, precision=precision)
            fps.append(sum(g.footprint()))
            g.close()
        budget = int(1.1 * max(fps))
    svc = []
    for p in probs[::max(5, count // 40)]:
        g = pb.Problem.from_inputs(ctx, p, precision=precision)
        g.solve()
        g.reset_operators()
        ts = time.perf_counter()
        g.solve()
        svc.append(time.perf_counter() - ts)
        g.close()
    out = {}
    prec = "mixed" if precision == pb.MIXED else "fp64"
    for load in loads:
        rate = load / (sum(svc) / len(svc))
        rng = np.random.default_rng([4, seed])
        gaps = rng.exponential(1.0 / rate, size=count)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        low = free0
        srv = pb.Server(ctx, hbm_budget_bytes=budget, max_slots=slots)
        t0 = time.perf_counter()
        gs = []
        for p in probs:
            gs.append(pb.Problem.from_inputs(ctx, p, precision=precision))
            if count > 100 and len(gs) % 250 == 0:
                progress(f"serve ({prec}, load {load}): {len(gs)} problems set up")
        progress(f"serve ({prec}, load {load}): {count} problems set up on the host in "
                 f"{time.perf_counter() - t0:.1f} s")
        submit, done, res = {}, {}, {}
        tickets, rejected = [], 0
        start = time.perf_counter()
        next_t = start
        i = 0
        while len(done) < len(tickets) or i < count:
            now = time.perf_counter()
            while i < count and now >= next_t:
                try:
                    t = srv.submit(gs[i])
                    tickets.append(t)
                    submit[t] = time.perf_counter()
                except pb.PbfbError as e:
                    if e.code != pb.ENOMEM:
                        raise
                    rejected += 1
                next_t += gaps[i]
                i += 1
            for t in tickets:
                if t not in done:
                    r = srv.poll(t)
                    if r is not None:
                        done[t] = time.perf_counter()
                        res[t] = r
                        if count > 100 and len(done) % 200 == 0:
                            progress(f"serve ({prec}, load {load}): {len(done)} of {count} requests done")
            low = min(low, torch.cuda.mem_get_info()[0])
            time.sleep(0.0005)
        makespan = time.perf_counter() - start
        srv.close()
        for g in gs:
            g.close()
        lat = [done[t] - submit[t] for t in tickets]
        waits = [res[t]["t_wait_s"] for t in tickets]
        bad = sum(1 for t in tickets if res[t]["status"] != 0)
        if bad:
            raise RuntimeError(f"{bad} served requests failed")
        progress(f"serve ({prec}, load {load}): {len(tickets)} requests in {makespan:.2f} s, p50 "
                 f"{percentile(lat, 0.5):.3f} s, p99 {percentile(lat, 0.99):.3f} s, admission wait p99 "
                 f"{percentile(waits, 0.99):.3f} s, peak device use {(free0 - low) / 2**30:.1f} GiB, {rejected} rejected")
        out[f"load_{load}"] = {"arrival_rate_per_s": rate, "load": load, "value": len(tickets) / makespan,
                               "unit": "PB solves/s",
                               "latency_s": {"p50": percentile(lat, 0.5), "p99": percentile(lat, 0.99)},
                               "admission_wait_s": {"p50": percentile(waits, 0.5), "p99": percentile(waits, 0.99),
                                                    "waited": sum(1 for w in waits if w > 1e-3)},
                               "peak_device_bytes": free0 - low, "failures": bad,
                               "rejected_over_budget": rejected}
    ctx.close()
    main = out["load_0.8"] if "load_0.8" in out else next(iter(out.values()))
    return dict(main, requests=count, precision=prec, max_triangles=int(max(p.tri_m.shape[0] for p in probs)),
                hbm_budget_bytes=budget, max_slots=slots, solo_service_s=sum(svc) / len(svc), by_load=out)


def host_info():
    """CPU model, logical CPUs and memory of the host the bench runs on."""
    model, mem = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem = float(line.split()[1]) * 1024 / 2**30
                break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "mem_gib": mem}


def cpu_baseline(prob, applies_per_solve, seed=0, budget_s=12.0):
    """The oracle timed on a bounded sample of the same workload and
    extrapolated to one solve (labelled so): sampled dense Galerkin rows of
    both interfaces (assembly), the oracle's dense row products on those rows,
    and its matrix-free FEM Jacobian product; solve time = assembly of every
    row + applies_per_solve (the GPU FP64 run's count) x (dense rows + FEM
    product).  Measured with all host threads and with one."""
    import numpy as np

    import oracle
    o = oracle.Oracle.from_problem(prob)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(o.n)
    all_threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {}
    for label, threads in (("all", all_threads), ("one", 1)):
        oracle.set_threads(threads)
        nrows = max(2, 2 * threads) if prob.tri_m.shape[0] > 40000 else 8 * threads
        t_asm = t_dense = 0.0
        for surf, nv in ((0, o.n_m), (1, o.n_s)):
            rows = np.sort(rng.choice(nv, size=nrows, replace=False))
            t0 = time.perf_counter()
            V, K = o.bem_rows(surf, rows)
            t_asm += (time.perf_counter() - t0) * nv / nrows
            reps = 5
            t0 = time.perf_counter()
            for _ in range(reps):
                o.dense_rows_apply(surf, V, K, x)
            t_dense += (time.perf_counter() - t0) / reps * nv / nrows
        t0 = time.perf_counter()
        o.fem_jacobian(oracle.HS, x, x)
        t_fem = time.perf_counter() - t0
        t_solve = t_asm + applies_per_solve * (t_dense + t_fem)
        out[label] = dict(threads=int(threads), rows_per_interface=int(nrows), t_assembly_s=t_asm,
                          t_dense_apply_s=t_dense, t_fem_product_s=t_fem, t_solve_s=t_solve)
    oracle.set_threads(all_threads)
    a, one = out["all"], out["one"]
    sample = (f"extrapolated: {a['rows_per_interface']} Galerkin rows per interface assembled by the oracle, their "
              f"dense row products x5, 1 FEM Jacobian product, scaled to one solve = assembly of every row + "
              f"{applies_per_solve} coupled applies (the GPU FP64 run's count); {a['threads']} threads: assembly "
              f"{a['t_assembly_s']:.1f} s, dense apply {a['t_dense_apply_s']:.3f} s, FEM product "
              f"{a['t_fem_product_s'] * 1e3:.1f} ms; 1 thread: {1.0 / one['t_solve_s']:.3g} solves/s")
    return dict(value=1.0 / a["t_solve_s"], unit="PB solves/s", cores=a["threads"], kind="oracle", sample=sample,
                extrapolated=True, single_core={"value": 1.0 / one["t_solve_s"], "unit": "PB solves/s",
                                                "t_solve_s": one["t_solve_s"]},
                host=host_info(), detail=out)


def leg_summary(leg, K, ref=None, u_ref=None):
    r = leg["res"]
    d = {"value": K / leg["elapsed"], "unit": "PB solves/s", "steps": K, "ms_per_step": 1e3 * leg["elapsed"] / K,
         "latency_s": {"p50": percentile(leg["lat"], 0.5), "p99": percentile(leg["lat"], 0.99)},
         "total_kcal_mol": r["total"], "lc": r["lc"], "nc": r["nc"], "dg_omega_i": r["dg_omega_i"],
         "newton_iters": r["newton_iters"], "gmres_iters_total": r["gmres_iters_total"], "omega": r["omega"],
         "coupled_applies_per_solve": r["applies"], "device_bytes": leg["hbm"], "status": r["status"],
         "setup_s": r["t_setup_s"], "solve_s": r["t_solve_s"]}
    if ref is not None:
        d["rel_err_vs_fp64"] = {k: abs(r[k] - ref[k]) / abs(ref[k]) for k in ("total", "lc", "nc", "dg_omega_i")}
    if u_ref is not None and leg["u_m"] is not None:
        d["surface_potential_rel_err_vs_fp64"] = float(np.linalg.norm(leg["u_m"] - u_ref) / np.linalg.norm(u_ref))
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2,
                    help="workload of the headline line: 2 = large RNA-like (mixed precision, the default), "
                         "1 = RNA-like (FP64), 0 = charged sphere (FP64)")
    ap.add_argument("--cmp-steps", type=int, default=5, help="timed steps of the comparison legs at the workload")
    ap.add_argument("--side-config", type=int, default=1, help="workload of the variant legs (Picard, schedules, "
                                                               "root finders, matrix-free, two-field)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-picard", action="store_true", help="skip the Picard comparison leg")
    ap.add_argument("--no-matrix-free", action="store_true", help="skip the matrix-free boundary-element leg")
    ap.add_argument("--no-schemes", action="store_true", help="skip the Taylor-schedule comparison leg")
    ap.add_argument("--no-two-field", action="store_true", help="skip the two-field form leg")
    ap.add_argument("--no-side", action="store_true", help="skip every variant leg")
    ap.add_argument("--batch", type=int, default=32, help="instances of the batched leg (0: skip)")
    ap.add_argument("--serve", type=int, default=40, help="requests of the serving leg (0: skip)")
    ap.add_argument("--serve-nmax", type=int, default=64, help="largest icosphere frequency of served requests")
    ap.add_argument("--serve-budget-gb", type=float, default=0.0,
                    help="HBM budget of the serving leg (0: 1.1 x the largest request's footprint)")
    ap.add_argument("--serve-loads", type=str, default="0.5,0.8,1.0")
    ap.add_argument("--serve-precisions", type=str, default="mixed,fp64",
                    help="precisions of the serving leg (the FP64 one at load 0.8)")
    ap.add_argument("--calib-copy-gb", type=float, default=0.0,
                    help="run one device copy of this size first (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU row-block sharding is a design, not built)", file=sys.stderr)
        sys.exit(2)
    reqs = serve_requests(args.serve, args.serve_nmax) if args.serve > 0 else None
    import torch

    import paper_2511_21713_amd as pb
    import pbgen
    assert torch.cuda.is_available()
    if args.calib_copy_gb > 0:
        n = int(args.calib_copy_gb * 1e9 / 8)
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        progress(f"calibration copy of {n * 8 / 1e9:.3f} GB done")
    K = args.steps
    cfg = args.config
    t0 = time.perf_counter()
    prob = pbgen.make_config(cfg)
    progress(f"generated workload {cfg} in {time.perf_counter() - t0:.1f} s: {prob.nodes.shape[0]} nodes, "
             f"{prob.tets.shape[0]} tets, {prob.tri_m.shape[0]} triangles per interface, {prob.q_z.size} charges")
    base_opts = dict()  # cubic start, self-adjusted omega, App. B settings (library defaults)
    if cfg == 0:
        base_opts = dict(omega_auto=0, omega_fixed=0.5)
    mixed_head = cfg == 2 and not args.no_mixed
    head_prec = pb.MIXED if mixed_head else pb.FP64
    head_opts = dict(base_opts, krylov_fp32=1) if mixed_head else dict(base_opts)
    head = run_leg(pb, torch, prob, head_prec, K, args.warmup, head_opts,
                   "mixed (fp32 krylov basis)" if mixed_head else "fp64")
    if mixed_head:
        f64 = run_leg(pb, torch, prob, pb.FP64, args.cmp_steps, 1, base_opts, "fp64")
    else:
        f64 = head
    res64 = f64["res"]
    nm, ns = head["n_m"], head["n_s"]
    elem = 4 if mixed_head else 8
    gemv_ms, gemv_cnt = head["timing"]["gemv"]
    apply_ms, apply_cnt = head["timing"]["apply"]
    sym = all(a == b for a, b in head["tiles"].values())  # square tiles: symmetric use of V'
    gb = gemv_bytes(nm, ns, elem, sym)
    achieved = gb / (gemv_ms * 1e-3) / 1e9 if gemv_ms else None
    res = head["res"]
    nnz = fem_nnz(prob)
    nn = prob.nodes.shape[0]
    flops = apply_flops(nm, ns, nnz)
    sym_tiles = all(a == b for a, b in f64["tiles"].values())
    kname = ("k_bgemv + k_bgemv_fin / k_gemv + k_gemv_fin (gemv_rows_symK / gemv_rows_symV work items: K' and "
             f"the lower triangle of V', {'FP32' if elem == 4 else 'FP64'} storage, FP64 accumulation, both "
             "interfaces)" if sym else
             f"k_bgemv / k_gemv (gemv_rows: dense [K'|V'] {'FP32' if elem == 4 else 'FP64'} GEMV, both interfaces)")
    tkey = gemv_traffic_key(cfg, elem)
    workload = (f"RNA-like solute, large: {prob.tri_m.shape[0]} triangles per interface, {prob.tets.shape[0]} shell "
                f"tets, {prob.q_z.size} charges, kappa {prob.kappa}; " if cfg == 2 else
                f"RNA-like solute: {prob.tri_m.shape[0]} triangles per interface, {prob.tets.shape[0]} shell tets, "
                f"{prob.q_z.size} charges, kappa {prob.kappa}; " if cfg == 1 else
                f"charged sphere: {prob.tri_m.shape[0]} triangles per interface, {prob.tets.shape[0]} shell tets; ")
    workload += ("mixed precision (FP32 BEM evaluation and storage, FP32 FEM values, FP64 accumulation; GMRES with "
                 "an FP32 Krylov basis inside FP64 iterative refinement); cubic-start Newton with self-adjusted "
                 "relaxation" if mixed_head else "FP64; cubic-start Newton with self-adjusted relaxation")
    out = {
        "metric": "PB solves/s + coupled-operator GFLOP/s, mixed vs FP64 at <=1e-5 rel energy; p50/p99",
        "value": K / head["elapsed"],
        "unit": "PB solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * head["elapsed"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64 mixed" if mixed_head else "f64",
        "data": "synthetic",
        "config": {"workload": workload, "unknowns": head["n"], "parallelism": "single GPU"},
        "latency_s": {"p50": percentile(head["lat"], 0.5), "p99": percentile(head["lat"], 0.99)},
        "solve": {"total_kcal_mol": res["total"], "lc": res["lc"], "nc": res["nc"], "dg_omega_i": res["dg_omega_i"],
                  "newton_iters": res["newton_iters"], "gmres_iters_total": res["gmres_iters_total"],
                  "omega": res["omega"], "status": res["status"], "coupled_applies_per_solve": res["applies"],
                  "device_bytes": head["hbm"]},
        "kernel_ms": {"gemv": gemv_ms, "coupled_apply": apply_ms},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": (GEMV_TRAFFIC[tkey]["bytes"] if tkey in GEMV_TRAFFIC and
                                 gemv_source_hash() == GEMV_TRAFFIC[tkey]["src_sha256_16"] else None),
                     "bytes_per_launch": gb},
    }
    if mixed_head:
        out["rel_energy_err_vs_fp64"] = abs(res["total"] - res64["total"]) / abs(res64["total"])
        out["surface_potential_rel_err_vs_fp64"] = float(np.linalg.norm(head["u_m"] - f64["u_m"]) /
                                                         np.linalg.norm(f64["u_m"]))
        out["fp64"] = leg_summary(f64, args.cmp_steps)
        g64_ms = f64["timing"]["gemv"][0]
        gb64 = gemv_bytes(nm, ns, 8, all(a == b for a, b in f64["tiles"].values()))
        t64 = gemv_traffic_key(cfg, 8)
        out["fp64"]["gemv"] = {"ms": g64_ms, "bytes_per_launch": gb64,
                               "traffic": (GEMV_TRAFFIC[t64]["bytes"] if t64 in GEMV_TRAFFIC and
                                           gemv_source_hash() == GEMV_TRAFFIC[t64]["src_sha256_16"] else None),
                               "achieved_gbs": gb64 / (g64_ms * 1e-3) / 1e9 if g64_ms else None,
                               "frac": gb64 / (g64_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if g64_ms else None}
        out["mixed_speedup_vs_fp64"] = out["value"] / out["fp64"]["value"]
        # the same mixed path with an FP64 Krylov basis
        mx64 = run_leg(pb, torch, prob, pb.MIXED, args.cmp_steps, 1, base_opts, "mixed (fp64 krylov basis)")
        out["mixed_fp64_krylov"] = leg_summary(mx64, args.cmp_steps, res64, f64["u_m"])
        out["mixed_fp64_krylov"]["coupled_operator_gflops"] = (flops / (mx64["timing"]["apply"][0] * 1e-3) / 1e9
                                                               if mx64["timing"]["apply"][0] else None)

    # regular BEM tiles: algorithmic flops per solve over the HIP-event time
    # of the tile launches (both interfaces; touching pairs excluded)
    asm_flops = 36 * (FLOPS_QP["laplace"] * regular_pairs(prob.tri_m) +
                      FLOPS_QP["yukawa" if prob.kappa > 0 else "laplace"] * regular_pairs(prob.tri_s))

    def asm_report(leg, peak, steps):
        ms, cnt = leg["timing"]["assembly"]
        t = ms * cnt / steps * 1e-3
        return {"kernel": "k_bem_regular (6 x 6 rule, non-touching pairs)", "tile_shapes_autotuned": leg["tiles"],
                "flops_per_solve": asm_flops,
                "ms_per_solve": t * 1e3, "tflops": asm_flops / t / 1e12 if t else None, "peak_tflops": peak,
                "frac": asm_flops / t / 1e12 / peak if t else None}

    def spmv_report(leg, e):
        ms, cnt = leg["timing"]["spmv"]
        b = spmv_bytes(nnz, nn, leg["n"], e)
        gbs = b / (ms * 1e-3) / 1e9 if ms else None
        return {"kernel": "k_bspmv / k_spmv (sell_part: sliced-ELL FEM rows)", "bound": "hbm",
                "bytes_per_launch": b, "working_set_bytes": b, "ms_per_launch": ms, "launches": cnt,
                "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS if gbs else None,
                "nnz": nnz, "value_bytes": e,
                "cache_note": (f"each launch follows the dense apply of the same coupled apply, which streams "
                               f"{gemv_bytes(nm, ns, e, sym_tiles) / 1e9:.1f} GB through the 256 MB "
                               f"Infinity Cache")}

    out["bem_assembly"] = {"fp64": asm_report(f64, FP64_PEAK_TFLOPS, f64["steps"])}
    out["fem_spmv"] = {"fp64": spmv_report(f64, 8)}
    out["kernel_ms"]["precond_per_solve"] = head["timing"]["precond"][0] * head["timing"]["precond"][1] / K
    if apply_ms:
        out["coupled_operator_gflops"] = flops / (apply_ms * 1e-3) / 1e9
    if f64["timing"]["apply"][0]:
        out["coupled_operator_gflops_fp64"] = flops / (f64["timing"]["apply"][0] * 1e-3) / 1e9
    if mixed_head:
        out["bem_assembly"]["mixed_fp32_eval"] = asm_report(head, FP32_PEAK_TFLOPS, K)
        out["fem_spmv"]["mixed_fp32_values"] = spmv_report(head, 4)
    elif not args.no_mixed:
        mx = run_leg(pb, torch, prob, pb.MIXED, args.cmp_steps, 1, dict(base_opts, krylov_fp32=1), "mixed")
        out["mixed"] = leg_summary(mx, args.cmp_steps, res64, f64["u_m"])
        out["bem_assembly"]["mixed_fp32_eval"] = asm_report(mx, FP32_PEAK_TFLOPS, args.cmp_steps)
        out["fem_spmv"]["mixed_fp32_values"] = spmv_report(mx, 4)
    cpu_applies = max(res64["applies"], 1)

    if not args.no_side:
        side_legs(pb, torch, pbgen, args, out)
    if args.batch > 0:
        out["batched"] = {"mixed": batch_leg(pb, torch, args.batch, 1, pb.MIXED),
                          "fp64": batch_leg(pb, torch, args.batch, 1, pb.FP64)}
    if args.serve > 0:
        loads = tuple(float(x) for x in args.serve_loads.split(","))
        bud = int(args.serve_budget_gb * 2**30) if args.serve_budget_gb > 0 else None
        out["serving"] = {}
        if "mixed" in args.serve_precisions:
            out["serving"]["mixed"] = serve_leg(pb, torch, reqs, args.serve_nmax, pb.MIXED, loads, budget=bud)
        if "fp64" in args.serve_precisions:
            out["serving"]["fp64"] = serve_leg(pb, torch, reqs, args.serve_nmax, pb.FP64, (0.8,), budget=bud)
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle, bounded sample, extrapolated)")
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(prob, cpu_applies)
        progress(f"cpu baseline took {time.perf_counter() - t0:.1f} s")
    print(json.dumps(out), flush=True)


def side_legs(pb, torch, pbgen, args, out):
    """Variants of the method on the RNA-like 20k-triangle workload, each
    compared with an FP64 Newton solve of that workload."""
    cfg = args.side_config
    prob = pbgen.make_config(cfg)
    opts = dict(omega_auto=0, omega_fixed=0.5) if cfg == 0 else dict()
    base = run_leg(pb, torch, prob, pb.FP64, 3, 1, opts, f"side fp64 (workload {cfg})")
    res = base["res"]
    side = {"workload": f"RNA-like solute (config {cfg}): {prob.tri_m.shape[0]} triangles per interface, "
                        f"{prob.tets.shape[0]} shell tets, {prob.q_z.size} charges",
            "fp64_newton": leg_summary(base, 3)}
    value = side["fp64_newton"]["value"]
    if not args.no_picard:
        # the paper's comparison path: Picard (A Delta = d) with the direct-secant
        # relaxation search and the norm-ratio reuse rule, omega in [0, 1]
        popts = dict(opts, nonlinear_method=pb.PICARD, omega_method=pb.OMEGA_BSEC_DF, omega_max=1.0, l_e=0.0,
                     max_newton=200)
        pc = run_leg(pb, torch, prob, pb.FP64, 1, 0, popts, "picard")
        rp = pc["res"]
        side["picard_fp64"] = {"value": 1.0 / pc["elapsed"], "unit": "PB solves/s", "ms_per_step": 1e3 * pc["elapsed"],
                               "nonlinear_iters": rp["newton_iters"], "gmres_iters_total": rp["gmres_iters_total"],
                               "total_kcal_mol": rp["total"],
                               "rel_energy_diff_vs_newton": abs(rp["total"] - res["total"]) / abs(res["total"]),
                               "newton_iters": res["newton_iters"], "status": rp["status"]}
    if not args.no_schemes:
        sch = {}
        for label, sched in (("T3-T5-HS", [pb.T3, pb.T5]), ("T3-T5-T7-T7-HS", [pb.T3, pb.T5, pb.T7, pb.T7])):
            lg = run_leg(pb, torch, prob, pb.FP64, 2, 0, dict(opts, schedule=sched), f"schedule {label}",
                         potential=False)
            r = lg["res"]
            sch[label] = {"value": 2 / lg["elapsed"], "unit": "PB solves/s", "ms_per_step": 1e3 * lg["elapsed"] / 2,
                          "newton_iters": r["newton_iters"], "gmres_iters_total": r["gmres_iters_total"],
                          "omega": r["omega"], "total_kcal_mol": r["total"],
                          "rel_energy_diff_vs_t3_hs": abs(r["total"] - res["total"]) / abs(res["total"]),
                          "status": r["status"]}
        sch["T3-HS"] = {"value": value, "newton_iters": res["newton_iters"], "gmres_iters_total": res["gmres_iters_total"]}
        side["scheme_schedules_fp64"] = sch
        om = {}
        for label, m in (("bisection", pb.OMEGA_BISECT), ("secant", pb.OMEGA_SECANT),
                         ("bisection_then_secant", pb.OMEGA_BSEC), ("newton_bisection_secant_start", pb.OMEGA_NEWTON_BS)):
            lg = run_leg(pb, torch, prob, pb.FP64, 2, 0, dict(opts, omega_method=m), f"omega {label}", potential=False)
            r = lg["res"]
            om[label] = {"value": 2 / lg["elapsed"], "unit": "PB solves/s", "ms_per_step": 1e3 * lg["elapsed"] / 2,
                         "newton_iters": r["newton_iters"], "fd_evaluations_after_the_first": r["omega_iters"],
                         "omega": r["omega"], "rel_energy_diff_vs_newton": abs(r["total"] - res["total"]) / abs(res["total"]),
                         "status": r["status"]}
        om["newton"] = {"value": value, "newton_iters": res["newton_iters"], "omega": res["omega"]}
        side["omega_root_finders_fp64"] = om
    if not args.no_matrix_free:
        # nothing dense stored: every coupled apply evaluates the regular
        # quadrature-point pairs of both interfaces again (k_mf_pot)
        mf_flops = 36 * (MF_FLOPS_QP["laplace"] * regular_pairs(prob.tri_m) +
                         MF_FLOPS_QP["yukawa" if prob.kappa > 0 else "laplace"] * regular_pairs(prob.tri_s))
        mf = {}
        for name, prec, peak in (("fp64", pb.FP64, FP64_PEAK_TFLOPS), ("mixed_fp32_eval", pb.MIXED, FP32_PEAK_TFLOPS)):
            if prec == pb.MIXED and args.no_mixed:
                continue
            lg = run_leg(pb, torch, prob, prec, 1, 0, opts, f"matrix-free {name}", bem_mode=pb.BEM_MATRIX_FREE,
                         potential=False)
            r = lg["res"]
            ams, acnt = lg["timing"]["gemv"]
            mf[name] = {"value": 1.0 / lg["elapsed"], "unit": "PB solves/s", "ms_per_step": 1e3 * lg["elapsed"],
                        "device_bytes": lg["hbm"], "newton_iters": r["newton_iters"],
                        "gmres_iters_total": r["gmres_iters_total"], "coupled_applies": r["applies"],
                        "total_kcal_mol": r["total"],
                        "rel_energy_diff_vs_dense_fp64": abs(r["total"] - res["total"]) / abs(res["total"]),
                        "bem_apply_ms": ams, "bem_apply_flops": mf_flops,
                        "flops_per_quadrature_pair": MF_FLOPS_QP,
                        "tflops": mf_flops / (ams * 1e-3) / 1e12 if ams else None, "peak_tflops": peak,
                        "frac": mf_flops / (ams * 1e-3) / 1e12 / peak if ams else None, "status": r["status"]}
        mf["dense_fp64_device_bytes"] = base["hbm"]
        side["matrix_free"] = mf
    if not args.no_two_field:
        # the paper's two-field form on the same surfaces: FEM also fills the
        # solute (three inner copies of Gamma_m, then coarsening layers), the
        # charges load the FEM rows, lambda_m is recovered for the energy
        ptf = pbgen.make_config(cfg, solute_layers=3)
        tf = {"solute_tets": int(ptf.n_tets_m), "shell_tets": int(len(ptf.tets) - ptf.n_tets_m)}
        for name, prec in (("fp64", pb.FP64), ("mixed", pb.MIXED)):
            if prec == pb.MIXED and args.no_mixed:
                continue
            lg = run_leg(pb, torch, ptf, prec, 2, 1, opts, f"two-field {name}", time_energy=True)
            r = lg["res"]
            tf[name] = {"value": 2 / lg["elapsed"], "unit": "PB solves/s", "ms_per_step": 1e3 * lg["elapsed"] / 2,
                        "n_unknowns": lg["n"], "newton_iters": r["newton_iters"],
                        "gmres_iters_total": r["gmres_iters_total"], "total_kcal_mol": r["total"],
                        "energy_with_lambda_m_recovery_ms": lg["energy_ms"],
                        "rel_energy_diff_vs_shell_only_fp64": abs(r["total"] - res["total"]) / abs(res["total"]),
                        "status": r["status"]}
        side["two_field"] = tf
    out["variants"] = side


if __name__ == "__main__":
    main()
