#!/usr/bin/env python
"""Benchmark of the nonlinear Poisson-Boltzmann FEM-BEM hot path on one MI355X.

One step = one complete solve of the RNA-like workload (20480 triangles per
interface, 614400 shell tets, 48 helix + 400 partial charges, kappa = 0.125):
device setup from the resident mesh (geometry, FEM values, Coulomb load, dense
Laplace and Yukawa Galerkin operators with touching-panel integrals), the
linear solve, cubic-start Newton with the self-adjusted relaxation factor,
and the energy.  The host-side mesh topology and the mesh upload happen
before the timed region (inputs resident in HBM).

Prints one JSON line: PB solves/s (FP64 path, the workload's precision),
coupled-operator GFLOP/s, step latency p50/p99, the mixed-precision leg and
its energy error against the FP64 path, the roofline of the dense GEMV (the
dominant kernel) from HIP events, and the CPU oracle baseline.
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

# HBM bytes per launch of k_gemv_f64 on this workload from the two rocprofv3
# --pmc runs (FETCH_SIZE then WRITE_SIZE, each scaled by the factor the same
# counter reads for a copy of known size), valid for the kernel source whose
# hash is recorded with it; see profiles/gemv_f64_rna20k_hbm_counters.md.
GEMV_TRAFFIC = {"config": 1, "src_sha256_16": "d9c2eb2ba90cdfa6", "bytes": 2.53424e9 + 7.9254e7 + 5.3112e7}
# algorithmic flops per quadrature-point pair of the regular tiles, counting
# add/mul/rsqrt/exp as 1 and FMA as 2: Laplace V and K 37, Yukawa 46
FLOPS_QP = {"laplace": 37, "yukawa": 46}
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
               tiles=tiles)
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


def serve_requests(count, nmax):
    import pbgen
    t0 = time.perf_counter()
    probs = [pbgen.serve_instance(i, n_hi=nmax) for i in range(count)]
    progress(f"serve: generated {count} requests in {time.perf_counter() - t0:.1f} s")
    return probs


def serve_leg(pb, torch, probs, nmax, precision, loads=(0.5, 0.8, 1.0), seed=0):
    """Serving workload: the requests `probs` (config-1 generator, triangles
    log-uniform over 320..20 n_max^2, random kappa) arriving as a Poisson
    process at `load` x the measured single-request service rate, submitted
    to a continuous-batching server; latency = submit to completion.  One run
    per load; the service rate comes from solo solves of the first requests."""
    import numpy as np

    count = len(probs)
    ctx = pb.Context(0)
    svc = []
    for p in probs[:4]:
        g = pb.Problem.from_inputs(ctx, p, precision=precision)
        g.solve()
        g.reset_operators()
        ts = time.perf_counter()
        g.solve()
        svc.append(time.perf_counter() - ts)
        g.close()
    out = {}
    for load in loads:
        rate = load / (sum(svc) / len(svc))
        rng = np.random.default_rng([4, seed])
        gaps = rng.exponential(1.0 / rate, size=count)
        srv = pb.Server(ctx, hbm_budget_bytes=64 << 30, max_slots=16)
        gs = [pb.Problem.from_inputs(ctx, p, precision=precision) for p in probs]
        submit, done, res = {}, {}, {}
        tickets = []
        start = time.perf_counter()
        next_t = start
        i = 0
        while len(done) < count:
            now = time.perf_counter()
            while i < count and now >= next_t:
                t = srv.submit(gs[i])
                tickets.append(t)
                submit[t] = time.perf_counter()
                next_t += gaps[i]
                i += 1
            for t in tickets:
                if t not in done:
                    r = srv.poll(t)
                    if r is not None:
                        done[t] = time.perf_counter()
                        res[t] = r
            time.sleep(0.0005)
        makespan = time.perf_counter() - start
        srv.close()
        for g in gs:
            g.close()
        lat = [done[t] - submit[t] for t in tickets]
        bad = sum(1 for t in tickets if res[t]["status"] != 0)
        if bad:
            raise RuntimeError(f"{bad} served requests failed")
        progress(f"serve ({'mixed' if precision == pb.MIXED else 'fp64'}, load {load}): {count} requests in "
                 f"{makespan:.2f} s, p50 {percentile(lat, 0.5):.3f} s, p99 {percentile(lat, 0.99):.3f} s")
        out[f"load_{load}"] = {"arrival_rate_per_s": rate, "load": load, "value": count / makespan,
                               "unit": "PB solves/s",
                               "latency_s": {"p50": percentile(lat, 0.5), "p99": percentile(lat, 0.99)},
                               "failures": bad}
    ctx.close()
    main = out["load_0.8"] if "load_0.8" in out else next(iter(out.values()))
    return dict(main, requests=count, precision="mixed" if precision == pb.MIXED else "fp64",
                max_triangles=20 * nmax * nmax, solo_service_s=sum(svc) / len(svc), by_load=out)


def cpu_baseline(prob, applies_per_solve, seed=0):
    """Oracle timed on a bounded sample of the same workload, extrapolated to
    one solve: sampled dense Galerkin rows (assembly), the oracle's dense row
    loop on those rows, and its matrix-free FEM products."""
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = oracle.Oracle.from_problem(prob)
    rng = np.random.default_rng(seed)
    nrows = 32 * max(1, threads)
    t_asm = t_dense = 0.0
    x = rng.standard_normal(o.n)
    for surf, nv in ((0, o.n_m), (1, o.n_s)):
        rows = np.sort(rng.choice(nv, size=nrows, replace=False))
        t0 = time.perf_counter()
        V, K = o.bem_rows(surf, rows)
        t_asm += (time.perf_counter() - t0) * nv / nrows
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            o.dense_rows_apply(surf, V, K, x)
        t_dense += (time.perf_counter() - t0) / reps * nv / nrows
    t0 = time.perf_counter()
    for _ in range(3):
        o.fem_jacobian(oracle.HS, x, x)
    t_fem = (time.perf_counter() - t0) / 3
    t_solve = t_asm + applies_per_solve * (t_dense + t_fem)
    sample = (f"{nrows} Galerkin rows per interface assembled, their dense row products x20, 3 FEM Jacobian "
              f"products; extrapolated to one solve = assembly of all rows + {applies_per_solve} coupled applies "
              f"(the GPU run's count); assembly {t_asm:.1f} s, dense apply {t_dense * 1e3:.1f} ms, "
              f"FEM product {t_fem * 1e3:.1f} ms")
    return dict(value=1.0 / t_solve, unit="PB solves/s", cores=threads, kind="oracle", sample=sample)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-picard", action="store_true", help="skip the Picard comparison leg")
    ap.add_argument("--no-matrix-free", action="store_true", help="skip the matrix-free boundary-element leg")
    ap.add_argument("--no-schemes", action="store_true", help="skip the Taylor-schedule comparison leg")
    ap.add_argument("--no-two-field", action="store_true", help="skip the two-field form leg")
    ap.add_argument("--batch", type=int, default=32, help="instances of the batched leg (0: skip)")
    ap.add_argument("--serve", type=int, default=48, help="requests of the serving leg (0: skip)")
    ap.add_argument("--serve-nmax", type=int, default=20, help="largest icosphere frequency of served requests")
    ap.add_argument("--calib-copy-gb", type=float, default=0.0,
                    help="run one device copy of this size first (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU row-block sharding is a design, not built)", file=sys.stderr)
        sys.exit(2)
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
    t0 = time.perf_counter()
    prob = pbgen.make_config(args.config)
    progress(f"generated workload {args.config} in {time.perf_counter() - t0:.1f} s: {prob.nodes.shape[0]} nodes, "
             f"{prob.tets.shape[0]} tets, {prob.tri_m.shape[0]} triangles per interface, {prob.q_z.size} charges")
    opts = dict()  # cubic start, self-adjusted omega, App. B settings (library defaults)
    if args.config == 0:
        opts = dict(omega_auto=0, omega_fixed=0.5)
    f64 = run_leg(pb, torch, prob, pb.FP64, args.steps, args.warmup, opts, "fp64")
    K = args.steps
    value = K / f64["elapsed"]
    ms_step = 1e3 * f64["elapsed"] / K
    nm, ns = f64["n_m"], f64["n_s"]
    gemv_ms, gemv_cnt = f64["timing"]["gemv"]
    apply_ms, apply_cnt = f64["timing"]["apply"]
    asm_ms, asm_cnt = f64["timing"]["assembly"]
    sym = all(a == b for a, b in f64["tiles"].values())  # square tiles: symmetric use of V'
    gb = gemv_bytes(nm, ns, 8, sym)
    achieved = gb / (gemv_ms * 1e-3) / 1e9 if gemv_ms else None
    res = f64["res"]
    applies = res["applies"]
    out = {
        "metric": "PB solves/s + coupled-operator GFLOP/s, mixed vs FP64 at <=1e-5 rel energy; p50/p99",
        "value": value,
        "unit": "PB solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"RNA-like solute (config {args.config}): {prob.tri_m.shape[0]} triangles per "
                               f"interface, {prob.tets.shape[0]} shell tets, {prob.q_z.size} charges, kappa "
                               f"{prob.kappa}, cubic-start Newton with self-adjusted relaxation, FP64",
                   "unknowns": f64["n"], "parallelism": "single GPU"},
        "latency_s": {"p50": percentile(f64["lat"], 0.5), "p99": percentile(f64["lat"], 0.99)},
        "solve": {"total_kcal_mol": res["total"], "lc": res["lc"], "nc": res["nc"], "dg_omega_i": res["dg_omega_i"],
                  "newton_iters": res["newton_iters"], "gmres_iters_total": res["gmres_iters_total"],
                  "omega": res["omega"], "status": res["status"], "coupled_applies_per_solve": applies},
        "kernel_ms": {"gemv": gemv_ms, "coupled_apply": apply_ms, "bem_assembly_launch": asm_ms},
        "roofline": {"bound": "hbm", "kernel": ("k_bgemv + k_bgemv_fin / k_gemv + k_gemv_fin (gemv_rows_sym: K' and the "
                                                "lower triangle of V', FP64, both interfaces)" if sym else
                                                "k_bgemv / k_gemv (gemv_rows: dense [K'|V'] FP64 GEMV, both interfaces)"),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": (GEMV_TRAFFIC["bytes"] if (args.config == GEMV_TRAFFIC["config"] and
                                                           gemv_source_hash() == GEMV_TRAFFIC["src_sha256_16"])
                                 else None),
                     "bytes_per_launch": gb},
    }
    # regular BEM tiles: algorithmic flops per solve over the HIP-event time
    # of the tile launches (both interfaces; touching pairs excluded)
    asm_flops = 36 * (FLOPS_QP["laplace"] * regular_pairs(prob.tri_m) +
                      FLOPS_QP["yukawa" if prob.kappa > 0 else "laplace"] * regular_pairs(prob.tri_s))

    def asm_report(leg, peak):
        ms, cnt = leg["timing"]["assembly"]
        t = ms * cnt / K * 1e-3
        return {"kernel": "k_bem_regular (6 x 6 rule, non-touching pairs)", "tile_shapes_autotuned": leg["tiles"],
                "flops_per_solve": asm_flops,
                "ms_per_solve": t * 1e3, "tflops": asm_flops / t / 1e12 if t else None, "peak_tflops": peak,
                "frac": asm_flops / t / 1e12 / peak if t else None}

    out["bem_assembly"] = {"fp64": asm_report(f64, FP64_PEAK_TFLOPS)}
    nnz = fem_nnz(prob)
    nn = prob.nodes.shape[0]

    def spmv_report(leg, elem):
        ms, cnt = leg["timing"]["spmv"]
        b = spmv_bytes(nnz, nn, leg["n"], elem)
        gbs = b / (ms * 1e-3) / 1e9 if ms else None
        return {"kernel": "k_bspmv / k_spmv (sell_part: sliced-ELL FEM rows)", "bound": "hbm",
                "bytes_per_launch": b, "ms_per_launch": ms, "launches": cnt, "achieved": gbs,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS if gbs else None,
                "nnz": nnz, "value_bytes": elem}

    out["fem_spmv"] = {"fp64": spmv_report(f64, 8)}
    out["kernel_ms"]["precond_per_solve"] = f64["timing"]["precond"][0] * f64["timing"]["precond"][1] / K
    flops = apply_flops(nm, ns, nnz)
    if apply_ms:
        out["coupled_operator_gflops"] = flops / (apply_ms * 1e-3) / 1e9
    if not args.no_mixed:
        mx = run_leg(pb, torch, prob, pb.MIXED, K, args.warmup, opts, "mixed")
        rm = mx["res"]
        mg_ms = mx["timing"]["gemv"][0]
        out["mixed"] = {
            "value": K / mx["elapsed"], "unit": "PB solves/s", "ms_per_step": 1e3 * mx["elapsed"] / K,
            "latency_s": {"p50": percentile(mx["lat"], 0.5), "p99": percentile(mx["lat"], 0.99)},
            "total_kcal_mol": rm["total"], "rel_energy_err_vs_fp64": abs(rm["total"] - res["total"]) / abs(res["total"]),
            "rel_err_vs_fp64": {k: abs(rm[k] - res[k]) / abs(res[k]) for k in ("total", "lc", "nc", "dg_omega_i")},
            "surface_potential_rel_err_vs_fp64": float(np.linalg.norm(mx["u_m"] - f64["u_m"]) /
                                                       np.linalg.norm(f64["u_m"])),
            "newton_iters": rm["newton_iters"], "gmres_iters_total": rm["gmres_iters_total"],
            "gemv_ms": mg_ms,
            "gemv_gbs": gemv_bytes(nm, ns, 4, all(a == b for a, b in mx["tiles"].values())) / (mg_ms * 1e-3) / 1e9
            if mg_ms else None,
            "coupled_operator_gflops": flops / (mx["timing"]["apply"][0] * 1e-3) / 1e9 if mx["timing"]["apply"][0] else None,
        }
        out["bem_assembly"]["mixed_fp32_eval"] = asm_report(mx, FP32_PEAK_TFLOPS)
        out["fem_spmv"]["mixed_fp32_values"] = spmv_report(mx, 4)
    if not args.no_picard:
        # the paper's comparison path: Picard (A Delta = d) with the direct-secant
        # relaxation search and the norm-ratio reuse rule, omega in [0, 1]
        popts = dict(opts, nonlinear_method=pb.PICARD, omega_method=pb.OMEGA_BSEC_DF, omega_max=1.0, l_e=0.0,
                     max_newton=200)
        pc = run_leg(pb, torch, prob, pb.FP64, 1, 0, popts, "picard")
        rp = pc["res"]
        out["picard_fp64"] = {"value": 1.0 / pc["elapsed"], "unit": "PB solves/s", "ms_per_step": 1e3 * pc["elapsed"],
                              "nonlinear_iters": rp["newton_iters"], "gmres_iters_total": rp["gmres_iters_total"],
                              "total_kcal_mol": rp["total"],
                              "rel_energy_diff_vs_newton": abs(rp["total"] - res["total"]) / abs(res["total"]),
                              "newton_iters": res["newton_iters"], "status": rp["status"]}
    if not args.no_schemes:
        # the reaction term raised through Taylor orders over the first
        # iterations (T3-HS is the default leg above)
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
        out["scheme_schedules_fp64"] = sch
        # the root finders of f_d for the relaxation factor (Newton is the default leg above)
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
        out["omega_root_finders_fp64"] = om
    if not args.no_matrix_free:
        # nothing dense stored: every coupled apply evaluates the regular
        # quadrature-point pairs again (the same flops as one assembly)
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
                        "bem_apply_ms": ams, "bem_apply_flops": asm_flops,
                        "tflops": asm_flops / (ams * 1e-3) / 1e12 if ams else None, "peak_tflops": peak,
                        "frac": asm_flops / (ams * 1e-3) / 1e12 / peak if ams else None, "status": r["status"]}
        mf["dense_fp64_device_bytes"] = f64["hbm"]
        out["matrix_free"] = mf
    if not args.no_two_field:
        # the paper's two-field form on the same surfaces: FEM also fills the
        # solute (three inner copies of Gamma_m, then coarsening layers), the
        # charges load the FEM rows, lambda_m is recovered for the energy
        ptf = pbgen.make_config(args.config, solute_layers=3)
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
        out["two_field"] = tf
    if args.batch > 0:
        out["batched"] = {"mixed": batch_leg(pb, torch, args.batch, 1, pb.MIXED),
                          "fp64": batch_leg(pb, torch, args.batch, 1, pb.FP64)}
    if args.serve > 0:
        reqs = serve_requests(args.serve, args.serve_nmax)
        out["serving"] = {"mixed": serve_leg(pb, torch, reqs, args.serve_nmax, pb.MIXED),
                          "fp64": serve_leg(pb, torch, reqs, args.serve_nmax, pb.FP64)}
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle, bounded sample)")
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(prob, max(applies, 1))
        progress(f"cpu baseline took {time.perf_counter() - t0:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
