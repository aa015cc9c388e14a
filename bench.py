#!/usr/bin/env python3
"""Throughput of the HDG trace multigrid solve on one MI355X.

Workload (default): 2D diffusion -div(kappa grad u) = f on the unit square,
512 x 512 quads, HDG degree k = 4, tau = 1, kappa per element log-uniform in
[1e-3, 1e3], nodal f ~ N(0, 1), zero Dirichlet data, seed 0 (synthetic).

A step is one complete solve: the load vector g from the nodal source, then
the outer iteration (V-cycle-preconditioned CG) until the FP64 residual
||g - A lambda|| <= 1e-10 ||g||.  `value` is the mixed-precision leg (FP32
V-cycle inside FP64 CG); the FP64 leg is reported beside it.  Operator setup
(element DtN maps, hierarchy) is outside the step and reported separately.

Prints one JSON line.
"""
import argparse
import json
import os
import subprocess
import sys
import time

METRIC = "trace DOFs/s to rel. resid 1e-10: FP64 vs FP32 V-cycle+FP64 refine"
HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
CAL_BYTES = 1 << 30
# HBM traffic of the finest-level FP32 sweeps of the 512^2, k = 4 workload
# (strip kernel + strip-edge kernel; "plain" sweeps and the "rz" sweep that
# also forms CG's r.z partials), from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of `bench.py --traffic-probe` (per-dispatch counter values,
# KiB units), each scaled by what the same counter reads for a kernel that
# reads and writes exactly CAL_BYTES.  Valid only for the kernel sources it
# was taken on.
TRAFFIC = {"plain": {"fetch": 137723.062 + 6252.500, "write": 11008.688 + 798.000},
           "rz": {"fetch": 147322.375 + 7167.000, "write": 11039.312 + 801.938},
           "cal_fetch": 524300.0, "cal_write": 1048576.0, "sources_sha256_16": "c507fc3d09621028"}
TRAFFIC_SOURCES = ["paper_1811_09909_amd/csrc/trace.hip", "paper_1811_09909_amd/csrc/trace_dev.hpp",
                   "paper_1811_09909_amd/csrc/hdg_internal.hpp", "paper_1811_09909_amd/csrc/build.hip"]


def sweep_traffic_bytes():
    """Measured bytes per launch of the two sweep kinds ({"plain": B, "rz": B}),
    or None when the kernel sources differ from the ones the counters were
    taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != TRAFFIC["sources_sha256_16"] or TRAFFIC["rz"] is None:
        return None
    kib = CAL_BYTES / 1024.0
    return {nm: (TRAFFIC[nm]["fetch"] * kib / TRAFFIC["cal_fetch"] + TRAFFIC[nm]["write"] * kib / TRAFFIC["cal_write"])
            * 1024.0 for nm in ("plain", "rz")}


# Solver configuration of the timed step; the full-size parity tests import it
SOLVER = {"method": "pcg", "sweeps": 2, "growth": 1, "coarse_n": 16, "max_it": 20000, "tol": 1e-10}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--method", default=SOLVER["method"], choices=["mg", "pcg", "gmres"])
    ap.add_argument("--sweeps", type=int, default=SOLVER["sweeps"])
    ap.add_argument("--growth", type=int, default=SOLVER["growth"])
    ap.add_argument("--coarse-n", type=int, default=SOLVER["coarse_n"],
                    help="coarsest macro grid (n x n) of the h-hierarchy, solved directly")
    ap.add_argument("--max-it", type=int, default=SOLVER["max_it"])
    ap.add_argument("--tol", type=float, default=SOLVER["tol"])
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=64)
    ap.add_argument("--cpu-min-s", type=float, default=10.0, help="repeat the oracle solve until this much time")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--batched", action="store_true",
                    help="instead of the headline solve: the batched workload (64 2D problems, n in {32..256}, "
                         "k in {2..5}, 16 right-hand sides each) through hdg_solve_batch; prints its own JSON line")
    ap.add_argument("--batched-nprob", type=int, default=64)
    ap.add_argument("--batched-nstreams", type=int, default=4)
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D (32^3, k = 3) FP64/mixed legs")
    ap.add_argument("--n3d", type=int, default=32)
    ap.add_argument("--steps3d", type=int, default=2)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched leg")
    ap.add_argument("--no-ipdg", action="store_true", help="skip the NIPG-H and multinumerics legs")
    ap.add_argument("--no-unstructured", action="store_true", help="skip the unstructured-mesh leg")
    ap.add_argument("--unx", type=int, default=256, help="unstructured leg: grid spacing 1/unx of the mesh points")
    ap.add_argument("--uk", type=int, default=3, help="unstructured leg: polynomial degree")
    ap.add_argument("--ucoarse-n", type=int, default=48,
                    help="unstructured leg: the hierarchy stops at the coarsest level with >= ucoarse_n^2 unknowns")
    ap.add_argument("--no-errors", action="store_true", help="skip the solve to the FP64 floor (error report)")
    ap.add_argument("--ref-tol", type=float, default=1e-13,
                    help="tolerance of the FP64 reference solve (stops at its floor if not reachable)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run only finest-level FP32 sweeps of the workload and a plain copy-like kernel of known "
                         "size (for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs), then exit")
    return ap.parse_args()


def cpu_baseline(n, k, coarse_n, min_s):
    """The oracle (plain FP64 NumPy/SciPy) on a bounded sample of the workload:
    same kappa/f distribution on an n x n mesh; times the solve only, repeated
    until min_s seconds have passed."""
    sys.path.insert(0, HERE)
    from oracle import mg as omg
    from oracle.hdg import HDG
    from paper_1811_09909_amd import inputs
    wl = inputs.diffusion2d(n, k, 1e-3, 1e3, seed=0)
    t0 = time.perf_counter()
    O = HDG(2, n, k, 1.0, wl.kappa)
    A, g, _ = O.assemble(wl.f)
    t1 = time.perf_counter()
    H = omg.Hierarchy(A, 2, n, k, sweeps=2, growth=1, local_corr=omg.LC_BOTH, coarsest_n=coarse_n)
    t2 = time.perf_counter()
    reps = 0
    while True:
        r = omg.pcg_solve(H, A, g, tol=1e-10, maxit=20000)
        reps += 1
        if time.perf_counter() - t2 >= min_s:
            break
    t3 = time.perf_counter()
    return {"n": n, "k": k, "trace_dofs": int(A.shape[0]), "setup_s": t1 - t0, "build_s": t2 - t1,
            "solve_s": (t3 - t2) / reps, "reps": reps, "iters": r.iters, "relres": r.relres}


def run_cpu_baseline(n, k, coarse_n, min_s):
    env = dict(os.environ)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        env[v] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--cpu-n", str(n),
                          "--k", str(k), "--coarse-n", str(coarse_n), "--cpu-min-s", str(min_s)], capture_output=True, text=True, env=env, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    res = json.loads(out.stdout.strip().splitlines()[-1])
    host_cores, cpu_model = host_info()
    return {"value": res["trace_dofs"] / res["solve_s"], "unit": "trace DOFs/s", "cores": 1, "kind": "oracle",
            "host_cores": host_cores, "cpu_model": cpu_model,
            "sample": f"diffusion2d n={n} k={k} (same kappa/f distribution, seed 0), oracle CG + V-cycle "
                      f"solve to 1e-10: {res['iters']} iterations, {res['solve_s']:.2f} s per solve over {res['reps']} solves "
                      f"(assembly {res['setup_s']:.1f} s, hierarchy {res['build_s']:.1f} s excluded); "
                      "single-threaded SciPy/NumPy",
            "iters": res["iters"], "trace_dofs": res["trace_dofs"]}


def traffic_probe(args):
    """Finest-level FP32 block-Jacobi sweeps of the benchmark workload (the
    dominant kernel, same template and launch shape as in the solve) and a
    calibration kernel that reads and writes exactly CAL_BYTES each."""
    import torch
    sys.path.insert(0, HERE)
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd import inputs
    from paper_1811_09909_amd.hdg import Problem
    wl = inputs.diffusion2d(args.n, args.k, 1e-3, 1e3, seed=0)
    P = Problem(2, args.n, args.k, torch.as_tensor(wl.kappa), tau=1.0, store_recovery=False)
    # eager launches: counters are read per dispatch
    P.build(sweeps=args.sweeps, growth=args.growth, local_corr=L.LC_BOTH, precision=L.MIXED,
            method=L.METHOD_PCG, coarse_n=args.coarse_n, variant=L.VARIANT_NO_GRAPH)
    r = torch.randn(P.nlam, dtype=torch.float32, device="cuda")
    for _ in range(3):
        P.level_smooth(0, r, 4, precision=L.FP32)  # one first step + 3 sweep launches
    # three CG iterations: the sweeps that also form r.z
    P.build(sweeps=args.sweeps, growth=args.growth, local_corr=L.LC_BOTH, precision=L.MIXED,
            method=L.METHOD_PCG, coarse_n=args.coarse_n, max_it=3, variant=L.VARIANT_NO_GRAPH)
    P.solve(torch.as_tensor(wl.f), tol=1e-30, allow_not_converged=True)
    x = torch.ones(CAL_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "done", "nlam": P.nlam, "cal_bytes": CAL_BYTES}))
    return 0


def batched(args):
    """Many meshes, many right-hand sides: problems of uneven size and degree,
    each with 16 right-hand sides, solved together by hdg_solve_batch (mixed
    precision PCG + symmetric V-cycle to 1e-10 per right-hand side).  The
    autotuner picks the coarsest grid and right-hand-side group size once per
    (n, k) class."""
    import torch
    sys.path.insert(0, HERE)
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd import inputs
    from paper_1811_09909_amd.hdg import Problem, solve_batch
    probs = inputs.batched2d(nprob=args.batched_nprob, nrhs=16, seed=0)
    base = dict(sweeps=2, growth=1, local_corr=L.LC_BOTH, precision=L.MIXED, method=L.METHOD_PCG, max_it=5000)
    t0 = time.perf_counter()
    Ps, rhs, tuned = [], [], {}
    for w in probs:
        P = Problem(2, w.n, w.k, torch.as_tensor(w.kappa), tau=1.0, store_recovery=False)
        key = (w.n, w.k)
        if key not in tuned:
            tuned[key] = P.autotune(16, **base)
        else:
            P.build(**dict(base, coarse_n=tuned[key]["coarse_n"], nrhs=tuned[key]["nrhs"],
                           variant=tuned[key]["variant"]))
        Ps.append(P)
        rhs.append(w.f)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    dofs = sum(P.nlam * 16 for P in Ps)
    progress(f"batched: {len(Ps)} problems set up and tuned in {t_setup:.1f} s")
    # warm-up: captures every handle's iteration graphs
    solve_batch(Ps, rhs, tol=1e-2, nstreams=0)
    solve_batch(Ps, rhs, tol=1e-2, nstreams=args.batched_nstreams)
    res = {}
    for ns in (0, -4, -8, -16, args.batched_nstreams):  # 0: one batch graph; -q: q graphs on q streams
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, infos = solve_batch(Ps, rhs, tol=1e-10, nstreams=ns)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[ns] = (el, infos)
        progress(f"batched: nstreams={ns} {1e3 * el:.1f} ms")
    el, infos = res[-8]
    out = {
        "metric": "trace DOFs/s to rel. resid 1e-10 (batched: sum over problems and right-hand sides)",
        "value": round(dofs / el, 1), "unit": "trace DOFs/s", "n_gpus": 1, "ms_per_batch": round(1e3 * el, 2),
        "higher_is_better": True, "dtype": "f32 V-cycle + f64 CG", "data": "synthetic",
        "config": {"workload": f"batched2d {len(Ps)} problems x 16 rhs, n in {{32,64,128,256}}, k in {{2..5}}, "
                               "kappa=logU[1e-2,1e2] seed=0 tau=1",
                   "trace_dofs_total": dofs,
                   "launch": "8 batch graphs (problems dealt to 8 streams), each advancing its problems by a group "
                             "of CG iterations per launch",
                   "one_graph_ms": round(1e3 * res[0][0], 2),
                   "graphs_on_streams_ms": {str(-q): round(1e3 * res[q][0], 2) for q in (-4, -8, -16)},
                   "streams_ms": {"nstreams": args.batched_nstreams,
                                  "ms": round(1e3 * res[args.batched_nstreams][0], 2)},
                   "max_iters": max(i["iters"] for i in infos),
                   "max_relres": max(i["relres"] for i in infos),
                   "setup_and_autotune_s": round(t_setup, 2),
                   "classes": {f"n{n}_k{k}": v for (n, k), v in sorted(tuned.items())}},
    }
    return out


def progress(msg):
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def host_info():
    """Cores this process may run on and the host CPU model."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None:
        try:
            with open("/proc/cpuinfo") as fh:
                for line in fh:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return cores, model


def timed_solves(P, f, tol, steps, warmup, **kw):
    """Warm-up solves (graph capture), then `steps` solves each bracketed by
    device synchronisations: per-step wall times (s), last solution, infos."""
    import torch
    for _ in range(warmup):
        P.solve(f, tol=tol, **kw)
    torch.cuda.synchronize()
    times, infos, lam = [], [], None
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, info = P.solve(f, tol=tol, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        infos.append(info)
    return times, lam, infos


def median(xs):
    xs = sorted(xs)
    m = len(xs)
    return xs[m // 2] if m % 2 else 0.5 * (xs[m // 2 - 1] + xs[m // 2])


def rel(a, b):
    return float((a - b).norm() / b.norm())


def cube3d_legs(args):
    """The 3D workload (32^3 hexahedra, k = 3, kappa(x) at the Gauss points,
    manufactured u): FP64 and mixed PCG + V-cycle to 1e-10, same launch path
    as the headline (graphs, no profiling); median step times."""
    import torch
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd import inputs
    from paper_1811_09909_amd.hdg import Problem
    n, k = args.n3d, 3
    wl = inputs.diffusion3d(n, k)
    probe = Problem(3, n, k, torch.ones(n ** 3, dtype=torch.float64), tau=1.0, store_recovery=False)
    X = probe.volume_qpoints().numpy()
    Xn = probe.volume_nodes().numpy()
    probe.close()
    kq = torch.as_tensor(wl.kappa_fn(X), device="cuda")
    f = torch.as_tensor(wl.f(Xn), device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = Problem(3, n, k, kq, tau=1.0, kappa_kind="qp", store_recovery=False)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    out = {"workload": wl.name + " tau=1", "trace_dofs": P.nlam, "setup_ms": round(1e3 * t_setup, 2)}
    lams = {}
    for nm, prec in (("fp64", L.FP64), ("mixed", L.MIXED)):
        P.build(sweeps=args.sweeps, growth=1, local_corr=L.LC_BOTH, precision=prec, method=L.METHOD_PCG,
                max_it=args.max_it, coarse_n=2)
        progress(f"3d {nm} leg: n={n} k={k}, {P.nlam} trace DOFs")
        times, lam, infos = timed_solves(P, f, args.tol, args.steps3d, 1)
        ms = 1e3 * median(times)
        progress(f"3d {nm}: {1e3 * median(times):.1f} ms/solve, {infos[-1]['iters']} iterations")
        lams[nm] = lam
        out[nm] = {"value": round(P.nlam / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
                   "iters": infos[-1]["iters"], "refinement_steps": infos[-1]["outer_iters"],
                   "relres": max(i["relres"] for i in infos), "build_ms": round(infos[-1]["t_build_ms"], 2)}
    out["lambda_mixed_vs_fp64"] = rel(lams["mixed"], lams["fp64"])
    out["mixed_over_fp64"] = round(out["mixed"]["value"] / out["fp64"]["value"], 3)
    # finest-level kernels of the mixed solve, event-timed in one more solve
    P.profile_begin()
    P.solve(f, tol=args.tol)
    kern = {}
    for mode, name in [(0, "apply"), (2, "sweep"), (3, "residual_prestrict"), (6, "sweep_rz")]:
        for pr, pn in [(L.FP64, "fp64"), (L.MIXED_CYCLE, "fp32ops_fp64vec")]:
            r = P.profile_read(mode, pr)
            if r["launches"]:
                t = r["total_ms"] / r["launches"]
                gbs = r["bytes_per_launch"] / (t * 1e-3) / 1e9
                kern[f"{name}_{pn}"] = {"launches": r["launches"], "avg_ms": round(t, 5), "GBps": round(gbs, 1),
                                        "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["kernels"] = kern
    P.close()
    return out


def ipdg_legs(args):
    """The hybridized IPDG workload (NIPG-H, eq. IPG_H) on the headline mesh:
    element maps timed on their own (a re-form through hdg_update_kappa),
    then GMRES + V-cycle to 1e-10 in FP64 and with the FP32 cycle, same
    launch path as the headline; median step times."""
    import torch
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd import inputs
    from paper_1811_09909_amd.hdg import Problem
    n, k = args.n, args.k
    wl = inputs.ipdg2d(n, k)
    kap = torch.as_tensor(wl.kappa, device="cuda")
    P = Problem(2, n, k, kap, tau=wl.tau, scheme="nipg", tau_kappa=True, store_recovery=False)
    f = torch.as_tensor(wl.f(P.volume_nodes().numpy()), device="cuda")
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.update_kappa(kap)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t_el = median(ts)
    nv, nl = (k + 1) ** 2, 4 * (k + 1)
    flops = n * n * (2 * (2 * nv * nv * nl + nl * nl * nv) + 2 * nv ** 3)
    out = {"workload": wl.name, "trace_dofs": P.nlam,
           "element_maps_ms": round(1e3 * t_el, 3),
           "element_maps_tflops": round(flops / t_el / 1e12, 2),
           "element_maps_note": "hdg_update_kappa wall time: kappa check + ipdg_dtn_kernel; flops of the "
                                "inverse and the three products per element"}
    lams = {}
    for nm, prec in (("fp64", L.FP64), ("mixed", L.MIXED)):
        P.build(sweeps=args.sweeps, growth=args.growth, local_corr=L.LC_PRE, precision=prec,
                method=L.METHOD_GMRES, max_it=200, coarse_n=args.coarse_n)
        progress(f"ipdg {nm} leg: n={n} k={k}, {P.nlam} trace DOFs")
        times, lam, infos = timed_solves(P, f, args.tol, args.steps, 1)
        ms = 1e3 * median(times)
        progress(f"ipdg {nm}: {ms:.1f} ms/solve, {infos[-1]['iters']} iterations")
        lams[nm] = lam
        out[nm] = {"value": round(P.nlam / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
                   "iters": infos[-1]["iters"], "relres": max(i["relres"] for i in infos)}
    out["lambda_mixed_vs_fp64"] = rel(lams["mixed"], lams["fp64"])
    out["mixed_over_fp64"] = round(out["mixed"]["value"] / out["fp64"]["value"], 3)
    P.close()
    return out


def multinumerics_legs(args):
    """Multinumerics (RT-H outside a disk, NIPG-H inside, Example VI's
    coefficient) on the headline mesh at k = 1: element maps timed alone,
    then GMRES + V-cycle to 1e-10 in FP64 and with the FP32 cycle."""
    import torch
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd import inputs
    from paper_1811_09909_amd.hdg import Problem
    n, k = args.n, 1
    wl = inputs.multinumerics2d(n, k)
    kap = torch.as_tensor(wl.kappa, device="cuda")
    P = Problem(2, n, k, kap, tau=wl.tau, tau_kappa=True, scheme_of_element=wl.schemes, store_recovery=False)
    f = torch.as_tensor(wl.f, device="cuda")
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.update_kappa(kap)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    out = {"workload": wl.name, "trace_dofs": P.nlam, "rt_elements": sum(s == "rt" for s in wl.schemes),
           "element_maps_ms": round(1e3 * median(ts), 3)}
    lams = {}
    for nm, prec in (("fp64", L.FP64), ("mixed", L.MIXED)):
        P.build(sweeps=args.sweeps, growth=args.growth, local_corr=L.LC_PRE, precision=prec,
                method=L.METHOD_GMRES, max_it=200, coarse_n=args.coarse_n)
        progress(f"multinumerics {nm} leg: n={n} k={k}, {P.nlam} trace DOFs")
        times, lam, infos = timed_solves(P, f, args.tol, args.steps, 1)
        ms = 1e3 * median(times)
        progress(f"multinumerics {nm}: {ms:.1f} ms/solve, {infos[-1]['iters']} iterations")
        lams[nm] = lam
        out[nm] = {"value": round(P.nlam / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
                   "iters": infos[-1]["iters"], "relres": max(i["relres"] for i in infos)}
    out["lambda_mixed_vs_fp64"] = rel(lams["mixed"], lams["fp64"])
    out["mixed_over_fp64"] = round(out["mixed"]["value"] / out["fp64"]["value"], 3)
    P.close()
    return out


def unstructured_legs(args):
    """HDG on the unstructured box with eight holes (Example II's setting:
    kappa = 1, f = 1, tau = 1) with the seed-point agglomeration hierarchy:
    setup (host agglomeration + element maps), then CG + V-cycle to 1e-10 in
    FP64 and with the mixed cycle, and MG as a solver in FP64; median step
    times on the headline's launch path; the finest-level apply and sweeps
    event-timed in one more mixed solve."""
    import torch
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd import inputs
    from paper_1811_09909_amd.hdg import Problem
    k = args.uk
    wl = inputs.unstructured2d(args.unx, k)
    kap = torch.as_tensor(wl.kappa, device="cuda")
    f = torch.as_tensor(wl.f, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = Problem.unstructured(wl.vertices, wl.triangles, k, kap, wl.seeds, wl.hlevels, tau=wl.tau)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    out = {"workload": wl.name, "triangles": int(len(wl.triangles)), "trace_dofs": P.nlam,
           "setup_ms": round(1e3 * t_setup, 2)}
    lams = {}
    for nm, meth, prec in (("pcg_fp64", L.METHOD_PCG, L.FP64), ("pcg_mixed", L.METHOD_PCG, L.MIXED),
                           ("mg_fp64", L.METHOD_MG, L.FP64)):
        P.build(sweeps=args.sweeps, growth=1, local_corr=L.LC_BOTH if meth == L.METHOD_PCG else L.LC_PRE,
                precision=prec, method=meth, max_it=500, coarse_n=args.ucoarse_n)
        out["levels"] = P.level_sizes()
        progress(f"unstructured {nm} leg: {len(wl.triangles)} triangles k={k}, {P.nlam} trace DOFs")
        times, lam, infos = timed_solves(P, f, args.tol, args.steps, 1)
        ms = 1e3 * median(times)
        progress(f"unstructured {nm}: {ms:.1f} ms/solve, {infos[-1]['iters']} iterations")
        lams[nm] = lam
        out[nm] = {"value": round(P.nlam / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
                   "iters": infos[-1]["iters"], "relres": max(i["relres"] for i in infos),
                   "build_ms": round(infos[-1]["t_build_ms"], 2)}
    out["lambda_mixed_vs_fp64"] = rel(lams["pcg_mixed"], lams["pcg_fp64"])
    out["mixed_over_fp64"] = round(out["pcg_mixed"]["value"] / out["pcg_fp64"]["value"], 3)
    P.build(sweeps=args.sweeps, growth=1, local_corr=L.LC_BOTH, precision=L.MIXED, method=L.METHOD_PCG, max_it=500,
            coarse_n=args.ucoarse_n)
    P.profile_begin()
    P.solve(f, tol=args.tol)
    kern = {}
    for mode, name in [(0, "apply"), (2, "sweep"), (3, "residual_prestrict"), (6, "sweep_rz")]:
        for pr, pn in [(L.FP64, "fp64"), (L.MIXED_CYCLE, "fp32ops_fp64vec")]:
            r = P.profile_read(mode, pr)
            if r["launches"]:
                t = r["total_ms"] / r["launches"]
                gbs = r["bytes_per_launch"] / (t * 1e-3) / 1e9
                kern[f"{name}_{pn}"] = {"launches": r["launches"], "avg_ms": round(t, 5), "GBps": round(gbs, 1),
                                        "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["kernels"] = kern
    P.close()
    # NIPG-H on the same mesh (Example II's Table NIPG setting, tau = (p+1)(p+2)/h_min): GMRES + V-cycle
    import numpy as np
    V, T = wl.vertices, wl.triangles
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    hmin = float(np.hypot(*(V[e[:, 0]] - V[e[:, 1]]).T).min())
    Pn = Problem.unstructured(V, T, k, kap, wl.seeds, wl.hlevels, tau=(k + 1) * (k + 2) / hmin, scheme="nipg")
    nip = {"tau": round((k + 1) * (k + 2) / hmin, 3)}
    for nm, prec in (("fp64", L.FP64), ("mixed", L.MIXED)):
        Pn.build(sweeps=args.sweeps, growth=1, local_corr=L.LC_PRE, precision=prec, method=L.METHOD_GMRES,
                 max_it=200, coarse_n=args.ucoarse_n)
        progress(f"unstructured nipg {nm} leg")
        times, _, infos = timed_solves(Pn, f, args.tol, args.steps, 1)
        ms = 1e3 * median(times)
        progress(f"unstructured nipg {nm}: {ms:.1f} ms/solve, {infos[-1]['iters']} iterations")
        nip[nm] = {"value": round(Pn.nlam / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
                   "iters": infos[-1]["iters"], "relres": max(i["relres"] for i in infos)}
    out["nipg_gmres"] = nip
    Pn.close()
    return out


def main():
    args = parse()
    if args.traffic_probe:
        return traffic_probe(args)
    if args.batched:
        print(json.dumps(batched(args)))
        return 0
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.cpu_n, args.k, args.coarse_n, args.cpu_min_s)))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding is a "
              "design note, not a build target", file=sys.stderr)
        return 2
    import torch
    sys.path.insert(0, HERE)
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd import inputs
    from paper_1811_09909_amd.hdg import Problem

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, k = args.n, args.k
    wl = inputs.diffusion2d(n, k, 1e-3, 1e3, seed=0)
    kap = torch.as_tensor(wl.kappa, device=dev)
    f = torch.as_tensor(wl.f, device=dev)
    method = {"mg": L.METHOD_MG, "pcg": L.METHOD_PCG, "gmres": L.METHOD_GMRES}[args.method]
    lc = L.LC_BOTH if args.method == "pcg" else L.LC_PRE

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = Problem(2, n, k, kap, tau=1.0, store_recovery=True)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    N = P.nlam

    def build(precision, max_it=None):
        P.build(sweeps=args.sweeps, growth=args.growth, local_corr=lc, precision=precision, method=method,
                max_it=args.max_it if max_it is None else max_it, coarse_n=args.coarse_n)

    def leg(precision):
        """The production path: graph-captured iteration bodies, no event
        bracketing; the median of per-step times."""
        t0 = time.perf_counter()
        build(precision)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        progress(f"2d leg precision={precision}: {args.warmup} warm-up + {args.steps} timed solves")
        times, lam, infos = timed_solves(P, f, args.tol, args.steps, args.warmup)
        ms = 1e3 * median(times)
        progress(f"2d leg precision={precision}: {ms:.1f} ms/solve, {infos[-1]['iters']} iterations")
        return {"ms_per_step": ms, "mean_ms": 1e3 * sum(times) / len(times), "value": N / (ms / 1e3),
                "iters": infos[-1]["iters"], "refinement_steps": infos[-1]["outer_iters"],
                "relres": max(i["relres"] for i in infos), "build_s": t_build,
                "n_levels": infos[-1]["n_levels"], "lam": lam, "elapsed_s": sum(times)}

    res64 = None if args.skip_fp64 else leg(L.FP64)
    resmx = leg(L.MIXED)
    # recovery of (u, q) from the mixed solution, timed once (outside the step)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, q = P.reconstruct(resmx["lam"], f)
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0

    # kernel timing: one more mixed solve, untimed, with HIP events around
    # every finest-level launch (eager launches: this pass is not the step)
    progress("profiled mixed solve (event-timed kernels)")
    P.profile_begin()
    P.solve(f, tol=args.tol)
    prof = {}
    for mode, name in [(0, "apply"), (1, "residual"), (2, "sweep"), (3, "residual_prestrict"), (6, "sweep_rz")]:
        for pr, pn in [(0, "fp64"), (1, "fp32")]:
            r = P.profile_read(mode, pr)
            if r["launches"]:
                prof[f"{name}_{pn}"] = r
    # transfer kernels: first h-transition level, and the p-prolongation
    for t in L.XFER_KINDS:
        for pr, pn in [(0, "fp64"), (1, "fp32")]:
            r = P.profile_read(0, pr, transfer=t)
            if r["launches"]:
                prof[f"{t}_{pn}"] = r

    # errors of the headline solutions against the FP64 reference: the FP64
    # solve driven to its floor (the relative residual it can reach)
    errors = None
    if not args.skip_fp64 and not args.no_errors:
        progress("FP64 reference solve for the error report")
        build(L.FP64, max_it=res64["iters"] + 400)  # a few hundred iterations past the metric's tolerance
        lam_ref, info_ref = P.solve(f, tol=args.ref_tol, allow_not_converged=True)
        u_ref, q_ref = P.reconstruct(lam_ref, f)
        u64, q64 = P.reconstruct(res64["lam"], f)
        errors = {"reference": f"FP64 PCG driven to relres {info_ref['relres']:.2e} ({info_ref['iters']} iterations)",
                  "mixed": {"lambda": rel(resmx["lam"], lam_ref), "u": rel(u, u_ref), "q": rel(q, q_ref)},
                  "fp64": {"lambda": rel(res64["lam"], lam_ref), "u": rel(u64, u_ref), "q": rel(q64, q_ref)}}

    # dominant kernel of the mixed leg: the finest-level FP32 block-Jacobi
    # sweep, every launch of it (the plain sweeps and the one per iteration
    # that also forms the r.z partials of CG): summed algorithmic bytes over
    # summed event time
    sw = [prof[nm] for nm in ("sweep_fp32", "sweep_rz_fp32") if nm in prof]
    if sw:
        launches = sum(v["launches"] for v in sw)
        tot_ms = sum(v["total_ms"] for v in sw)
        tot_bytes = sum(v["launches"] * v["bytes_per_launch"] for v in sw)
        dom_label = "sweep_fp32 (finest level, strip kernel + strip-edge kernel; with the r.z sweeps)"
    else:
        dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
        launches, tot_ms = dom["launches"], dom["total_ms"]
        tot_bytes = launches * dom["bytes_per_launch"]
        dom_label = dom_name
    avg_ms = tot_ms / launches
    bytes_per_launch = tot_bytes / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = None
    if sw and n == 512 and k == 4:
        tp = sweep_traffic_bytes()
        if tp is not None:
            traffic = sum(v["launches"] * tp[nm] for nm, v in (("plain", prof.get("sweep_fp32")),
                                                              ("rz", prof.get("sweep_rz_fp32"))) if v) / launches
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 4),
                "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                "kernel": f"trace {dom_label}",
                "avg_launch_ms": round(avg_ms, 5), "launches": launches,
                "algorithmic_bytes_per_launch": round(bytes_per_launch, 1),
                "timing": "HIP events around each launch in a separate eager solve (not the timed step)"}
    kernels = {name: {"launches": v["launches"], "avg_ms": round(v["total_ms"] / v["launches"], 5),
                      "GBps": round(v["bytes_per_launch"] / (v["total_ms"] / v["launches"] * 1e-3) / 1e9, 1),
                      "frac": round(v["bytes_per_launch"] / (v["total_ms"] / v["launches"] * 1e-3) / 1e12 / 8.0, 4)}
               for name, v in prof.items()}
    P.close()

    cube = None
    if not args.no_3d:
        try:
            cube = cube3d_legs(args)
        except Exception as e:  # reported; the headline stands on its own
            cube = {"error": str(e)[:300]}
    ipdg = None
    if not args.no_ipdg:
        try:
            ipdg = ipdg_legs(args)
        except Exception as e:  # reported; the headline stands on its own
            ipdg = {"error": str(e)[:300]}
    multi = None
    if not args.no_ipdg:
        try:
            multi = multinumerics_legs(args)
        except Exception as e:  # reported; the headline stands on its own
            multi = {"error": str(e)[:300]}
    unst = None
    if not args.no_unstructured:
        try:
            unst = unstructured_legs(args)
        except Exception as e:  # reported; the headline stands on its own
            unst = {"error": str(e)[:300]}
    batch = None
    if not args.no_batched:
        progress("batched leg")
        try:
            batch = batched(args)
        except Exception as e:
            batch = {"error": str(e)[:300]}

    cpu = None
    if not args.no_cpu_baseline:
        progress("oracle baseline on the host")
        try:
            cpu = run_cpu_baseline(args.cpu_n, k, args.coarse_n, args.cpu_min_s)
        except Exception as e:  # reported, never fatal for the GPU figure
            cpu = {"error": str(e)[:300]}

    out = {
        "metric": METRIC, "value": round(resmx["value"], 1), "unit": "trace DOFs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(resmx["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 V-cycle + f64 CG",
        "data": "synthetic",
        "config": {"workload": wl.name + " tau=1", "trace_dofs": N, "levels": resmx["n_levels"],
                   "method": f"{args.method} + V-cycle (sweeps {args.sweeps}, growth {args.growth}, "
                             f"coarsest {args.coarse_n}x{args.coarse_n} macro grid)",
                   "step_time": "median of per-step wall times (graph-captured production path)",
                   "tol": args.tol, "iters_mixed": resmx["iters"], "refinement_steps_mixed": resmx["refinement_steps"],
                   "relres_mixed": resmx["relres"], "mean_ms_mixed": round(resmx["mean_ms"], 3),
                   "fp64": None if res64 is None else {"value": round(res64["value"], 1),
                                                       "ms_per_step": round(res64["ms_per_step"], 3),
                                                       "iters": res64["iters"], "relres": res64["relres"]},
                   "mixed_over_fp64": None if res64 is None else round(resmx["value"] / res64["value"], 3),
                   "setup_ms": round(1e3 * t_setup, 2), "build_ms_mixed": round(1e3 * resmx["build_s"], 2),
                   "reconstruct_ms": round(1e3 * t_rec, 3),
                   "end_to_end_dofs_per_s": round(N / (t_setup + resmx["build_s"] + resmx["ms_per_step"] / 1e3), 1),
                   "errors": errors, "diffusion3d": cube, "ipdg2d": ipdg, "multinumerics2d": multi,
                   "unstructured2d": unst, "batched": batch},
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
