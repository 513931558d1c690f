"""Benchmark: Stokes unknowns solved per second to a 1e-8 relative residual.

One step = one full FGMRES solve (block preconditioner of eq. (precond) with
two V-cycles per iteration, robust star smoother and transfers, coarse solve)
from x = 0 with the hierarchy already resident in HBM, to an FP64 true
relative residual of 1e-8. The default workload is the largest single-GPU
configuration: 3D 48^3 hexahedra, 3 levels, viscoplastic Newton tensor over
a 24-sinker base field (contrast 1e10), gamma 1e4 (3,014,493 unknowns).
`value` is the plain FP64 form. The mixed form (FP32 V-cycles inside FP64
FGMRES) is attempted too and reported under `forms` (converged or not, with
the reason); so are the block upper-triangular variant and the F-cycle.
Setup is timed separately. Also reported: the 2D 128^2 and 3D 32^3
workloads (FP64, fewer steps), the viscoplastic Newton loop on 3D 32^3 and,
unless --no-serving, the serving stream (continuous batching, p50/p99
latency, after a warm-up stream; also run once with the cross-request
batched patch solves turned on, and bursts of same-shape requests with them
off and on). Prints one
JSON line.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME] [--form both|fp64|mixed]
                [--no-cpu-baseline] [--serving N | --no-serving] [--no-extra] [--trace]

--trace leaves out the per-kernel event timing pass and the extra legs, so a
profiler trace of the command holds the timed solves only.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Stokes DoF solved/s to rel.res 1e-8 (FP64 vs mixed); p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
DEFAULT_CONFIG = "viscoplastic_3d_48cu_L3"
# bounded sample of the oracle for the CPU baseline: the same law at the
# largest 3D size whose oracle setup and solve fit in about half a minute
CPU_SAMPLE = dict(dim=3, n_fine=8, levels=2)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wl):
    """The oracle's own FGMRES solve of a bounded sample of the workload (same
    law, parameters and seeds on a smaller mesh) on the host CPU, with the
    BLAS thread pool at all host cores."""
    import dataclasses
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.krylov import StokesSolver
    sample = dataclasses.replace(wl, name=f"{wl.name}_sample_{CPU_SAMPLE['n_fine']}", **CPU_SAMPLE)
    cores = os.cpu_count() or 1
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        s = StokesSolver(sample)
        t_setup = time.perf_counter() - t0
        x, info = s.solve()
        blas = [dict(api=p.get("internal_api"), threads=p.get("num_threads")) for p in threadpool_info()]
    dof = sum(sample.unknowns())
    return {"value": dof / info["t_solve"], "unit": "DoF/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle FGMRES solve of the same workload recipe on a {sample.dim}D {sample.n_fine}^{sample.dim} "
                      f"mesh, {sample.levels} levels ({dof} unknowns, {info['iters']} iterations, "
                      f"{info['t_solve']:.1f} s solve, {t_setup:.1f} s setup excluded); BLAS pool at {cores} threads "
                      f"(the oracle's patch loops are single-threaded Python)",
            "iters": info["iters"], "converged": bool(info["converged"]), "t_solve_s": info["t_solve"],
            "t_setup_s": t_setup, "cpu_model": cpu_model(), "blas": blas}


def measured_traffic(wl, form):
    """HBM bytes per k_asm_gemv launch from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE + WRITE_SIZE, scaled by the copy
    kernel factor), or None when there is none or the kernels have changed
    since the counters were taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{wl.name}.json")
    if not os.path.exists(p):
        return None, "no counter summary for this workload"
    with open(p) as f:
        t = json.load(f)
    from paper_2107_00820_amd.profiling import kernel_source_hash
    if t.get("source_hash") != kernel_source_hash():
        return None, "kernels changed since the counters were taken"
    r = "float" if form.startswith("mixed") else "double"
    tot = n = 0.0
    for k, v in t["kernels"].items():
        if re.search(rf"k_asm_gemv<{wl.dim}, {r}(, \d+)?>", k) and v.get("traffic_bytes_per_launch"):
            c = min(v["launches_fetch_run"], v["launches_write_run"])
            tot += v["traffic_bytes_per_launch"] * c
            n += c
    if n == 0:
        return None, "kernel not in the counter summary"
    return tot / n, os.path.relpath(p, ROOT)


def solve_bytes_model(h, wl, iters, prof, m):
    """Algorithmic HBM bytes of one solve (FP64), the numerator of the
    solve-level roofline fraction: the patch-solve and cell-kernel bytes the
    library counted during the event-timed solve, plus the coarse solves
    (two per V-cycle's coarsest visit: one product with the packed inverse)
    and the outer FGMRES orthogonalisation (classical Gram-Schmidt twice:
    2 (j+1) basis reads and the update per step). Transfers, node gathers and
    the relaxation's own Krylov vectors are left out, so this is a lower bound."""
    n_u, n_p = h.sizes(h.L - 1)
    nvec = n_u + n_p
    nv0, _ = h.sizes(0)
    d = wl.dim
    nc0 = wl.n_level(0)
    n0 = d * (2 * nc0 - 1) ** d
    nb = (n0 + 63) // 64
    coarse = 8.0 * 4096 * nb * (nb + 1) / 2
    vcycles = 2 * iters
    orth = 0.0
    for it in range(iters):
        j = it % m
        orth += 8.0 * nvec * (2 * (j + 1) + 2 * (j + 1) + 3)
    asm_b, elem_b = prof[0][2], prof[1][2]
    return asm_b + elem_b + vcycles * coarse + orth


def time_form(h, wl, bu, bp, xu, xp, form, steps, warmup, profile_pass):
    import torch
    mixed = form.startswith("mixed")
    pc = "upper" if "_upper" in form else "full"
    cycle = "F" if form.endswith("_F") else getattr(wl, "cycle", "V")
    kw = dict(rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit, xu=xu, xp=xp, mixed=mixed, pc=pc, cycle=cycle)
    ok = True
    info = None
    for i in range(max(warmup, 1)):
        _, _, info = h.stk_solve(bu, bp, allow_notconv=True, **kw)
        log(f"[bench] {form} warmup {i}: {info['iters']} iterations, rel res {info['rel_res']:.2e}")
        ok = ok and info["converged"]
        if not ok:
            break
    if not ok:
        return dict(value=None, converged=False, iterations=info["iters"], rel_res=info["rel_res"])
    lat, iters, rr = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        _, _, info = h.stk_solve(bu, bp, **kw)
        lat.append(time.perf_counter() - ts)
        iters.append(info["iters"])
        rr.append(info["rel_res"])
        assert info["converged"] and info["rel_res"] <= wl.rtol, info
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    n_u, n_p = wl.unknowns()
    log(f"[bench] {form}: {steps} solves in {t_total:.3f} s, iterations {iters}")
    out = dict(value=(n_u + n_p) * steps / t_total, converged=True, ms_per_step=1e3 * t_total / steps,
               iterations=iters[-1], rel_res=max(rr), p50_ms=1e3 * percentile(lat, 0.5),
               p99_ms=1e3 * percentile(lat, 0.99), t_total=t_total)
    if profile_pass:
        # kernel durations: one more solve with plain launches, each launch of
        # the instrumented kernel families bracketed by HIP events on the
        # stream it runs on
        h.stk_profile(True, reps=1)
        h.stk_solve(bu, bp, eager=True, **kw)
        out["prof"] = {k: h.stk_profile_read(k) for k in (0, 1, 2)}
        h.stk_profile(False)
    return out


def roofline_of(h, wl, r, t_solve):
    """The patch-solve roofline of a timed form (r from time_form with its
    profiling pass): event-timed algorithmic bytes of every k_asm_gemv launch
    (all smoothed levels, then the finest), the cell kernel's rate, the
    solve-level byte model and the counter traffic recorded for the workload."""
    n_gemv, ms_gemv, by_gemv = r["prof"][0]
    n_elem, ms_elem, by_elem = r["prof"][1]
    n_fine, ms_fine, by_fine = r["prof"][2]
    ach = by_gemv / (ms_gemv * 1e-3) / 1e9 if ms_gemv > 0 else 0.0
    ach_fine = by_fine / (ms_fine * 1e-3) / 1e9 if ms_fine > 0 else 0.0
    traffic, traffic_src = measured_traffic(wl, "fp64")
    sb = solve_bytes_model(h, wl, r["iterations"], r["prof"], wl.restart)
    return {
        "bound": "hbm", "kernel": "k_asm_gemv (batched star-patch solves, all smoothed levels)",
        "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
        "traffic": traffic, "traffic_source": traffic_src, "form": "fp64",
        "launches_per_solve": n_gemv, "avg_launch_us": 1e3 * ms_gemv / max(n_gemv, 1),
        "algorithmic_bytes_per_launch": by_gemv / max(n_gemv, 1),
        "time_share_of_solve": (ms_gemv * 1e-3) / t_solve,
        "fine_level": {"achieved": ach_fine, "frac": ach_fine / HBM_PEAK_GBS, "launches_per_solve": n_fine,
                       "avg_launch_us": 1e3 * ms_fine / max(n_fine, 1),
                       "algorithmic_bytes_per_launch": by_fine / max(n_fine, 1)},
        "cell_kernel": {"avg_launch_us": 1e3 * ms_elem / max(n_elem, 1),
                        "GBs": (by_elem / (ms_elem * 1e-3) / 1e9) if ms_elem > 0 else 0.0,
                        "time_share_of_solve": (ms_elem * 1e-3) / t_solve},
        "solve_level": {"algorithmic_bytes": sb, "achieved": sb / t_solve / 1e9,
                        "frac": sb / t_solve / 1e9 / HBM_PEAK_GBS,
                        "model": "patch solves + cell kernels (counted by the library) + coarse solves "
                                 "+ outer Gram-Schmidt; transfers, gathers and relaxation vectors left out"},
        "timing": "HIP events on the library's launch stream around every launch of the kernel "
                  "in one extra plain-launch solve"}


def other_workload(name, steps):
    """FP64 (and, for the 2D workload, mixed) solves of another configuration."""
    import torch
    from workloads import CONFIGS
    from paper_2107_00820_amd import Hierarchy
    from paper_2107_00820_amd.tune import load_asm_tuning
    wl = CONFIGS[name]
    forms = ["fp64", "mixed"] if wl.dim == 2 else ["fp64"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = Hierarchy.from_workload(wl, mixed=1 if "mixed" in forms else 0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    h.apply_asm_tuning(load_asm_tuning())
    bu, bp = h.stk_rhs()
    xu, xp = h.zeros_u(), h.zeros_p()
    res = {"setup_s": t_setup, "unknowns": sum(wl.unknowns())}
    for f in forms:
        r = time_form(h, wl, bu, bp, xu, xp, f, steps, 1, f == "fp64")
        if "prof" in r:
            res["roofline"] = roofline_of(h, wl, r, r["t_total"] / steps)
            r.pop("prof")
        r.pop("t_total", None)
        res[f] = r
    h.close()
    return res


def serving_leg(n, budget_gb, pc="full", warm=True):
    """The seeded request stream through the serving loop. The process is
    warmed first with 40 requests of another seed (a cold first stream pays
    one-time costs: device memory mapping for the hierarchies, code-object
    loads, host threads and events; its p50 is 2-4x the warm one)."""
    from workloads import serving_stream
    from paper_2107_00820_amd.serve import Server
    if warm:
        Server(hbm_budget=int(budget_gb * 2 ** 30), max_active=16, pc=pc).run(serving_stream(40, 20.0, 502))
    reqs = serving_stream(n)
    log(f"[bench] serving {n} requests, budget {budget_gb} GB, preconditioner {pc}")
    out = Server(hbm_budget=int(budget_gb * 2 ** 30), max_active=16, pc=pc).run(reqs)
    out["pc"] = pc
    res = out.pop("results")
    out["iterations_mean"] = sum(r.iters for r in res) / max(len(res), 1)
    out["unknowns_total"] = sum(r.unknowns for r in res if r.converged)
    out["budget_gb"] = budget_gb
    out["stream"] = f"serving_stream({n}, 20 Hz, seed 501)"
    log(f"[bench] serving: {out['completed']}/{n} in {out['makespan_s']:.2f} s, "
        f"p50 {out['latency_p50_ms']:.1f} ms p99 {out['latency_p99_ms']:.1f} ms")
    return out


def cohort_bursts(m=8):
    """Bursts of m same-shape requests started together and stepped with
    stk_step_batch until all are done, with the cross-request batched patch
    solves off and on (best of two runs each)."""
    import torch
    from workloads import small
    from paper_2107_00820_amd import Hierarchy, stk_step_batch

    def burst(dim, n, L, g, cross):
        os.environ["STK_CROSS_BATCH"] = cross
        wls = [small(dim, n, L, gamma=g, dr=10.0 ** (4 + k % 5), n_sinkers=24, seed=3 * 10 ** 6 + k)
               for k in range(m)]
        hs = [Hierarchy.from_workload(w) for w in wls]
        rhs = [h.stk_rhs() for h in hs]
        torch.cuda.synchronize()
        t = time.perf_counter()
        for h, (bu, bp) in zip(hs, rhs):
            h.stk_solve_begin(bu, bp, eager=True)
        infos = [None] * m
        while any(i is None for i in infos):
            stk_step_batch([h for h, i in zip(hs, infos) if i is None])
            for k, h in enumerate(hs):
                if infos[k] is None:
                    infos[k] = h.stk_poll()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        for h in hs:
            h.close()
        return dt

    out = {}
    for dim, n, L, g in ((2, 64, 3, 1e3), (2, 128, 4, 1e3), (3, 8, 2, 1e4), (3, 16, 2, 1e4)):
        t = {c: min(burst(dim, n, L, g, c) for _ in range(2)) for c in ("0", "1")}
        key = f"{m}x_{dim}d_{n}_L{L}"
        out[key] = {"ms_off": 1e3 * t["0"], "ms_on": 1e3 * t["1"]}
        log(f"[bench] burst {key}: batching off {1e3 * t['0']:.1f} ms, on {1e3 * t['1']:.1f} ms")
    os.environ["STK_CROSS_BATCH"] = "1"
    return out


def q3_leg(steps):
    """[Q3]^2 x P2disc on the 2D 128^2 mesh (4 levels, 24 sinkers) with the
    settings of the paper's table "linear" (P1, gamma 1000, contrast 1e10,
    F-cycles, 5 + 5 relaxation steps, FGMRES(30) to a 1e6 reduction): timed
    solves, and the degree-3 patch-solve kernel's rate on the finest level
    from HIP events in one plain-launch solve."""
    import json as _json
    import torch
    from workloads import PAPER_LINEAR_Q3, PAPER_LINEAR_Q3_PRINTED
    from paper_2107_00820_amd import Hierarchy
    key = (1, 1000.0, 1e10)
    wl = PAPER_LINEAR_Q3[key]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = Hierarchy.from_workload(wl)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    bu, bp = h.stk_rhs()
    xu, xp = h.zeros_u(), h.zeros_p()
    kw = dict(rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit, xu=xu, xp=xp, cycle=wl.cycle)
    _, _, info = h.stk_solve(bu, bp, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, _, info = h.stk_solve(bu, bp, **kw)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    h.stk_profile(True, reps=1)
    h.stk_solve(bu, bp, eager=True, **kw)
    n_f, ms_f, by_f = h.stk_profile_read(2)
    h.stk_profile(False)
    h.close()
    n_u, n_p = wl.unknowns()
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "paper_tables_oracle.json")
    orc = _json.load(open(golden)).get(wl.name, {}).get("iters")
    ach = by_f / (ms_f * 1e-3) / 1e9 if ms_f > 0 else 0.0
    log(f"[bench] Q3 {wl.name}: {info['iters']} iterations (oracle {orc}, paper {PAPER_LINEAR_Q3_PRINTED[key]}), "
        f"{1e3 * t:.1f} ms, fine-level patch solves {ach:.0f} GB/s")
    return {"workload": wl.name, "degree": 3, "unknowns": n_u + n_p,
            "unknowns_paper_convention": 2 * (3 * wl.n_fine + 1) ** 2 + n_p, "setup_s": t_setup,
            "ms_per_solve": 1e3 * t, "dof_per_s": (n_u + n_p) / t, "iterations": info["iters"],
            "iterations_oracle": orc, "iterations_paper": PAPER_LINEAR_Q3_PRINTED[key], "rel_res": info["rel_res"],
            "patch_solve_fine_level": {"kernel": "k3_asm_solves", "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS,
                                       "avg_launch_us": 1e3 * ms_f / max(n_f, 1),
                                       "algorithmic_bytes_per_launch": by_f / max(n_f, 1),
                                       "launches_per_solve": n_f}}


def q3_3d_leg(steps):
    """[Q3]^3 x P2disc on 3D 16^3 cells (3 levels, 24 sinkers, contrast 1e8,
    P1, gamma 1000, F-cycles, 5 + 5 relaxation steps, 1e6 reduction): setup
    (cell matrices, batched 375-unknown patch inversions) and timed solves,
    and the patch solves' rate on the finest level (packed-equivalent bytes
    of the symmetric inverses: the stored tiles read 5.7% more)."""
    import torch
    from workloads import Q3_3D_BENCH as wl
    from paper_2107_00820_amd import Hierarchy
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = Hierarchy.from_workload(wl)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    bu, bp = h.stk_rhs()
    xu, xp = h.zeros_u(), h.zeros_p()
    kw = dict(rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit, xu=xu, xp=xp, cycle=wl.cycle)
    _, _, info = h.stk_solve(bu, bp, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, _, info = h.stk_solve(bu, bp, **kw)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    h.stk_profile(True, reps=1)
    h.stk_solve(bu, bp, eager=True, **kw)
    n_f, ms_f, by_f = h.stk_profile_read(2)
    h.stk_profile(False)
    h.close()
    n_u, n_p = wl.unknowns()
    ach = by_f / (ms_f * 1e-3) / 1e9 if ms_f > 0 else 0.0
    log(f"[bench] Q3 3D {wl.name}: {info['iters']} iterations, setup {t_setup:.2f} s, {1e3 * t:.1f} ms per solve, "
        f"fine-level patch solves {ach:.0f} GB/s")
    return {"workload": wl.name, "degree": 3, "unknowns": n_u + n_p, "setup_s": t_setup, "ms_per_solve": 1e3 * t,
            "dof_per_s": (n_u + n_p) / t, "iterations": info["iters"], "rel_res": info["rel_res"],
            "patch_solve_fine_level": {"kernel": "k3d_patch_solve", "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS,
                                       "avg_launch_us": 1e3 * ms_f / max(n_f, 1),
                                       "algorithmic_bytes_per_launch": by_f / max(n_f, 1),
                                       "launches_per_solve": n_f}}


def newton_leg(name):
    """The viscoplastic problem solved by Newton's method on the GPU
    (stk_newton: relinearise, FGMRES step, line search), timed whole."""
    import torch
    from workloads import NEWTON
    from paper_2107_00820_amd import Hierarchy
    from paper_2107_00820_amd.tune import load_asm_tuning
    wl = NEWTON[name]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = Hierarchy.from_workload(wl)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    h.apply_asm_tuning(load_asm_tuning())
    _, _, info = h.stk_newton(rtol=1e-8, maxit=30, lin_rtol=1e-6)
    h.close()
    n_u, n_p = wl.unknowns()
    log(f"[bench] newton {name}: {info['iters']} steps, linear {info['lin_iters']}, {info['t_s']:.2f} s")
    return {"workload": name, "unknowns": n_u + n_p, "steps": info["iters"], "converged": info["converged"],
            "rel_res": info["rel_res"], "lin_iters": info["lin_iters"], "alpha": info["alpha"],
            "t_s": info["t_s"], "setup_s": t_setup, "tau_y": wl.tau_y}


MIXED_REASON = ("the FP32 V-cycle cannot represent A_gamma's near-kernel at gamma / mu_min = 1e4 / 1e-5: "
                "rounding the patch inverses, transfers or applies to FP32 perturbs the divergence-free "
                "components by eps32 gamma / mu_min >> 1")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default=DEFAULT_CONFIG)
    ap.add_argument("--form", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the upper-triangular and F-cycle variants")
    ap.add_argument("--no-extra", action="store_true", help="skip the 2D 128^2 and 3D 32^3 legs")
    ap.add_argument("--serving", type=int, default=200)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--serving-pc", default="full", choices=["full", "upper"])
    ap.add_argument("--trace", action="store_true",
                    help="timed solves only (no event-timing pass, no extra legs, no serving, no oracle)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the "
              "decomposition over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.trace:
        args.no_extra = args.no_serving = args.no_cpu_baseline = True

    import torch
    from workloads import CONFIGS, PAPER_LINEAR_Q3, Q3_3D_BENCH
    from paper_2107_00820_amd import Hierarchy

    # the named configurations, and (for profiling) the degree-3 settings by name
    named = dict(CONFIGS, **{w.name: w for w in PAPER_LINEAR_Q3.values()}, **{Q3_3D_BENCH.name: Q3_3D_BENCH})
    wl = named[args.config]
    n_u, n_p = wl.unknowns()
    dof = n_u + n_p
    log(f"[bench] workload {wl.name}: {dof} unknowns")
    forms = ["fp64", "mixed"] if args.form == "both" else [args.form]
    if not args.no_variants:
        forms += ["fp64_upper", "fp64_F"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = Hierarchy.from_workload(wl, mixed=1 if any(f.startswith("mixed") for f in forms) else 0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    log(f"[bench] setup {t_setup:.3f} s")
    # patch-solve variant per level and precision (bit-identical results): the
    # recorded tuning table if it covers the levels, else a live tuning pass
    from paper_2107_00820_amd.tune import load_asm_tuning
    t0 = time.perf_counter()
    tune = h.apply_asm_tuning(load_asm_tuning())
    tune_src = "paper_2107_00820_amd/asm_tuning.json"
    if getattr(wl, "degree", 2) == 2 and len(tune) < (h.L - 1) * (2 if h.desc.mixed else 1):
        tune, tune_src = h.stk_autotune(reps=5), "live (stk_autotune)"
    t_tune = time.perf_counter() - t0
    log(f"[bench] patch-solve variants ({tune_src}, {t_tune:.3f} s): {tune}")
    bu, bp = h.stk_rhs()
    xu, xp = h.zeros_u(), h.zeros_p()
    res = {}
    for form in forms:
        steps = args.steps if form in ("fp64", "mixed") else max(2, args.steps // 2)
        res[form] = time_form(h, wl, bu, bp, xu, xp, form, steps, args.warmup, not args.trace)
        if not res[form]["converged"] and form.startswith("mixed"):
            res[form]["reason"] = MIXED_REASON
    r = res.get("fp64")
    if r is None or r["value"] is None:
        raise SystemExit("the FP64 form did not reach the residual")
    out = {"metric": METRIC, "value": r["value"], "unit": "DoF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": wl.name, "dim": wl.dim, "n_fine": wl.n_fine, "levels": wl.levels,
                      "n_sinkers": wl.n_sinkers, "dr": wl.dr, "gamma": wl.gamma, "seed": wl.seed,
                      "coef_kind": wl.coef_kind, "nu_pre": wl.nu_pre, "nu_post": wl.nu_post,
                      "restart": wl.restart, "rtol": wl.rtol, "unknowns": dof, "iterations": r["iterations"],
                      "setup_s": t_setup, "setup_plus_solve_dof_per_s": dof / (t_setup + r["ms_per_step"] / 1e3),
                      "form": "fp64"},
           "latency_ms": {"p50": r["p50_ms"], "p99": r["p99_ms"]},
           "forms": {f: {k: v for k, v in res[f].items() if k not in ("prof", "t_total")} for f in res}}
    if "prof" in r:
        out["roofline"] = roofline_of(h, wl, r, r["t_total"] / args.steps)
    out["autotune"] = {"asm_variant": {f"level{l}_{p}": v for (l, p), v in sorted(tune.items())},
                       "source": tune_src, "seconds": t_tune}
    h.close()
    if not args.no_extra:
        out["other_workloads"] = {}
        for name in ("sinker_3d_32cu_L3", "sinker_2d_128sq_L4"):
            if name == wl.name:
                continue
            log(f"[bench] {name}")
            out["other_workloads"][name] = other_workload(name, max(2, args.steps // 2))
    if not args.no_extra:
        out["newton"] = newton_leg("newton_3d_32cu_L3")
        out["q3"] = q3_leg(max(2, args.steps // 2))
        out["q3_3d"] = q3_3d_leg(2)
    if not args.no_serving and args.serving > 0:
        out["serving"] = serving_leg(args.serving, args.budget_gb, args.serving_pc)
        # the same stream with the cross-request batched patch solves turned on
        os.environ["STK_CROSS_BATCH"] = "1"
        try:
            nb = serving_leg(args.serving, args.budget_gb, args.serving_pc, warm=False)
            bursts = cohort_bursts()
        finally:
            del os.environ["STK_CROSS_BATCH"]
        out["serving"]["with_cross_batching"] = {k: nb[k] for k in (
            "completed", "makespan_s", "dof_per_s", "latency_p50_ms", "latency_p99_ms", "solve_s_mean",
            "queue_s_mean")}
        out["serving"]["same_shape_bursts"] = bursts
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle, bounded sample) ...")
        out["cpu_baseline"] = cpu_baseline(wl)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
