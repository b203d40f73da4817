#!/usr/bin/env python3
"""Benchmark of the Stokes-preconditioned BEFE hot path on one MI355X.

Workload (default): plane Couette flow, Re = 1000, box 2pi/1.14 x 2 x 2pi/2.5,
grid 48 x 65 x 48 (Fourier x Chebyshev x Fourier), dt = T = 100, initial field
= laminar flow + the seeded divergence-free perturbation (energy 1e-2, seed 0).

A timed step is one evaluation of Phi_dt(u) = (I - dt L)^{-1}(u + dt N(u)) in
FP64 on a field resident in HBM; `value` is FP64 evaluations per second. The
same JSON line also reports the mixed-precision Phi rate, the JVP rates (the
GMRES matvec), the roofline position of the dominant kernel and of the whole
step (timed live with HIP events), the CPU oracle timed on whole evaluations,
and Newton-GMRES to ||r|| < 1e-10 with FP64 and mixed Jacobian actions. The
perturbation family's starts do not converge at Re 1000, so the Newton leg
starts from a non-laminar equilibrium continued in Re: found at 32x33x32,
Re 400, interpolated to the workload grid and continued to Re 950 (not timed);
the timed solves converge it at Re 1000, and the oracle's residual norm is
evaluated at every iterate.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    "couette_48x65x48_re1000_dt100": dict(nx=48, ny=65, nz=48, re=1000.0, dt=100.0,
                                           lx=2 * math.pi / 1.14, lz=2 * math.pi / 2.5),
    "couette_16x17x16_re400_dt100": dict(nx=16, ny=17, nz=16, re=400.0, dt=100.0,
                                          lx=2 * math.pi / 1.14, lz=2 * math.pi / 2.5),
    "couette_32x33x32_re400_dt100": dict(nx=32, ny=33, nz=32, re=400.0, dt=100.0,
                                          lx=2 * math.pi / 1.14, lz=2 * math.pi / 2.5),
    "couette_96x97x96_re2000_dt100": dict(nx=96, ny=97, nz=96, re=2000.0, dt=100.0,
                                           lx=4 * math.pi, lz=2 * math.pi, input="streak_roll"),
}
DEFAULT = "couette_48x65x48_re1000_dt100"
HBM_PEAK_GBS = 8000.0
CAL_COPY_BYTES = 256 * 1024 * 1024

# HBM traffic of the longest Phi kernels measured with rocprofv3 --pmc FETCH_SIZE
# and --pmc WRITE_SIZE over this script (KiB per dispatch, see profiles/), the
# calibration factors from the 256 MiB copy above, and the hash of the kernel's
# sources (KERNEL_SOURCES) the counters were taken with: a changed source
# reports traffic null.
KERNEL_SOURCES = {
    "k_stokes_solve": ["kernels.hip", "solve_row.h", "solve_core.h", "device_common.h"],
    "k_z_product": ["zline.hip", "device_common.h"],
}
MEASURED_TRAFFIC = {
    "couette_48x65x48_re1000_dt100": {
        # 256 MiB copy: FETCH_SIZE 131095.3 KiB, WRITE_SIZE 262144.0 KiB
        "k_stokes_solve": {
            "fetch_kib": 5611.6, "write_kib": 3674.3,
            "fetch_factor": 262144.0 / 131095.3, "write_factor": 1.0,
            "sources_sha256": "6d8eab5a02c7bee69b1cf019c8fb8eb0cc3333c2d80294df2cb5a5525c6c53f6",
        },
        "k_z_product": {
            "fetch_kib": 3337.1, "write_kib": 5265.0,
            "fetch_factor": 262144.0 / 131095.3, "write_factor": 1.0,
            "sources_sha256": "9a914b3f355c42eb20a1920283f7ef6e70b740bf1c393267c7e68a08b5f87e08",
        },
    },
}
STAGE_OF_KERNEL = {}  # profiler kernel name -> sp_time_stage stage (filled in main)


def sources_sha256(kernel="k_stokes_solve"):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1804_05087_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def spectral_field_bytes(w):
    """S: one complex FP64 spectral field [nx][nz/2+1][ny] (16 bytes per entry)."""
    return w["nx"] * (w["nz"] // 2 + 1) * w["ny"] * 16


def solve_modes(w):
    """Fourier modes whose solve loads a record: all but the Nyquist row and column."""
    nzh = w["nz"] // 2 + 1
    return w["nx"] * nzh - (nzh + w["nx"] - 1)


def algorithmic_bytes(w, fp32=False, jvp=False, fused=False):
    """Compulsory HBM bytes per launch of each kernel (read once + written once).

    fused: the z-line kernel takes the inverse x transforms itself, reading
    the five y-valued fields instead of the six x-physical ones, and there is
    no separate inverse x launch.

    The per-mode solve follows the phase count of the whole step, 27 S per
    evaluation with S one spectral field: its phase (Chebyshev analysis, right-
    hand side u/dt + N, solve) reads the three product fields and u and writes
    Phi, 9 S. Its precomputed per-mode records are plan data, reported apart
    (record_bytes)."""
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    nzm, pz, px = nz // 2, 3 * nz // 2, 3 * nx // 2
    c = 8 if fp32 else 16            # complex element of the transform path
    r = 4 if fp32 else 8
    yv1 = ny * nzm * nx * c          # one y-valued spectral field
    xp1 = ny * px * nzm * c          # one x-physical field
    S = spectral_field_bytes(w)
    base = 6 * ny * px * pz * r if jvp else 0
    ab = {
        "k_synth_y": 3 * nx * nzm * ny * 16 + 5 * yv1,
        "k_fft_x_inv": 5 * yv1 + 6 * xp1,
        "k_z_product": 6 * xp1 + 3 * xp1 + base,
        "k_fft_x_fwd": 3 * xp1 + 3 * yv1,
        "k_stokes_solve": 9 * S,
    }
    if fused:
        del ab["k_fft_x_inv"]
        ab["k_z_product"] = 5 * yv1 + 3 * xp1 + base
    return ab


def record_bytes(w):
    """Per-mode solve records (sweep factors of the two operators, influence
    solutions, 2x2 inverse influence matrices: 6 (N+1) + 12 doubles) and the
    three weight rows read by one solve launch."""
    n1 = w["ny"]
    stride = ((6 * n1 + 12) + 1) // 2 * 2
    return solve_modes(w) * stride * 8 + 3 * n1 * 8


def time_loop(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1000.0, wall


def _host_cpu():
    """CPU model and the thread count the host grants this process."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        n = min(n, int(omp))
    return model, max(1, n)


def cpu_baseline(w, u_np, reps=3):
    """The CPU oracle timed on the same workload: whole Phi evaluations (the
    dealiased nonlinear term and the dense solve of every mode), one warm-up
    and then the median of `reps`, on one thread and on every thread the host
    grants; the per-mode factorisations are set up before timing, like the
    GPU plan. `value` is the faster of the two settings."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.befe import Befe
    from oracle.grid import Grid
    model, nthreads = _host_cpu()
    g = Grid(w["nx"], w["ny"], w["nz"], w["lx"], w["lz"])
    t0 = time.perf_counter()
    B = Befe(g, w["re"], w["dt"])
    setup_s = time.perf_counter() - t0
    med = {}
    for threads in sorted({1, nthreads}):
        with threadpool_limits(limits=threads):
            B.phi(u_np)
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                B.phi(u_np)
                ts.append(time.perf_counter() - t0)
        med[threads] = float(np.median(ts))
        log("cpu oracle", threads, "threads: Phi", ts)
    best = min(med, key=med.get)
    return {"value": round(1.0 / med[best], 4), "unit": "evals/s", "cores": best,
            "kind": "oracle",
            "sample": (f"whole Phi evaluations of the workload, median of {reps} after one "
                       f"warm-up, on 1 and {nthreads} threads"),
            "seconds_per_eval": {str(k): round(v, 3) for k, v in med.items()},
            "setup_seconds": round(setup_s, 2), "cpu_model": model,
            "threads_available": nthreads}


def dt_sweep(seeds=range(10), dts=(1.0, 10.0, 100.0), max_krylov=400,
             first_rtols=(1e-2, 1e-3, 1e-6), solve_rtol=1e-4, max_newton=30):
    """Krylov counts against the time step at 32x33x32, Re = 400, from the
    perturbation family (energy 1e-2, seeds 0-9): for each dt and seed, the
    GMRES iterations of the first Newton step to each relative tolerance in
    `first_rtols` (at most `max_krylov`, with the relative residual reached),
    then the trust-region (hookstep) Newton solve to ||r|| < 1e-10 with GMRES
    to `solve_rtol` (converged flag, Newton steps, total Krylov iterations,
    Phi/JVP evaluations, seconds, distance of the root from laminar flow)."""
    import torch
    from paper_1804_05087_amd import Plan, synth
    w = WORKLOADS["couette_32x33x32_re400_dt100"]
    dev = torch.device("cuda", 0)
    dims = (w["nx"], w["ny"], w["nz"])
    lam = torch.from_numpy(synth.laminar_field(*dims)).to(dev)
    out = {}
    for dt in dts:
        P = Plan(*dims, w["lx"], w["lz"], w["re"], dt, device=dev)
        rows = []
        for seed in seeds:
            u0 = torch.from_numpy(synth.perturbation_field(*dims, w["lx"], w["lz"],
                                                           seed=seed)).to(dev)
            row = {"seed": seed}
            for rt in first_rtols:
                u = u0.clone()
                first = P.newton_gmres(u, max_newton=1, max_krylov=max_krylov, gmres_rtol=rt,
                                       newton_tol=0.0)
                row[f"K_first_{rt:g}"] = first["krylov"][0]
                row[f"relres_first_{rt:g}"] = float(f"{first['gmres_relres'][0]:.2e}")
            u = u0.clone()
            full = P.newton_hookstep(u, max_newton=max_newton, max_krylov=max_krylov,
                                     gmres_rtol=solve_rtol, newton_tol=1e-10)
            row.update({"converged": full["converged"], "newton_iters": full["newton_iters"],
                        "K_total": full["total_krylov"], "actions": full["total_actions"],
                        "final_res": float(f"{full['res_norm'][-1]:.3e}"),
                        "seconds": round(full["seconds"], 3),
                        "dist_to_laminar_L2": float(f"{P.norm((u - lam).contiguous()):.3e}")})
            log("dt", dt, row)
            rows.append(row)
        summary = {}
        for rt in first_rtols:
            ks = [r[f"K_first_{rt:g}"] for r in rows]
            summary[f"K_first_{rt:g}"] = {"mean": sum(ks) / len(ks), "min": min(ks),
                                          "max": max(ks)}
        conv = [r for r in rows if r["converged"]]
        summary["converged"] = len(conv)
        if conv:
            summary["K_total_mean_converged"] = sum(r["K_total"] for r in conv) / len(conv)
        out[str(dt)] = {"summary": summary, "runs": rows}
    return {"metric": "krylov_iterations_vs_dt", "workload": "couette_32x33x32_re400",
            "max_krylov": max_krylov, "solve_gmres_rtol": solve_rtol, "energy": 1e-2,
            "newton": "hookstep", "sweep": out}


def _timesteps(rep, n):
    """BEFE steps spent by a Newton solve on an n-step operator: every residual
    and every Jacobian action costs n (linearised) steps, and each Newton step
    recomputes its n - 1 step trajectory for the chain rule."""
    return rep["total_actions"] * n + rep["newton_iters"] * (n - 1)


def _history(rep, n):
    """(cumulative BEFE steps, ||r||) after each Newton iteration."""
    out, steps = [], n
    out.append((steps, rep["res_norm"][0]))
    for i, k in enumerate(rep["krylov"]):
        trials = rep["trials"][i] if i < len(rep["trials"]) else 0
        steps += (k + trials) * n + (n - 1)
        out.append((steps, rep["res_norm"][i + 1]))
    return [(s_, float(f"{r:.3e}")) for s_, r in out]


def _steps_to_reduction(hist, factor):
    """BEFE steps after which ||r|| first fell below factor * ||r_0||."""
    r0 = hist[0][1]
    for steps, r in hist:
        if r <= factor * r0:
            return steps
    return None


def gint_compare(seeds=(8, 1, 0, 2, 3), re_find=400.0, re=380.0, t_stokes=100.0,
                 int_cases=((0.5, 1 / 32), (1.0, 1 / 32), (2.0, 1 / 32), (1.0, 1 / 64),
                            (2.0, 1 / 64), (0.5, 1 / 32, 1), (1.0, 1 / 32, 1),
                            (2.0, 1 / 32, 1)),
                 max_krylov=1000, rtol=1e-4, max_newton=12):
    """The paper's comparison of the Stokes operator B_T - I (one BEFE step,
    T = 100) with the time-integration operator (B_dt)^{T/dt} - I (BEFE steps
    of dt = 1/32 and 1/64, SBDF2 steps of 1/32) in plane Couette flow (Sec. 3.3): a
    non-laminar equilibrium is
    found at Re = 400 with the Stokes operator from the perturbation family at
    32x33x32, Re is lowered to 380, and both operators' hookstep Newton solves
    start from it; the cost is counted in BEFE time steps."""
    import torch
    from paper_1804_05087_amd import Plan, synth
    w = WORKLOADS["couette_32x33x32_re400_dt100"]
    dev = torch.device("cuda", 0)
    dims = (w["nx"], w["ny"], w["nz"])
    box = (w["lx"], w["lz"])
    lam = torch.from_numpy(synth.laminar_field(*dims)).to(dev)
    P = Plan(*dims, *box, re_find, t_stokes, device=dev)
    start = None
    for seed in seeds:
        u = torch.from_numpy(synth.perturbation_field(*dims, *box, seed=seed)).to(dev)
        rep = P.newton_hookstep(u, max_newton=30, max_krylov=400, gmres_rtol=rtol,
                                newton_tol=1e-12)
        dist = P.norm((u - lam).contiguous())
        log("equilibrium search seed", seed, rep["converged"], rep["res_norm"][-1], dist)
        if rep["converged"] and dist > 1e-3:
            start = {"seed": seed, "dist_to_laminar_L2": dist, "res": rep["res_norm"][-1]}
            break
    if start is None:
        return {"metric": "gint_vs_stokes_timesteps", "error": "no non-laminar equilibrium"}
    u_eq = u.clone()
    out = {"metric": "gint_vs_stokes_timesteps", "workload": "couette_32x33x32",
           "re_found": re_find, "re": re, "start": start, "gmres_rtol": rtol,
           "max_krylov": max_krylov, "newton_tol": 1e-10, "runs": {}}
    finals = {}
    PS = Plan(*dims, *box, re, t_stokes, device=dev)
    uS = u_eq.clone()
    rep = PS.newton_hookstep(uS, max_newton=max_newton, max_krylov=max_krylov,
                             gmres_rtol=rtol, newton_tol=1e-10)
    finals["stokes"] = uS
    out["runs"][f"stokes_T{t_stokes:g}"] = {
        "converged": rep["converged"], "newton_iters": rep["newton_iters"],
        "total_krylov": rep["total_krylov"], "timesteps": _timesteps(rep, 1),
        "seconds": round(rep["seconds"], 3), "history": _history(rep, 1)}
    log("stokes", out["runs"][f"stokes_T{t_stokes:g}"])
    for case in int_cases:
        T, dt_int = case[0], case[1]
        scheme = case[2] if len(case) > 2 else 0
        # SBDF2 (scheme 1): the plan's dt is the implicit step 2 dt_int / 3
        PI = Plan(*dims, *box, re, dt_int * (2.0 / 3.0 if scheme else 1.0), device=dev)
        n = int(round(T / dt_int))
        PI.set_steps(n)
        PI.set_scheme(scheme)
        uI = u_eq.clone()
        rep = PI.newton_hookstep(uI, max_newton=max_newton, max_krylov=max_krylov,
                                 gmres_rtol=rtol, newton_tol=1e-10)
        key = f"int{'_sbdf2' if scheme else ''}_T{T:g}_dt1/{round(1 / dt_int)}"
        finals[key] = uI
        out["runs"][key] = {
            "nsteps": n, "dt": dt_int, "scheme": "sbdf2" if scheme else "befe",
            "krylov": rep["krylov"],
            "converged": rep["converged"], "newton_iters": rep["newton_iters"],
            "total_krylov": rep["total_krylov"], "timesteps": _timesteps(rep, n),
            "seconds": round(rep["seconds"], 3), "history": _history(rep, n),
            "dist_to_stokes_root_L2": P.norm((uI - uS).contiguous())}
        log(key, out["runs"][key])
        del PI
    for v in out["runs"].values():
        for f in (1e-4, 1e-6):
            v[f"steps_to_reduce_{f:g}"] = _steps_to_reduction(v["history"], f)
    st = out["runs"][f"stokes_T{t_stokes:g}"]
    for f in (1e-4, 1e-6):
        key = f"steps_to_reduce_{f:g}"
        ints = [v[key] for k, v in out["runs"].items() if k.startswith("int") and v[key]]
        if ints and st[key]:
            out[f"int_best_over_stokes_{f:g}"] = min(ints) / st[key]
    done = [v["timesteps"] for k, v in out["runs"].items() if k.startswith("int") and v["converged"]]
    if done and st["converged"]:
        out["int_best_over_stokes_converged"] = min(done) / st["timesteps"]
    out["root_dist_to_laminar_L2"] = P.norm((uS - lam).contiguous())
    return out


def _truncate(u, dims):
    """Spectral truncation of a canonical field to a smaller grid (Fourier
    modes |m| < n/2 in x and z, Chebyshev coefficients n < ny; Nyquist zero)."""
    import numpy as np
    nx, ny, nz = dims
    a = u.cpu().numpy()
    NX = a.shape[1]
    out = np.zeros((3, nx, nz // 2 + 1, ny), dtype=np.complex128)
    for i in range(nx):
        if i == nx // 2:
            continue
        m = i if i < nx // 2 else i - nx
        out[:, i, :nz // 2, :] = a[:, m % NX, :nz // 2, :ny]
    return out


def spectra_report(dims=(12, 17, 12), re_find=400.0, re=500.0, seeds=(8, 1, 0, 2, 3),
                   stokes_T=(1e-4, 0.1, 100.0), int_T=(1.0, 10.0), dt_int=0.03125):
    """Spectra of the Newton operators' Jacobians (Sec. 3.5) on a small grid of
    the Couette box, restricted to admissible fields. The base state is a
    non-laminar equilibrium: found by the Stokes solver at 32x33x32, Re = 400
    from the perturbation family, truncated to the small grid, re-converged
    there and continued to Re = 500 (laminar flow if any of that fails).
    Operators: G^Stokes_T for several T (with Beaume's rescaling) and G^int_T
    with dt = 0.03125. Eigenvalues on the host."""
    import torch
    from paper_1804_05087_amd import SP_OP_PHI, Plan, spectra, synth
    dev = torch.device("cuda", 0)
    box = (2 * math.pi / 1.14, 2 * math.pi / 2.5)
    lam0 = torch.from_numpy(synth.laminar_field(*dims)).to(dev)
    base, where = lam0.clone(), "laminar"
    big = (32, 33, 32)
    lamb = torch.from_numpy(synth.laminar_field(*big)).to(dev)
    PB = Plan(*big, *box, re_find, 100.0, device=dev)
    for seed in seeds:
        u = torch.from_numpy(synth.perturbation_field(*big, *box, seed=seed)).to(dev)
        rep = PB.newton_hookstep(u, max_newton=30, max_krylov=400, gmres_rtol=1e-4,
                                 newton_tol=1e-12)
        if not (rep["converged"] and PB.norm((u - lamb).contiguous()) > 1e-3):
            continue
        us = torch.from_numpy(_truncate(u, dims)).to(dev)
        ok = True
        for r2 in (re_find, 450.0, re):
            P2 = Plan(*dims, *box, r2, 100.0, device=dev)
            rep = P2.newton_hookstep(us, max_newton=30, max_krylov=400, gmres_rtol=1e-6,
                                     newton_tol=1e-12)
            ok = ok and rep["converged"]
            log("spectra base seed", seed, "Re", r2, rep["converged"], rep["res_norm"][-1])
        d = P2.norm((us - lam0).contiguous())
        if ok and d > 1e-3:
            base = us.clone()
            where = (f"equilibrium (seed {seed} at 32x33x32, Re 400, truncated and continued; "
                     f"||u - U_lam|| = {d:.4f})")
            break
    log("spectra base:", where)
    out = {"metric": "jacobian_spectra", "grid": list(dims), "re": re, "base": where,
           "operators": {}}

    # the admissible subspace, from one BEFE step's Jacobian (shared by all operators)
    Q = spectra.admissible_basis(spectra.jacobian_dense(Plan(*dims, *box, re, 1.0, device=dev),
                                                        base, op=SP_OP_PHI))

    def one(P, T, scale):
        t0 = time.perf_counter()
        J = spectra.jacobian_dense(P, base)
        lam = spectra.eigenvalues(spectra.restrict(J, Q))
        s = spectra.summary(spectra.beaume_scale(lam, T) if scale else lam)
        s["admissible_dim"] = int(Q.shape[1])
        s["seconds"] = round(time.perf_counter() - t0, 2)
        return s

    for T in stokes_T:
        out["operators"][f"stokes_T{T:g}_beaume_scaled"] = s = one(
            Plan(*dims, *box, re, T, device=dev), T, True)
        log("stokes", T, s)
    PI = Plan(*dims, *box, re, dt_int, device=dev)
    for T in int_T:
        PI.set_steps(int(round(T / dt_int)))
        out["operators"][f"int_T{T:g}"] = s = one(PI, T, False)
        log("int", T, s)
    # SBDF2 steps of dt_int (the plan's dt is the implicit step 2 dt_int / 3)
    PS = Plan(*dims, *box, re, dt_int * 2.0 / 3.0, device=dev)
    PS.set_scheme(1)
    for T in int_T:
        PS.set_steps(int(round(T / dt_int)))
        out["operators"][f"int_sbdf2_T{T:g}"] = s = one(PS, T, False)
        log("int sbdf2", T, s)
    return out


def advect_compare(seeds=range(5), dts=(10.0, 100.0), max_krylov=400, rtol=1e-3,
                   workload="couette_32x33x32_re400_dt100"):
    """The Stokes step against the step with the laminar advection in its
    implicit operator (Sec. 3.6's proposed remedy) on `workload` (32x33x32,
    Re = 400 by default):
    GMRES iterations of the first Newton step to `rtol` (with the relative
    residual after at most `max_krylov`), and hookstep Newton solves to
    ||r|| < 1e-10 (GMRES to 1e-4), from the energy-1e-2 perturbation family;
    plus the cost of one step of each kind."""
    import torch
    from paper_1804_05087_amd import Plan, synth
    w = WORKLOADS[workload]
    dev = torch.device("cuda", 0)
    dims = (w["nx"], w["ny"], w["nz"])
    box = (w["lx"], w["lz"])
    lam = torch.from_numpy(synth.laminar_field(*dims)).to(dev)
    out = {"metric": "krylov_iterations_stokes_vs_advected", "workload": workload,
           "first_step_rtol": rtol, "max_krylov": max_krylov, "energy": 1e-2, "runs": {}}
    for dt in dts:
        for adv in (False, True):
            P = Plan(*dims, *box, w["re"], dt, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if adv:
                P.set_advection(True)
            build = time.perf_counter() - t0
            u0 = torch.from_numpy(synth.perturbation_field(*dims, *box, seed=0)).to(dev)
            o = P.empty()
            s, _ = time_loop(torch, lambda: P.befe_step(u0, o), 200, 20)
            rows = []
            for seed in seeds:
                u0 = torch.from_numpy(synth.perturbation_field(*dims, *box, seed=seed)).to(dev)
                u = u0.clone()
                first = P.newton_gmres(u, max_newton=1, max_krylov=max_krylov, gmres_rtol=rtol,
                                       newton_tol=0.0)
                u = u0.clone()
                full = P.newton_hookstep(u, max_newton=30, max_krylov=max_krylov,
                                         gmres_rtol=1e-4, newton_tol=1e-10)
                rows.append({"seed": seed, "K_first": first["krylov"][0],
                             "relres_first": float(f"{first['gmres_relres'][0]:.2e}"),
                             "converged": full["converged"], "newton_iters": full["newton_iters"],
                             "K_total": full["total_krylov"], "seconds": round(full["seconds"], 3),
                             "dist_to_laminar_L2": float(f"{P.norm((u - lam).contiguous()):.3e}")})
                log("dt", dt, "advected" if adv else "stokes", rows[-1])
            key = f"dt{dt:g}_{'advected' if adv else 'stokes'}"
            ks = [r["K_first"] for r in rows]
            conv = [r for r in rows if r["converged"]]
            out["runs"][key] = {
                "phi_us": round(1e6 * s / 200, 2), "build_seconds": round(build, 3),
                "K_first_mean": sum(ks) / len(ks),
                "relres_first_mean": sum(r["relres_first"] for r in rows) / len(rows),
                "converged": len(conv),
                "K_total_mean_converged": (sum(r["K_total"] for r in conv) / len(conv)
                                           if conv else None),
                "runs": rows}
    return out


def symmetric_compare(seeds=range(10), energies=(1e-2, 5e-2), re_find=400.0, re=380.0,
                      t_stokes=100.0, int_cases=((1.0, 1 / 32), (2.0, 1 / 32), (1.0, 1 / 64),
                                                 (2.0, 1 / 64), (1.0, 1 / 128),
                                                 (1.0, 1 / 32, 1), (2.0, 1 / 32, 1),
                                                 (1.0, 1 / 64, 1)),
                      max_krylov=1000, rtol=1e-4):
    """The Stokes / time-integration comparison of gint_compare confined to the
    shift-reflect invariant subspace of EQ1's symmetry group (the paper's EQ1
    computations stay in it): starts are the perturbation family projected
    onto the subspace (perturbation rescaled to the given energy); the first
    non-laminar invariant equilibrium found at Re = 400 is continued to 380."""
    import torch
    from paper_1804_05087_amd import Plan, synth
    w = WORKLOADS["couette_32x33x32_re400_dt100"]
    dev = torch.device("cuda", 0)
    dims = (w["nx"], w["ny"], w["nz"])
    box = (w["lx"], w["lz"])
    lam = torch.from_numpy(synth.laminar_field(*dims)).to(dev)
    P = Plan(*dims, *box, re_find, t_stokes, device=dev)
    P.set_symmetry(True)
    found, tried = None, []
    for energy in energies:
        for seed in seeds:
            pert = torch.from_numpy(synth.perturbation(*dims, *box, seed, 0.5)).to(dev)
            P.symmetrize(pert)
            e = 0.5 * P.norm(pert) ** 2
            u = (lam + pert * math.sqrt(energy / e)).contiguous()
            rep = P.newton_hookstep(u, max_newton=40, max_krylov=400, gmres_rtol=1e-4,
                                    newton_tol=1e-12)
            d = P.norm((u - lam).contiguous())
            tried.append({"energy": energy, "seed": seed, "converged": rep["converged"],
                          "dist_to_laminar_L2": float(f"{d:.4e}"),
                          "newton_iters": rep["newton_iters"]})
            log("symmetric search", tried[-1])
            if rep["converged"] and d > 1e-3:
                found = u.clone()
                break
        if found is not None:
            break
    out = {"metric": "gint_vs_stokes_timesteps_symmetric", "workload": "couette_32x33x32",
           "subspace": "shift-reflect {1, s1, s2, s1 s2}", "search": tried}
    if found is None:
        return out
    u_eq = found
    runs = {}
    PS = Plan(*dims, *box, re, t_stokes, device=dev)
    PS.set_symmetry(True)
    uS = u_eq.clone()
    rep = PS.newton_hookstep(uS, max_newton=12, max_krylov=max_krylov, gmres_rtol=rtol,
                             newton_tol=1e-10)
    runs[f"stokes_T{t_stokes:g}"] = {
        "converged": rep["converged"], "newton_iters": rep["newton_iters"],
        "total_krylov": rep["total_krylov"], "timesteps": _timesteps(rep, 1),
        "seconds": round(rep["seconds"], 3), "history": _history(rep, 1)}
    log("symmetric stokes", runs[f"stokes_T{t_stokes:g}"])
    for case in int_cases:
        T, dt_int = case[0], case[1]
        scheme = case[2] if len(case) > 2 else 0
        # SBDF2 (scheme 1): the plan's dt is the implicit step 2 dt_int / 3
        PI = Plan(*dims, *box, re, dt_int * (2.0 / 3.0 if scheme else 1.0), device=dev)
        PI.set_symmetry(True)
        n = int(round(T / dt_int))
        PI.set_steps(n)
        PI.set_scheme(scheme)
        uI = u_eq.clone()
        rep = PI.newton_hookstep(uI, max_newton=12, max_krylov=max_krylov, gmres_rtol=rtol,
                                 newton_tol=1e-10)
        key = f"int{'_sbdf2' if scheme else ''}_T{T:g}_dt1/{round(1 / dt_int)}"
        runs[key] = {
            "nsteps": n, "dt": dt_int, "scheme": "sbdf2" if scheme else "befe", "krylov": rep["krylov"],
            "converged": rep["converged"], "newton_iters": rep["newton_iters"],
            "total_krylov": rep["total_krylov"], "timesteps": _timesteps(rep, n),
            "seconds": round(rep["seconds"], 3), "history": _history(rep, n),
            "dist_to_stokes_root_L2": P.norm((uI - uS).contiguous())}
        log("symmetric int", T, dt_int, scheme, runs[key])
        del PI
    out["runs"] = runs
    out["root_dist_to_laminar_L2"] = P.norm((uS - lam).contiguous())
    for f in (1e-4, 1e-6):
        key = f"steps_to_reduce_{f:g}"
        for v in runs.values():
            v[key] = _steps_to_reduction(v["history"], f)
        st = runs[f"stokes_T{t_stokes:g}"][key]
        ints = [v[key] for k, v in runs.items() if k.startswith("int") and v[key]]
        if ints and st:
            out[f"int_best_over_stokes_{f:g}"] = min(ints) / st
    done = [v["timesteps"] for k, v in runs.items() if k.startswith("int") and v["converged"]]
    if done and runs[f"stokes_T{t_stokes:g}"]["converged"]:
        out["int_best_over_stokes_converged"] = min(done) / runs[f"stokes_T{t_stokes:g}"]["timesteps"]
    return out


def mixed_error(workload=DEFAULT, energy=1e-6, max_krylov=200, rtol=1e-4, max_newton=20):
    """Per-Newton-step error of the mixed-precision solves against the FP64 one
    at 48x65x48, Re 1000, dt 100 (same start as the benchmark's Newton solve).
    Each solve advances one Newton step per call, so the iterate after every
    step is kept; the FP64 path is the reference (its Jacobian actions agree
    with the oracle to 1e-12 relative). Reported per step: ||r|| of each
    solve and the volume-normalised L2 distance of each mixed iterate from
    the FP64 iterate of the same step, absolute and relative to the FP64
    Newton update of that step."""
    import torch
    from paper_1804_05087_amd import SP_FP64, SP_MIXED, Plan, synth
    w = WORKLOADS[workload]
    dev = torch.device("cuda", 0)
    P = Plan(w["nx"], w["ny"], w["nz"], w["lx"], w["lz"], w["re"], w["dt"], device=dev)
    u0 = torch.from_numpy(synth.perturbation_field(
        w["nx"], w["ny"], w["nz"], w["lx"], w["lz"], seed=0, energy=energy)).to(dev)
    iterates, res = {}, {}
    for name, prec, kf32 in (("fp64", SP_FP64, False), ("mixed", SP_MIXED, False),
                             ("mixed_krylov_fp32", SP_MIXED, True)):
        P.set_precision(prec)
        uu = u0.clone()
        its, rs = [u0.clone()], []
        for _ in range(max_newton):
            # one Newton step per call; the report also holds ||r|| after the step
            rep = P.newton_gmres(uu, max_newton=1, max_krylov=max_krylov, gmres_rtol=rtol,
                                 newton_tol=1e-10, krylov_fp32=kf32)
            if not rs:
                rs.append(rep["res_norm"][0])
            if rep["newton_iters"] == 1:
                its.append(uu.clone())
                rs.append(rep["res_norm"][-1])
            if rep["converged"] or rep["newton_iters"] == 0:
                break
        iterates[name], res[name] = its, rs
        log("mixed-error", name, "steps", len(its) - 1, "final ||r||", rs[-1])
    P.set_precision(SP_FP64)
    ref = iterates["fp64"]
    out = {"metric": "mixed_vs_fp64_newton_error", "workload": workload,
           "start": {"energy": energy, "seed": 0, "max_krylov": max_krylov, "gmres_rtol": rtol},
           "res_norm": {k: [float(f"{x:.3e}") for x in v] for k, v in res.items()}}
    for name in ("mixed", "mixed_krylov_fp32"):
        rows = []
        for k in range(1, min(len(ref), len(iterates[name]))):
            d = P.norm((iterates[name][k] - ref[k]).contiguous())
            step = P.norm((ref[k] - ref[k - 1]).contiguous())
            rows.append({"step": k, "dist_L2": float(f"{d:.3e}"),
                         "fp64_update_L2": float(f"{step:.3e}"),
                         "dist_over_update": float(f"{d / step:.3e}") if step > 0 else None})
        out[name] = rows
    return out


def re_continuation(dev, u, dims, box, re0, re1, dre, max_krylov=800, rtol=1e-4, tol=1e-10):
    """Hookstep Newton roots at Re = re0, re0 + dre, ..., re1 in the box, each
    the start of the next solve (the step is halved after a failed solve, down
    to dre / 8). Returns the root at re1 (or None) and the path."""
    import torch
    from paper_1804_05087_amd import Plan, synth
    lam = torch.from_numpy(synth.laminar_field(*dims)).to(dev)
    path, re, step = [], re0, dre
    while True:
        P = Plan(*dims, *box, re, 100.0, device=dev)
        x = u.clone()
        rep = P.newton_hookstep(x, max_newton=50, max_krylov=max_krylov, gmres_rtol=rtol,
                                newton_tol=tol)
        dist = P.norm((x - lam).contiguous())
        path.append({"re": re, "converged": rep["converged"], "newton_iters": rep["newton_iters"],
                     "res": float(f"{rep['res_norm'][-1]:.2e}"),
                     "seconds": round(rep["seconds"], 2),
                     "dist_to_laminar_L2": float(f"{dist:.4e}")})
        log("continuation", dims, path[-1])
        del P
        if not rep["converged"] or dist < 1e-3:
            if step <= dre / 8:
                return None, path
            re -= step
            step /= 2
            re += step
            continue
        u = x
        if re >= re1:
            return u, path
        re = min(re + step, re1)


def box_continued_equilibrium(dev, box, dims=(32, 33, 32), re=400.0, nsteps=8):
    """An equilibrium of the box at Re 400: the one of PAPER_BOX found at 32x33x32
    from the perturbation family (seed 8), carried to the box by continuation in
    (Lx, Lz) in nsteps equal steps (halved after a failed solve)."""
    import torch
    from paper_1804_05087_amd import Plan, synth
    lam = torch.from_numpy(synth.laminar_field(*dims)).to(dev)
    P = Plan(*dims, *PAPER_BOX, re, 100.0, device=dev)
    u = torch.from_numpy(synth.perturbation_field(*dims, *PAPER_BOX, seed=8)).to(dev)
    rep = P.newton_hookstep(u, max_newton=30, max_krylov=400, gmres_rtol=1e-4, newton_tol=1e-12)
    if not rep["converged"] or P.norm((u - lam).contiguous()) < 1e-3:
        return None, {"error": "no non-laminar root from seed 8"}
    path, s, ds = [], 0.0, 1.0 / nsteps
    while s < 1.0:
        s1 = min(1.0, s + ds)
        lx = PAPER_BOX[0] + s1 * (box[0] - PAPER_BOX[0])
        lz = PAPER_BOX[1] + s1 * (box[1] - PAPER_BOX[1])
        P = Plan(*dims, lx, lz, re, 100.0, device=dev)
        x = u.clone()
        rep = P.newton_hookstep(x, max_newton=30, max_krylov=400, gmres_rtol=1e-4,
                                newton_tol=1e-11)
        dist = P.norm((x - lam).contiguous())
        path.append({"lx": round(lx, 4), "lz": round(lz, 4), "converged": rep["converged"],
                     "newton_iters": rep["newton_iters"],
                     "dist_to_laminar_L2": float(f"{dist:.4e}")})
        del P
        if rep["converged"] and dist > 1e-3:
            u, s = x, s1
        else:
            ds /= 2
            if ds < 1.0 / 256:
                return None, {"error": "box continuation failed", "path": path}
    return u, {"found_in": "PAPER_BOX, 32x33x32, Re 400, seed 8", "box_path": path}


def large_newton(workload="couette_96x97x96_re2000_dt100", max_newton=20, max_krylov=800,
                 rtol=1e-4, full_newton=8, oracle_modes=24):
    """Newton to ||r|| < 1e-10 on the large workload (96x97x96, Re 2000, 4pi x 2 x
    2pi box) by continuation, as the paper reaches Re 2000 (Sec. 3.3): the
    equilibrium of PAPER_BOX is carried to the 2pi x pi box (half the workload's
    periods), continued in Re to Re 1950 on the workload's y-grid (48x97x48),
    and then
    - timed: hookstep Newton at Re 2000 in that box (FP64, mixed, mixed with an
      FP32 Krylov basis), which is the workload's problem restricted to its
      invariant subspace of fields periodic over half the box (the embedding
      of synth.embed_periodic maps roots to roots exactly);
    - the FP64 root embedded in the workload's grid: its residual there on the
      GPU, and the oracle's residual on sampled modes against the GPU's;
    - hookstep Newton on the full workload grid from the embedded Re-1950 root
      (full_newton steps, FP64), reported as measured."""
    import numpy as np
    import torch
    from paper_1804_05087_amd import SP_FP64, SP_MIXED, Plan, synth
    w = WORKLOADS[workload]
    dev = torch.device("cuda", 0)
    big = (w["nx"], w["ny"], w["nz"])
    sub = (w["nx"] // 2, w["ny"], w["nz"] // 2)
    box_s = (w["lx"] / 2, w["lz"] / 2)
    t0 = time.perf_counter()
    u32, info = box_continued_equilibrium(dev, box_s)
    out = {"metric": "large_grid_newton", "workload": workload, "newton": "hookstep",
           "max_krylov": max_krylov, "gmres_rtol": rtol, "newton_tol": 1e-10,
           "start": info}
    if u32 is None:
        return out
    u = torch.from_numpy(synth.regrid(u32.cpu().numpy(), *sub)).to(dev)
    u, path = re_continuation(dev, u, sub, box_s, 400.0, w["re"] - 50.0, 100.0,
                              max_krylov=max_krylov, rtol=rtol)
    out["start"].update({"re_path": path, "continued_to_re": w["re"] - 50.0,
                         "grid": list(sub), "box": list(box_s),
                         "seconds": round(time.perf_counter() - t0, 1)})
    if u is None:
        return out
    lam_s = torch.from_numpy(synth.laminar_field(*sub)).to(dev)
    P = Plan(*sub, *box_s, w["re"], w["dt"], device=dev)
    roots = {}
    sub_out = {"grid": list(sub), "box": list(box_s)}
    for name, prec, kf32 in (("fp64", SP_FP64, False), ("mixed", SP_MIXED, False),
                             ("mixed_krylov_fp32", SP_MIXED, True)):
        P.set_precision(prec)
        x = u.clone()
        torch.cuda.synchronize()
        rep = P.newton_hookstep(x, max_newton=max_newton, max_krylov=max_krylov,
                                gmres_rtol=rtol, newton_tol=1e-10, krylov_fp32=kf32)
        roots[name] = x
        sub_out[name] = {"converged": rep["converged"], "newton_iters": rep["newton_iters"],
                         "total_krylov": rep["total_krylov"], "actions": rep["total_actions"],
                         "seconds": round(rep["seconds"], 3),
                         "res_history": [float(f"{v:.3e}") for v in rep["res_norm"]],
                         "krylov": rep["krylov"],
                         "dist_to_laminar_L2": float(f"{P.norm((x - lam_s).contiguous()):.4e}")}
        if name != "fp64":
            sub_out[name]["vs_fp64_final_L2"] = float(
                f"{P.norm((x - roots['fp64']).contiguous()):.3e}")
        log("large newton (subspace)", name, sub_out[name])
    out["subspace"] = sub_out
    del P
    # the FP64 root on the workload's grid
    xb_np = synth.embed_periodic(roots["fp64"].cpu().numpy(), 2, 2)
    xb = torch.from_numpy(xb_np).to(dev)
    PB = Plan(*big, w["lx"], w["lz"], w["re"], w["dt"], device=dev)
    rb, rbn = PB.residual(xb, norm=True)
    phib = PB.befe_step(xb)
    emb = {"gpu_res_norm": float(f"{rbn:.3e}")}
    if oracle_modes:
        from oracle.befe import Befe
        from oracle.grid import Grid
        rng = np.random.default_rng(0)
        valid = [(i, j) for i in range(big[0]) for j in range(big[2] // 2)
                 if i != big[0] // 2]
        pick = [valid[k] for k in rng.choice(len(valid), oracle_modes - 1, replace=False)]
        pick = [(0, 0)] + pick
        B = Befe(Grid(big[0], big[1], big[2], w["lx"], w["lz"]), w["re"], w["dt"], modes=pick)
        to = time.perf_counter()
        ro = B.residual(xb_np)
        rg = rb.cpu().numpy()
        sel = np.zeros_like(ro)
        for (i, j) in pick:
            sel[:, i, j, :] = 1.0
        scale = (PB.norm(phib) + PB.norm(xb)) / w["dt"]
        emb.update({"oracle_modes": len(pick),
                    "oracle_res_norm_sampled": float(f"{B.norm_l2(ro * sel):.3e}"),
                    "gpu_res_norm_sampled": float(f"{B.norm_l2(rg * sel):.3e}"),
                    "max_abs_diff_over_scale": float(
                        f"{np.max(np.abs((rg - ro) * sel)) / scale:.3e}"),
                    "oracle_seconds": round(time.perf_counter() - to, 1)})
    out["embedded_root"] = emb
    log("large newton (embedded root)", emb)
    # full-space Newton from the embedded Re-1950 root
    lam_b = torch.from_numpy(synth.laminar_field(*big)).to(dev)
    x = torch.from_numpy(synth.embed_periodic(u.cpu().numpy(), 2, 2)).to(dev)
    rep = PB.newton_hookstep(x, max_newton=full_newton, max_krylov=max_krylov, gmres_rtol=rtol,
                             newton_tol=1e-10)
    out["full_space_fp64"] = {
        "converged": rep["converged"], "newton_iters": rep["newton_iters"],
        "seconds": round(rep["seconds"], 3),
        "res_history": [float(f"{v:.3e}") for v in rep["res_norm"]],
        "gmres_relres": [float(f"{v:.2e}") for v in rep["gmres_relres"]],
        "dist_to_laminar_L2": float(f"{PB.norm((x - lam_b).contiguous()):.4e}")}
    log("large newton (full space)", out["full_space_fp64"])
    return out


PAPER_BOX = (2 * math.pi / 1.14, 2 * math.pi / 2.5)


def continued_equilibrium(dev, w, seeds=(8, 1, 0, 2, 3), re_find=400.0, dre=100.0,
                          last_gap=50.0, max_krylov=400, rtol=1e-4):
    """A non-laminar equilibrium of the workload's box and grid at Re = w["re"]
    - last_gap, the start of the timed Newton solve at w["re"]: found at
    32x33x32, Re 400, from the perturbation family (hookstep Newton, the first
    seed that converges away from laminar flow), spectrally interpolated to the
    workload's grid and continued in Re in steps of dre, each root the start of
    the next solve, as the paper continues its equilibria in Re (Sec. 3.3)."""
    import torch
    from paper_1804_05087_amd import Plan, synth
    dims32 = (32, 33, 32)
    box = (w["lx"], w["lz"])
    lam32 = torch.from_numpy(synth.laminar_field(*dims32)).to(dev)
    P = Plan(*dims32, *box, re_find, w["dt"], device=dev)
    found = None
    for seed in seeds:
        u = torch.from_numpy(synth.perturbation_field(*dims32, *box, seed=seed)).to(dev)
        rep = P.newton_hookstep(u, max_newton=30, max_krylov=max_krylov, gmres_rtol=rtol,
                                newton_tol=1e-12)
        dist = P.norm((u - lam32).contiguous())
        log("equilibrium search seed", seed, rep["converged"], rep["res_norm"][-1], dist)
        if rep["converged"] and dist > 1e-3:
            found = (seed, u, dist)
            break
    if found is None:
        return None, {"error": "no non-laminar equilibrium at 32x33x32, Re 400"}
    dims = (w["nx"], w["ny"], w["nz"])
    x = torch.from_numpy(synth.regrid(found[1].cpu().numpy(), *dims)).to(dev)
    lam = torch.from_numpy(synth.laminar_field(*dims)).to(dev)
    path = []
    re_end = w["re"] - last_gap
    re = re_find
    while True:
        Pr = Plan(*dims, *box, re, w["dt"], device=dev)
        rep = Pr.newton_hookstep(x, max_newton=30, max_krylov=max_krylov, gmres_rtol=rtol,
                                 newton_tol=1e-11)
        path.append({"re": re, "converged": rep["converged"], "newton_iters": rep["newton_iters"],
                     "res": float(f"{rep['res_norm'][-1]:.2e}"),
                     "dist_to_laminar_L2": float(f"{Pr.norm((x - lam).contiguous()):.4e}")})
        log("continuation", path[-1])
        del Pr
        if not rep["converged"]:
            return None, {"error": f"continuation failed at Re {re}", "path": path}
        if re >= re_end:
            break
        re = min(re + dre, re_end)
    return x, {"found_at": {"grid": list(dims32), "re": re_find, "seed": found[0],
                            "dist_to_laminar_L2": float(f"{found[2]:.4e}")},
               "continued_to_re": re_end, "path": path}


def oracle_residual_norms(w, fields):
    """The oracle's ||r|| = ||(Phi(u) - u)/dt|| (volume-normalised L2) of each
    canonical field: the per-step error of a GPU Newton iterate measured by the
    FP64 CPU reference."""
    from oracle.befe import Befe
    from oracle.grid import Grid
    B = Befe(Grid(w["nx"], w["ny"], w["nz"], w["lx"], w["lz"]), w["re"], w["dt"])
    return [float(f"{B.norm_l2(B.residual(f)):.3e}") for f in fields]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-newton", action="store_true")
    ap.add_argument("--no-rates", action="store_true",
                    help="skip the multi-stream, batched, mixed, JVP and VJP rates: the FP64 "
                         "Phi loop and the stage timing only (a kernel trace of this run "
                         "averages the Phi kernels over back-to-back launches on one stream)")
    ap.add_argument("--newton-krylov", type=int, default=600,
                    help="Krylov cap per Newton step (from the continued equilibrium at "
                         "48x65x48, Re 1000: caps of 200-350 stall before 1e-10; 400 is "
                         "fastest with FP64 actions, 600 with the FP32 basis)")
    ap.add_argument("--newton-max", type=int, default=16)
    ap.add_argument("--newton-rtol", type=float, default=1e-4)
    ap.add_argument("--newton-energy", type=float, default=0.0,
                    help="start the Newton leg from the perturbation family at this energy "
                         "instead of the equilibrium continued from Re 400 (the default "
                         "start in the paper's box; E = 1e-2 does not converge)")
    ap.add_argument("--no-oracle-newton", action="store_true",
                    help="skip the oracle's residual norms at the Newton iterates")
    ap.add_argument("--large-newton", action="store_true",
                    help="instead of the benchmark line, reach Re 2000 at 96x97x96 (4pi x 2pi "
                         "box) by continuation and time hookstep Newton to 1e-10 there "
                         "(several minutes)")
    ap.add_argument("--large-krylov", type=int, default=0,
                    help="Krylov cap of --large-newton (default 800)")
    ap.add_argument("--large-steps", type=int, default=0,
                    help="Newton steps of the timed solves of --large-newton (default 20)")
    ap.add_argument("--large-full-steps", type=int, default=-1,
                    help="Newton steps on the full 96x97x96 grid in --large-newton (default 8)")
    ap.add_argument("--large-oracle-modes", type=int, default=-1,
                    help="modes of the oracle residual check in --large-newton (default 24, 0 "
                         "to skip)")
    ap.add_argument("--mixed-error", action="store_true",
                    help="instead of the benchmark line, print the per-Newton-step distance of "
                         "the mixed-precision iterates from the FP64 ones at 48x65x48")
    ap.add_argument("--dt-sweep", action="store_true",
                    help="instead of the benchmark line, print the Krylov-count sweep over "
                         "dt in {1, 10, 100} and seeds 0-9 at 32x33x32, Re 400")
    ap.add_argument("--gint-compare", action="store_true",
                    help="instead of the benchmark line, print the time-step count of "
                         "Newton solves with the Stokes operator (T = 100) against the "
                         "time-integration operator (dt = 0.03125) at 32x33x32, Re 380")
    ap.add_argument("--spectra", action="store_true",
                    help="instead of the benchmark line, print spectra statistics of the "
                         "Stokes and time-integration Jacobians at 12x17x12")
    ap.add_argument("--advect-workload", default="couette_32x33x32_re400_dt100",
                    choices=sorted(WORKLOADS), help="workload of --advect-compare")
    ap.add_argument("--advect-compare", action="store_true",
                    help="instead of the benchmark line, compare Krylov counts of the Stokes "
                         "step and the step with laminar advection in its implicit operator")
    ap.add_argument("--symmetric-compare", action="store_true",
                    help="instead of the benchmark line, run the Stokes / time-integration "
                         "comparison inside the shift-reflect invariant subspace")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the library runs on a single MI355X; sharding across GPUs is not implemented)",
              file=sys.stderr)
        sys.exit(2)
    if args.large_newton:
        kw = {}
        if args.large_krylov:
            kw["max_krylov"] = args.large_krylov
        if args.large_steps:
            kw["max_newton"] = args.large_steps
        if args.large_full_steps >= 0:
            kw["full_newton"] = args.large_full_steps
        if args.large_oracle_modes >= 0:
            kw["oracle_modes"] = args.large_oracle_modes
        print(json.dumps(large_newton(**kw)), flush=True)
        return
    if args.mixed_error:
        print(json.dumps(mixed_error()), flush=True)
        return
    if args.dt_sweep:
        print(json.dumps(dt_sweep()), flush=True)
        return
    if args.gint_compare:
        print(json.dumps(gint_compare()), flush=True)
        return
    if args.spectra:
        print(json.dumps(spectra_report()), flush=True)
        return
    if args.advect_compare:
        print(json.dumps(advect_compare(workload=args.advect_workload)), flush=True)
        return
    if args.symmetric_compare:
        print(json.dumps(symmetric_compare()), flush=True)
        return
    import numpy as np
    import torch
    from paper_1804_05087_amd import (SP_FP64, SP_MIXED, SP_OP_RESIDUAL, SP_STAGE_SOLVE,
                                      SP_STAGE_SYNTH, SP_STAGE_XFWD, SP_STAGE_XINV,
                                      SP_STAGE_ZLINE, Plan, synth)
    STAGE_OF_KERNEL.update({"k_synth_y": SP_STAGE_SYNTH, "k_fft_x_inv": SP_STAGE_XINV,
                            "k_z_product": SP_STAGE_ZLINE, "k_fft_x_fwd": SP_STAGE_XFWD,
                            "k_stokes_solve": SP_STAGE_SOLVE})

    w = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if w.get("input") == "streak_roll":
        u_np = synth.streak_roll_field(w["nx"], w["ny"], w["nz"], w["lx"], w["lz"], seed=0)
    else:
        u_np = synth.perturbation_field(w["nx"], w["ny"], w["nz"], w["lx"], w["lz"], seed=0)
    u = torch.from_numpy(u_np).to(dev)
    du_np = synth.random_admissible(w["nx"], w["ny"], w["nz"], w["lx"], w["lz"], seed=1)
    du = torch.from_numpy(du_np).to(dev)
    t0 = time.perf_counter()
    P = Plan(w["nx"], w["ny"], w["nz"], w["lx"], w["lz"], w["re"], w["dt"], device=dev)
    plan_s = time.perf_counter() - t0
    out = P.empty()
    log("workload", args.workload, "plan", round(plan_s, 3), "s")
    # Copy of known size (256 MiB, larger than the sum of the L2 caches): the
    # reference dispatch for calibrating the FETCH_SIZE / WRITE_SIZE counters
    # when this script runs under rocprofv3 --pmc.
    cal_src = torch.ones(CAL_COPY_BYTES // 8, dtype=torch.float64, device=dev)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    del cal_src, cal_dst

    # ---- FP64 Phi: the headline
    gpu_s, wall_s = time_loop(torch, lambda: P.befe_step(u, out), args.steps, args.warmup)
    ms_per_step = 1000.0 * gpu_s / args.steps
    evals = args.steps / gpu_s
    log("phi fp64", evals, "evals/s", ms_per_step, "ms/eval; wall", wall_s)
    res = {}
    if not args.no_rates:
        steps2 = max(10, args.steps // 2)
        # independent evaluations on 4 plans / 4 streams (default priority): the
        # throughput available to callers with several fields (seeds, sweeps,
        # Jacobian columns); not the headline, which is one field at a time
        streams = [torch.cuda.Stream(device=dev) for _ in range(4)]
        plans4, outs4 = [], []
        for st in streams:
            with torch.cuda.stream(st):
                plans4.append(Plan(w["nx"], w["ny"], w["nz"], w["lx"], w["lz"], w["re"], w["dt"],
                                   device=dev))
                outs4.append(plans4[-1].empty())
        torch.cuda.synchronize()

        def four():
            for k in range(4):
                with torch.cuda.stream(streams[k]):
                    plans4[k].befe_step(u, outs4[k])

        four()
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        for _ in range(steps2):
            four()
        torch.cuda.synchronize()
        res["phi_fp64_4streams_evals_per_s"] = 4 * steps2 / (time.perf_counter() - t4)
        del plans4, outs4
        # the same from one plan: sp_befe_step_batch, 64 fields per call on 3 member
        # streams (with the plan's own stream, the 4 hardware queues of the process)
        ub = u.unsqueeze(0).expand(64, *u.shape).contiguous()
        ob = torch.empty_like(ub)
        P.befe_step_batch(ub, ob, streams=3)
        torch.cuda.synchronize()
        nb = max(1, steps2 // 64)
        tb = time.perf_counter()
        for _ in range(nb):
            P.befe_step_batch(ub, ob, streams=3)
        torch.cuda.synchronize()
        res["phi_fp64_batch64_3streams_evals_per_s"] = 64 * nb / (time.perf_counter() - tb)
        del ub, ob
        P.set_precision(SP_MIXED)
        s, _ = time_loop(torch, lambda: P.befe_step(u, out), steps2, args.warmup)
        res["phi_mixed_evals_per_s"] = steps2 / s
        P.linearize(u)
        s, _ = time_loop(torch, lambda: P.jvp_lin(du, SP_OP_RESIDUAL, out), steps2, args.warmup)
        res["jvp_mixed_evals_per_s"] = steps2 / s
        P.set_precision(SP_FP64)
        P.linearize(u)
        s, _ = time_loop(torch, lambda: P.jvp_lin(du, SP_OP_RESIDUAL, out), steps2, args.warmup)
        res["jvp_fp64_evals_per_s"] = steps2 / s
        # the vector-Jacobian product (the transposed pipeline), FP64 and mixed
        s, _ = time_loop(torch, lambda: P.vjp_lin(du, SP_OP_RESIDUAL, out), steps2, args.warmup)
        res["vjp_fp64_evals_per_s"] = steps2 / s
        P.set_precision(SP_MIXED)
        P.linearize(u)
        s, _ = time_loop(torch, lambda: P.vjp_lin(du, SP_OP_RESIDUAL, out), steps2, args.warmup)
        res["vjp_mixed_evals_per_s"] = steps2 / s
        P.set_precision(SP_FP64)
        P.linearize(u)
        log("rates", res)

    # ---- per-kernel durations of the FP64 Phi step: each stage kernel launched
    # back to back between two HIP events on the plan's stream (sp_time_stage)
    reps = max(50, min(1000, args.steps))
    stage_us = {name: P.time_stage(stage, u, out, reps=reps)
                for name, stage in STAGE_OF_KERNEL.items()}
    # a stage with no launch of its own (the inverse x transforms taken by the
    # z-line kernel) reports 0
    fused = stage_us["k_fft_x_inv"] == 0.0
    ab = algorithmic_bytes(w, fused=fused)
    kernels = {}
    for name, avg_us in stage_us.items():
        if name in ab:
            kernels[name] = {"avg_us": round(avg_us, 3), "alg_bytes": ab[name],
                             "achieved_GBs": round(ab[name] / (avg_us * 1e-6) / 1e9, 1)}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"])
    dom_us = kernels[dom]["avg_us"]
    alg = kernels[dom]["alg_bytes"]
    achieved = round(alg / (dom_us * 1e-6) / 1e9, 1)
    traffic = None
    mt = MEASURED_TRAFFIC.get(args.workload, {}).get(dom)
    if mt and mt["sources_sha256"] == sources_sha256(dom):
        traffic = round(1024 * (mt["fetch_kib"] * mt["fetch_factor"] +
                                mt["write_kib"] * mt["write_factor"]))
    S = spectral_field_bytes(w)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "bytes_per_launch": alg,
                "bytes_rule": "9 S (reads the three product fields and u, writes Phi), "
                              f"S = {S} B",
                "record_bytes_per_launch": record_bytes(w),
                "avg_us": round(dom_us, 3),
                "timing": f"hip events around {reps} back-to-back launches (sp_time_stage)",
                "step": {"bytes": 27 * S, "us": round(ms_per_step * 1000.0, 3),
                         "achieved": round(27 * S / (ms_per_step * 1e-3) / 1e9, 1),
                         "frac": round(27 * S / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    sum_us = sum(k["avg_us"] for k in kernels.values())
    log("kernels", kernels)

    # ---- Newton-GMRES to ||r|| < 1e-10 (FP64 and mixed Jacobian actions)
    newton = {}
    if not args.no_newton:
        lam = torch.from_numpy(synth.laminar_field(w["nx"], w["ny"], w["nz"])).to(dev)
        u0, cinfo = None, None
        if (w["lx"], w["lz"]) == PAPER_BOX and w["re"] > 400.0 and not args.newton_energy:
            tc = time.perf_counter()
            u0, cinfo = continued_equilibrium(dev, w)
            cinfo["seconds"] = round(time.perf_counter() - tc, 2)
        if u0 is None:
            energy = args.newton_energy or 1e-6
            u0 = torch.from_numpy(synth.perturbation_field(
                w["nx"], w["ny"], w["nz"], w["lx"], w["lz"], seed=0, energy=energy)).to(dev)
            newton["start"] = {"kind": "perturbation family", "energy": energy, "seed": 0,
                               "continuation": cinfo}
        else:
            newton["start"] = {"kind": "continued equilibrium", **cinfo,
                               "dist_to_laminar_L2": P.norm((u0 - lam).contiguous())}
        newton["settings"] = {"max_krylov": args.newton_krylov, "gmres_rtol": args.newton_rtol,
                              "newton_tol": 1e-10, "driver": "sp_newton_gmres (full step)"}
        finals, iterates = {}, {}
        for name, prec, kf32 in (("fp64", SP_FP64, False), ("mixed", SP_MIXED, False),
                                 ("mixed_krylov_fp32", SP_MIXED, True),
                                 ("fp64_krylov_fp32", SP_FP64, True)):
            P.set_precision(prec)
            uu = u0.clone()
            torch.cuda.synchronize()
            rep = P.newton_gmres(uu, max_newton=args.newton_max, max_krylov=args.newton_krylov,
                                 gmres_rtol=args.newton_rtol, newton_tol=1e-10,
                                 krylov_fp32=kf32)
            finals[name] = uu
            newton[name] = {
                "converged": rep["converged"], "seconds": round(rep["seconds"], 4),
                "newton_iters": rep["newton_iters"], "total_krylov": rep["total_krylov"],
                "total_actions": rep["total_actions"],
                "final_res_norm": rep["res_norm"][-1],
                "dist_to_laminar_L2": P.norm((uu - lam).contiguous()),
                "res_history": [float(f"{x:.3e}") for x in rep["res_norm"]],
                "krylov": rep["krylov"],
                "gmres_relres": [float(f"{x:.2e}") for x in rep["gmres_relres"]],
            }
            log("newton", name, newton[name])
            # the same solve one Newton step per call (the full-step driver keeps no
            # state between steps), to keep every iterate for the per-step errors
            its, uu = [u0.clone()], u0.clone()
            for _ in range(rep["newton_iters"]):
                r1 = P.newton_gmres(uu, max_newton=1, max_krylov=args.newton_krylov,
                                    gmres_rtol=args.newton_rtol, newton_tol=1e-10,
                                    krylov_fp32=kf32)
                its.append(uu.clone())
                if r1["newton_iters"] == 0:
                    break
            iterates[name] = its
            newton[name]["replay_final_vs_timed_L2"] = P.norm((its[-1] - finals[name]).contiguous())
        P.set_precision(SP_FP64)
        for name in ("mixed", "mixed_krylov_fp32", "fp64_krylov_fp32"):
            ref = iterates["fp64"]
            newton[name]["dist_to_fp64_iterate_L2"] = [
                float(f"{P.norm((a - b).contiguous()):.3e}")
                for a, b in zip(iterates[name][1:], ref[1:])]
        if not args.no_oracle_newton:
            to = time.perf_counter()
            for name, its in iterates.items():
                newton[name]["oracle_res_norm"] = oracle_residual_norms(
                    w, [x.cpu().numpy() for x in its])
                log("oracle ||r|| at the", name, "iterates", newton[name]["oracle_res_norm"])
            newton["oracle_seconds"] = round(time.perf_counter() - to, 1)
        newton["mixed_vs_fp64_final_L2"] = P.norm((finals["mixed"] - finals["fp64"]).contiguous())
        newton["mixed_krylov_fp32_vs_fp64_final_L2"] = P.norm(
            (finals["mixed_krylov_fp32"] - finals["fp64"]).contiguous())
        newton["fp64_krylov_fp32_vs_fp64_final_L2"] = P.norm(
            (finals["fp64_krylov_fp32"] - finals["fp64"]).contiguous())
        # the same solve with the laminar advection in the implicit operator
        # (Sec. 3.6's proposed remedy; same roots, fewer Krylov iterations)
        PA = Plan(w["nx"], w["ny"], w["nz"], w["lx"], w["lz"], w["re"], w["dt"], device=dev)
        tb = time.perf_counter()
        PA.set_advection(True)
        build_s = time.perf_counter() - tb
        oa = PA.empty()
        sa, _ = time_loop(torch, lambda: PA.befe_step(u, oa), 200, 20)
        res["phi_fp64_advected_evals_per_s"] = 200 / sa
        PA.set_precision(SP_MIXED)
        sa, _ = time_loop(torch, lambda: PA.befe_step(u, oa), 200, 20)
        res["phi_mixed_advected_evals_per_s"] = 200 / sa
        PA.set_precision(SP_FP64)
        uu = u0.clone()
        torch.cuda.synchronize()
        rep = PA.newton_gmres(uu, max_newton=args.newton_max, max_krylov=args.newton_krylov,
                              gmres_rtol=args.newton_rtol, newton_tol=1e-10)
        newton["fp64_advected"] = {
            "converged": rep["converged"], "seconds": round(rep["seconds"], 4),
            "plan_build_seconds": round(build_s, 3),
            "newton_iters": rep["newton_iters"], "total_krylov": rep["total_krylov"],
            "total_actions": rep["total_actions"], "final_res_norm": rep["res_norm"][-1],
            "res_history": [float(f"{x:.3e}") for x in rep["res_norm"]],
            "krylov": rep["krylov"],
            "gmres_relres": [float(f"{x:.2e}") for x in rep["gmres_relres"]],
            "vs_fp64_final_L2": P.norm((uu - finals["fp64"]).contiguous())}
        log("newton fp64_advected", newton["fp64_advected"])
        del PA

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, u_np)
        log("cpu baseline", cpu)

    line = {
        "metric": "phi_dt_evals_per_s_fp64",
        "value": round(evals, 2),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded divergence-free perturbation of laminar Couette flow)",
        "config": {"workload": args.workload, "grid": [w["nx"], w["ny"], w["nz"]],
                   "re": w["re"], "dt": w["dt"], "box": [w["lx"], 2.0, w["lz"]],
                   "parallelism": "single-gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "rates": {k: round(v, 2) for k, v in res.items()},
        "kernel_us_per_eval": round(sum_us, 3),  # sum of the stage kernels' averages
        "kernels": kernels,
        "newton": newton,
        "plan_seconds": round(plan_s, 4),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
