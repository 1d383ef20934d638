"""Benchmark: time-to-1e-8 of the pMG-preconditioned SE Poisson solve on one MI355X.

Workload (default): the anisotropic "layer-shift" box, 32^3 = 32768 hexahedra,
p = 7 (11,390,625 unique nodes, 16,777,216 local points), homogeneous
Dirichlet, f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z); preconditioner Cheby-RAS(2)
p-multigrid (7,3,1) with the smoother in FP32 and FDM local solves, coarse
p = 1 level solved exactly by block-tridiagonal elimination over z-planes
(--coarse pcg: Jacobi-PCG to 1e-10 instead), outer FP64 flexible CG to
relative residual 1e-8.

One step = one full solve from x = 0 (inputs resident in HBM, setup excluded).
value = unique DOF solved per second (GDOF/s) over the timed steps.  Kernel
durations come from HIP events the library records around every finest-level
launch during the timed steps (sem_profile), on the stream the kernels run on.

After the timed steps the default run also measures, once each: the plain
FP64 solve and the FP16/BF16 matrix-core FDM solves; the FP64 oracle's
residual of every solution; the 16^3 sine-map FP64 Cheby-Jacobi solve; the
64-problem batched workload; and the oracle timed on the host (a bounded
sample).  Prints one JSON line.
"""
import argparse
import json
import os
import subprocess
import sys
import time
from types import SimpleNamespace

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32, help="elements per direction")
    ap.add_argument("--p", type=int, default=7)
    ap.add_argument("--coarse-tol", type=float, default=1e-10,
                    help="relative tolerance of the coarse Jacobi-PCG")
    ap.add_argument("--coarse", choices=("auto", "pcg", "direct"), default="auto",
                    help="coarse p=1 solve: Jacobi-PCG, exact block-tridiagonal elimination, "
                         "or the library default (direct when its storage fits 4 GiB)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain-FP64 comparison solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=1, help="oracle FCG iterations timed")
    ap.add_argument("--no-oracle", action="store_true", help="skip the oracle residual checks")
    ap.add_argument("--no-config2", action="store_true", help="skip the 16^3 sine-map leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-workload leg")
    ap.add_argument("--mode", choices=("solve", "kernels", "batch", "sensitivity", "projection",
                                       "config2", "cpu"),
                    default="solve",
                    help="kernels: repeat single finest-level kernels (for counter runs); "
                         "batch: the 64-problem x 4-RHS batched workload; sensitivity: "
                         "iteration counts over the Chebyshev bound multipliers; projection: "
                         "successive right sides with and without prior-solution projection; "
                         "config2: the 16^3 sine-map FP64 Cheby-Jacobi solve; cpu: the oracle "
                         "timed on the host (full protocol)")
    ap.add_argument("--nprob", type=int, default=64, help="problems in --mode batch")
    ap.add_argument("--no-tune", action="store_true", help="--mode batch: skip the auto-tuner")
    ap.add_argument("--reps", type=int, default=5, help="repetitions per kernel in --mode kernels")
    return ap.parse_args()


def kernels_mode(a):
    """Repeats each finest-level kernel class `reps` times on the benchmark mesh,
    plus a plain 1 GiB device copy (torch) that calibrates the HBM counters."""
    import torch
    from paper_2110_07663_amd import sem
    from paper_2110_07663_amd import workloads as wl
    torch.cuda.set_device(0)
    n, p = a.n, a.p
    sched = (p, 3, 1) if p > 3 else (p, 1)
    opts = sem.make_opts(schedule=sched, smoother=sem.SMOOTH_RAS, smoother_prec=sem.F32,
                         lambda_override=[2.0, 2.0])
    s = sem.Solver(n, n, n, wl.layer_shift_vertices(n, seed=3), 1, p, opts=opts)
    L = s.levels[0]
    u = s.gather(torch.as_tensor(wl.random_global(L.nglobal, 0)).cuda())
    u32 = u.float()
    v, v32 = torch.empty_like(u), torch.empty_like(u32)
    for _ in range(a.reps):
        s.apply_A(u, out=v)
        s.apply_A(u32, out=v32)
        s.apply_S(u32, out=v32)
    # Cheby-RAS(2) smoothing: the FDM and Ax forms the solve runs (A's output
    # leaving its x and y gather-scatter steps to the FDM, the residual form)
    x32 = torch.zeros_like(u32)
    for _ in range(a.reps):
        s.smooth(u32, x32, level=0)
    # the other Ax kernel shapes at p = 7 (the default is variant 2)
    for av in (0, 1):
        oa = sem.make_opts(schedule=sched, smoother=sem.SMOOTH_RAS, smoother_prec=sem.F32,
                           lambda_override=[2.0, 2.0], ax_variant=av)
        sa = sem.Solver(n, n, n, wl.layer_shift_vertices(n, seed=3), 1, p, opts=oa)
        for _ in range(a.reps):
            sa.apply_A(u, out=v)
            sa.apply_A(u32, out=v32)
        sa.close()
    # the matrix-core FDM in both 16-bit formats
    for fp in (sem.F16, sem.BF16):
        o16 = sem.make_opts(schedule=sched, smoother=sem.SMOOTH_RAS, smoother_prec=sem.F32,
                            fdm_prec=fp, lambda_override=[2.0, 2.0])
        s16 = sem.Solver(n, n, n, wl.layer_shift_vertices(n, seed=3), 1, p, opts=o16)
        for _ in range(a.reps):
            s16.apply_S(u32, out=v32)
        s16.close()
    # the FP32 Ax reading FP16 geometric factors (p = 7)
    og = sem.make_opts(schedule=sched, smoother=sem.SMOOTH_RAS, smoother_prec=sem.F32,
                       lambda_override=[2.0, 2.0], geom_prec=sem.F16)
    sg = sem.Solver(n, n, n, wl.layer_shift_vertices(n, seed=3), 1, p, opts=og)
    for _ in range(a.reps):
        sg.apply_A(u32, out=v32)
    sg.close()
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "kernels", "reps": a.reps, "copy_bytes": 2 * src.numel() * 8}))


def batch_mode(a):
    print(json.dumps({"mode": "batch", **batch_run(a, oracle_lanes=not a.no_oracle)}), flush=True)


def batch_run(a, oracle_lanes=True):
    """Batched workload: `nprob` independent Poisson solves on the smooth
    sinusoidal map, E = side^3 with side in {8, 12, 16, 24} and p in {5, 7, 9}
    drawn by seed 5, each with 4 sinusoidal right sides of random frequencies
    1..4; mixed precision Cheby-RAS pMG, tol 1e-8.  The auto-tuner picks the
    Chebyshev order, the Ax kernel shape and the storage of the geometric
    factors (FP32 or FP16) per (p, side) bucket on its first problem.  Reports the time of the batched solve (one recorded graph per
    outer iteration of all 4*nprob lanes) against solving every lane in turn,
    and the FP64 oracle's residual of the lanes of the four smallest problems."""
    import torch
    from paper_2110_07663_amd import sem
    from paper_2110_07663_amd import workloads as wl
    torch.cuda.set_device(0)
    spec = wl.batch_spec(nprob=a.nprob, seed=5)

    def note(msg):
        print(f"[batch] {msg}", file=sys.stderr, flush=True)
    sched_of = {5: (5, 3, 1), 7: (7, 3, 1), 9: (9, 5, 1)}
    tuned = {}
    solvers, bs, t_tune = [], [], 0.0
    total_dof = 0
    for side, p, freqs in spec:
        xyz = wl.sampled_mesh(side, side, side, sem.gll_nodes(p)[0], wl.sin_map(0.05))
        base = sem.make_opts(schedule=sched_of[p], smoother=sem.SMOOTH_RAS, cheb_order=2,
                             smoother_prec=sem.F32, batch_rhs=4)
        key = (p, side)
        if key not in tuned and not a.no_tune:
            probe = sem.Solver(side, side, side, xyz, p, p, opts=base)
            X = probe.coords(0).cpu().numpy()
            f, _ = wl.sinusoid(*freqs[0])
            b0 = probe.rhs(torch.as_tensor(f(X[0], X[1], X[2])).cuda())
            req = sem.TuneRequest()
            req.ncand = 0
            for order in (1, 2, 3):
                for av in ((0, 1) if p == 7 else (-1,)):
                    for gp in (sem.F32, sem.F16):
                        o = sem.make_opts(schedule=sched_of[p], smoother=sem.SMOOTH_RAS,
                                          cheb_order=order, smoother_prec=sem.F32, batch_rhs=4,
                                          ax_variant=av, geom_prec=gp)
                        req.cand[req.ncand] = o
                        req.ncand += 1
            t0 = time.perf_counter()
            best, res, _ = sem.tune(side, side, side, xyz, p, p, b0, request=req, repeats=1)
            t_tune += time.perf_counter() - t0
            note(f"tuned p={p} side={side}: order {best.cheb_order} ax {best.ax_variant} "
                 f"geom {'f16' if best.geom_prec == sem.F16 else 'f32'} "
                 f"({time.perf_counter() - t0:.1f} s)")
            probe.close()
            best.batch_rhs = 4
            tuned[key] = best
        opts = tuned.get(key, base)
        s = sem.Solver(side, side, side, xyz, p, p, opts=opts)
        X = s.coords(0).cpu().numpy()
        row = []
        for fr in freqs:
            f, _ = wl.sinusoid(*fr)
            row.append(s.rhs(torch.as_tensor(f(X[0], X[1], X[2])).cuda()))
        solvers.append(s)
        bs.append(row)
        total_dof += s.levels[0].nglobal * len(freqs)
        note(f"set up problem {len(solvers)}/{len(spec)} (side {side}, p {p})")
    torch.cuda.synchronize()
    # sequential: every lane through sem_solve
    xs_seq = [[torch.zeros_like(b) for b in row] for row in bs]
    for s_, row, xrow in zip(solvers, bs, xs_seq):   # warm-up of every context
        s_.solve(row[0], x=torch.zeros_like(row[0]), rtol=1e-8, maxit=300)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters_seq = []
    for i, (s_, row, xrow) in enumerate(zip(solvers, bs, xs_seq)):
        for b, x in zip(row, xrow):
            _, info = s_.solve(b, x=x, rtol=1e-8, maxit=300)
            iters_seq.append(info.iters)
        if i % 8 == 7:
            note(f"sequential: {i + 1} problems solved")
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    note(f"sequential {t_seq:.2f} s; batched solve starts")
    # batched: the 4 right sides of a problem share each operator application and
    # V-cycle (one launch per kernel for all 4); first an untimed warm-up call
    def batched(joint):
        os.environ["SEM_BATCH_JOINT"] = "1" if joint else "0"
        try:
            xs = [[torch.zeros_like(b) for b in row] for row in bs]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = sem.batch_solve(solvers, bs, xs, rtol=1e-8, maxit=300, iters_per_launch=2)
            torch.cuda.synchronize()
            return time.perf_counter() - t0, infos, xs
        finally:
            del os.environ["SEM_BATCH_JOINT"]

    batched(True)
    t_bat, infos, xs_last = batched(True)
    note(f"batched {t_bat:.2f} s")
    t_turn, infos_turn, _ = batched(False)
    note(f"batched, lanes of a problem in turn {t_turn:.2f} s")
    # plain FP64 sequential baseline: one context at a time (set up, 4 solves timed, freed)
    t_seq64, iters64 = 0.0, []
    for i, ((side, p, freqs), row) in enumerate(zip(spec, bs)):
        xyz = wl.sampled_mesh(side, side, side, sem.gll_nodes(p)[0], wl.sin_map(0.05))
        o64 = sem.make_opts(schedule=sched_of[p], smoother=sem.SMOOTH_RAS, cheb_order=2,
                            smoother_prec=sem.F64)
        s64 = sem.Solver(side, side, side, xyz, p, p, opts=o64)
        s64.solve(row[0], x=torch.zeros_like(row[0]), rtol=1e-8, maxit=300)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in row:
            _, info = s64.solve(b, x=torch.zeros_like(b), rtol=1e-8, maxit=300)
            iters64.append(info.iters)
        torch.cuda.synchronize()
        t_seq64 += time.perf_counter() - t0
        s64.close()
        del s64
        if i % 8 == 7:
            note(f"fp64 sequential: {i + 1} problems")
    worst = max(i.true_rel_res for i in infos)
    out = {"problems": len(solvers), "rhs_per_problem": 4,
           "lanes": len(infos), "unique_dof_total": int(total_dof),
           "sequential_s": round(t_seq, 3), "batched_s": round(t_bat, 3),
           "speedup_batched_vs_sequential": round(t_seq / t_bat, 3),
           "batched_lanes_in_turn_s": round(t_turn, 3),
           "speedup_shared_vs_lanes_in_turn": round(t_turn / t_bat, 3),
           "iters_in_turn_equal": [i.iters for i in infos_turn] == [i.iters for i in infos],
           "sequential_fp64_s": round(t_seq64, 3),
           "speedup_batched_vs_sequential_fp64": round(t_seq64 / t_bat, 3),
           "iters_sequential_fp64_max": max(iters64),
           "batched_gdof_s": round(total_dof / t_bat / 1e9, 4),
           "worst_true_rel_res": worst, "all_converged": all(i.converged for i in infos),
           "iters_batched_max": max(i.iters for i in infos),
           "iters_sequential_max": max(iters_seq), "tune_s": round(t_tune, 2),
           "tuned": {f"p{k[0]}_side{k[1]}": {"cheb_order": v.cheb_order, "ax_variant": v.ax_variant,
                                              "geom": "f16" if v.geom_prec == sem.F16 else "f32"}
                     for k, v in tuned.items()}}
    if oracle_lanes:
        # the FP64 oracle's residual of every lane of the four smallest problems
        order = sorted(range(len(spec)), key=lambda i: (spec[i][0], spec[i][1], i))[:4]
        worst_o = 0.0
        for i in order:
            side, p, freqs = spec[i]
            L, X = oracle_level_sin(side, p)
            for k, fr in enumerate(freqs):
                f, _ = wl.sinusoid(*fr)
                bo = oracle_rhs(L, f, X)
                worst_o = max(worst_o, oracle_rel_res(L, bo, xs_last[i][k].cpu().numpy()))
        out["oracle_lanes_checked"] = 16
        out["oracle_worst_rel_res"] = worst_o
        note(f"oracle residual of 16 lanes: worst {worst_o:.2e}")
    for s_ in solvers:
        s_.close()
    return out


def sensitivity_mode(a):
    """The (lambda_min, lambda_max) multiplier grid of the paper's bound study
    (Sec. 2.2, Table 1): 24^3 elements, p = 7, Cheby-ASM(2) in the (7, 3, 1)
    V-cycle, tol 1e-8, at most 1000 iterations, on the layer-shift mesh (seed 3)
    standing in for Kershaw eps = 0.3.  The Arnoldi estimate of every level is
    taken once and reused, so only the multipliers change between entries."""
    import torch
    from paper_2110_07663_amd import sem
    from paper_2110_07663_amd import workloads as wl
    torch.cuda.set_device(0)
    n, p = 24, 7
    sched = (7, 3, 1)
    xyz = wl.layer_shift_vertices(n, seed=3)
    f, _ = wl.sinusoid(1, 1, 1)

    def opts(lmin, lmax, lam=None):
        return sem.make_opts(schedule=sched, smoother=sem.SMOOTH_ASM, cheb_order=2,
                             smoother_prec=sem.F32, lmin_fac=lmin, lmax_fac=lmax,
                             lambda_override=lam)

    s0 = sem.Solver(n, n, n, xyz, 1, p, opts=opts(0.1, 1.1))
    X = s0.coords(0)
    b = s0.rhs(torch.as_tensor(f(*(X.cpu().numpy())), dtype=torch.float64).cuda())
    _, info = s0.solve(b, rtol=1e-8, maxit=1000, allow_noconv=True)
    lam = [info.lambda_tilde[l] for l in range(len(sched) - 1)]
    s0.close()
    lmins = (0.0, 0.025, 0.05, 0.1, 0.2, 0.25)
    lmaxs = (0.9, 0.95, 1.0, 1.1, 1.2, 1.3)
    grid = {}
    for lmin in lmins:
        row = {}
        for lmax in lmaxs:
            s = sem.Solver(n, n, n, xyz, 1, p, opts=opts(lmin, lmax, lam))
            _, inf = s.solve(b, rtol=1e-8, maxit=1000, allow_noconv=True)
            row[str(lmax)] = inf.iters if inf.converged else None
            s.close()
            print(f"[sensitivity] lmin {lmin} lmax {lmax}: "
                  f"{inf.iters if inf.converged else '-'}", file=sys.stderr, flush=True)
        grid[str(lmin)] = row
    print(json.dumps({"mode": "sensitivity", "mesh": "layer-shift 24^3 seed 3", "p": p,
                      "smoother": "Cheby-ASM(2) FP32", "schedule": list(sched), "tol": 1e-8,
                      "maxit": 1000, "lambda_tilde": lam,
                      "iters (row lambda_min factor, column lambda_max factor; null = no "
                      "convergence)": grid}), flush=True)


def projection_mode(a):
    """Successive right sides (Sec. 3.2 / 4.2: a pressure solve per time step,
    started from the A-conjugate projection onto up to 10 prior solutions) on
    the benchmark workload: T = 12 right sides f_t = (1 + 0.1 sin 0.5t) s(1,1,1)
    + 0.05 cos(0.3t) s(2,1,3) + 0.02 sin(pi (x + 0.05 t)) sin(pi y) sin(2 pi z),
    s(a,b,c) = sin(a pi x) sin(b pi y) sin(c pi z), each solved to 1e-8 relative
    to ||b||, with the projection (proj_max = 10) and from x = 0."""
    import numpy as np
    import torch
    from paper_2110_07663_amd import sem
    from paper_2110_07663_amd import workloads as wl
    torch.cuda.set_device(0)
    n, p = a.n, a.p
    sched = (p, 3, 1) if p > 3 else (p, 1)
    xyz = wl.layer_shift_vertices(n, seed=3)
    T = 12

    def make(proj):
        return sem.Solver(n, n, n, xyz, 1, p, opts=sem.make_opts(
            schedule=sched, smoother=sem.SMOOTH_RAS, cheb_order=2, smoother_prec=sem.F32,
            krylov=sem.KRYLOV_FCG, proj_max=proj))

    s_proj, s_zero = make(10), make(0)
    X = s_proj.coords(0).cpu().numpy()
    s111 = wl.sinusoid(1, 1, 1)[0](X[0], X[1], X[2])
    s213 = wl.sinusoid(2, 1, 3)[0](X[0], X[1], X[2])
    rhs = []
    for t in range(T):
        drift = np.sin(np.pi * (X[0] + 0.05 * t)) * np.sin(np.pi * X[1]) * np.sin(2 * np.pi * X[2])
        f = (1 + 0.1 * np.sin(0.5 * t)) * s111 + 0.05 * np.cos(0.3 * t) * s213 + 0.02 * drift
        rhs.append(s_proj.rhs(torch.as_tensor(f, dtype=torch.float64).cuda()))
    out = {}
    for name, s in (("projection", s_proj), ("zero_start", s_zero)):
        s.solve(rhs[0], rtol=1e-8, maxit=300)   # warm-up (also fills the basis once)
        if name == "projection":
            s.projection_reset()
        its, ms, r0s = [], [], []
        for b in rhs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = s.solve(b, rtol=1e-8, maxit=300)
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
            its.append(info.iters)
            r0s.append(info.r0_norm)
            if not info.converged:
                raise RuntimeError(f"{name}: a solve did not converge")
        out[name] = {"iters": its, "ms": [round(v, 2) for v in ms], "total_ms": round(sum(ms), 1),
                     "initial_residual": [float(f"{v:.3e}") for v in r0s]}
        print(f"[projection] {name}: iters {its} total {sum(ms):.1f} ms", file=sys.stderr, flush=True)
    s_proj.close()
    s_zero.close()
    # from x = 0 the initial residual is ||b||: the ratio is the projection's reduction
    out["projection"]["initial_residual_rel"] = [
        float(f"{rp / rz:.3e}") for rp, rz in zip(out["projection"]["initial_residual"],
                                                  out["zero_start"]["initial_residual"])]
    print(json.dumps({"mode": "projection", "workload": "layer-shift box 32^3 hex, p=7, "
                      "12 successive right sides, tol 1e-8 of ||b||", "proj_max": 10, **out,
                      "speedup": round(out["zero_start"]["total_ms"] / out["projection"]["total_ms"], 3)}),
          flush=True)


def algorithmic_bytes(kind, L):
    """HBM bytes one launch must move (each operand read or written once)."""
    p, E = L.p, L.E
    N3 = (p + 1) ** 3
    pb = p + 3
    if kind == "ax64":   # u, v and 6 geometric factors, FP64
        return E * N3 * 8 * 8
    if kind == "ax32":   # FP32 u, v, G
        return E * N3 * 8 * 4
    if kind == "fdm":    # FP32: input and output E-vectors (and the stored RAS weight at
        # p <= 3; from p = 4 the kernel computes it); S (3 pb^2); lambda (3 pb)
        return E * ((2 if p >= 4 else 3) * N3 * 4 + 3 * pb * pb * 4 + 3 * pb * 4)
    if kind in ("gs32", "gs64"):
        w = 4 if kind == "gs32" else 8
        if os.environ.get("SEM_GS_SORTED") == "1":  # + index per member, offset per segment
            return L.nmembers * (2 * w + 4) + (L.nshared + 1) * 4
        return L.nmembers * 2 * w  # value read + write per member of a shared or Dirichlet node
    raise ValueError(kind)


def fdm_flops(L):
    """Multiply-adds x 2 of the six 1D contractions plus the diagonal scaling, per launch."""
    pb = L.p + 3
    return L.E * (12 * pb ** 4 + pb ** 3)


# HBM bytes per launch measured on this workload (2 x FETCH_SIZE + WRITE_SIZE,
# KiB x 1024, calibrated on a 1 GiB device copy; commands and raw counter
# values in profiles/kernels_layer_shift_32cube_p7.md).  A kernel whose code
# changed after its counters were taken is left out (traffic null).
TRAFFIC_32CUBE_P7 = {
    "ax64": 1072564224,   # k_ax8_f64<true,false> as the solve runs it (x-faces left to the FCG update)
    "ax32": 536990080,    # k_ax8_f32<true,false> (the smoother's A, 5 of 6 launches per V-cycle)
    # matrix-core RAS local solves per finest-level launch as a V-cycle mixes
    # them: 4 x k_fdm_mf32<7,1,false,1,true,false> (192,954,816 B), 1 x the
    # residual form <7,1,true,2,true,true> (279,285,589 B), 1 x the zero-start
    # form <7,1,false,0,false,true> (194,233,173 B)
    "fdm": 207556338,
}
# dense FP32 on the matrix cores (the FDM contractions run there)
FP32_MATRIX_PEAK_TFLOPS = 157.3


# --- the oracle as test infrastructure: residual checks and the CPU baseline ---

def oracle_level_shift(n, p):
    """The oracle's finest level on the layer-shift mesh (FP64 operator only)."""
    from oracle.hierarchy import Level
    from paper_2110_07663_amd import workloads as wl
    L = Level(n, n, n, wl.layer_shift_vertices(n, seed=3), 1, p, (1,) * 6, "jacobi")
    return L, L.X


def oracle_level_sin(n, p):
    """The oracle's level on the sine map sampled at the oracle's own GLL nodes."""
    from oracle import gll as ogll
    from oracle.hierarchy import Level
    from paper_2110_07663_amd import workloads as wl
    xyz = wl.sampled_mesh(n, n, n, ogll.gll_nodes_weights(p)[0], wl.sin_map(0.05))
    L = Level(n, n, n, xyz, p, p, (1,) * 6, "jacobi")
    return L, L.X


def oracle_rhs(L, f, X):
    from oracle.operator import rhs
    return rhs(L.num, L.BL, f(X[0], X[1], X[2]))


def oracle_rel_res(L, bo, x):
    """||b - A x|| / ||b|| with the oracle's FP64 operator (unique free nodes)."""
    x = np.asarray(x, dtype=np.float64).reshape(bo.shape)
    r = bo - L.apply_A(x)
    return float(np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)))


def host_info():
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    share = os.environ.get("OMP_NUM_THREADS")
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "threads_all": int(share) if share and share.isdigit() else os.cpu_count()}


def config2_run(a):
    """The 16^3 sine-map workload (x' = x + 0.05 s, likewise y, z) at p = 7:
    plain FP64 PCG preconditioned by the (7, 3, 1) V-cycle with Chebyshev-
    Jacobi(2) smoothing and a Jacobi-PCG coarse solve to 1e-10, tol 1e-8.
    Median of 5 solves from x = 0, and the oracle's residual of the solution."""
    import torch
    from paper_2110_07663_amd import sem
    from paper_2110_07663_amd import workloads as wl
    n, p = 16, 7
    xyz = wl.sampled_mesh(n, n, n, sem.gll_nodes(p)[0], wl.sin_map(0.05))
    opts = sem.make_opts(schedule=(7, 3, 1), smoother=sem.SMOOTH_JACOBI, cheb_order=2,
                         smoother_prec=sem.F64, krylov=sem.KRYLOV_PCG, coarse_tol=1e-10,
                         coarse_solver=sem.COARSE_PCG)
    t0 = time.perf_counter()
    s = sem.Solver(n, n, n, xyz, p, p, opts=opts)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    f, _ = wl.sinusoid(1, 1, 1)
    X = s.coords(0).cpu().numpy()
    b = s.rhs(torch.as_tensor(f(X[0], X[1], X[2])).cuda())
    s.solve(b, rtol=1e-8, maxit=300)
    ms, infos = [], []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = s.solve(b, rtol=1e-8, maxit=300)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - t0))
        infos.append(info)
    L0 = s.levels[0]
    out = {"workload": "sine map 16^3 hex, p=7 (x'=x+0.05 sin 2pi x sin 2pi y sin 2pi z), Dirichlet, "
                       "sin RHS; FP64 PCG + pMG(7,3,1) Cheby-Jacobi(2), coarse Jacobi-PCG 1e-10, tol 1e-8",
           "n_unique": int(L0.nglobal), "setup_s": round(t_setup, 3),
           "ms_median": round(float(np.median(ms)), 3), "iters": infos[-1].iters,
           "coarse_iters_last_vcycle": infos[-1].coarse_iters,
           "true_rel_res": infos[-1].true_rel_res,
           "gdof_s": round(L0.nglobal / (np.median(ms) * 1e-3) / 1e9, 4)}
    if not a.no_oracle:
        Lo, Xo = oracle_level_sin(n, p)
        out["oracle_rel_res"] = oracle_rel_res(Lo, oracle_rhs(Lo, f, Xo), x.cpu().numpy())
    s.close()
    return out


def config2_mode(a):
    import torch
    torch.cuda.set_device(0)
    print(json.dumps({"mode": "config2", **config2_run(a)}), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the library has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    if a.mode == "cpu":
        cpu_mode(a)
        return
    if a.mode == "kernels":
        kernels_mode(a)
        return
    if a.mode == "batch":
        import torch
        torch.cuda.set_device(0)
        batch_mode(a)
        return
    if a.mode == "sensitivity":
        sensitivity_mode(a)
        return
    if a.mode == "projection":
        projection_mode(a)
        return
    if a.mode == "config2":
        config2_mode(a)
        return
    import torch

    from paper_2110_07663_amd import sem
    from paper_2110_07663_amd import workloads as wl

    torch.cuda.set_device(0)
    n, p = a.n, a.p
    sched = (p, 3, 1) if p > 3 else (p, 1)
    xyz = wl.layer_shift_vertices(n, seed=3)
    f, _ = wl.sinusoid(1, 1, 1)

    coarse = {"auto": sem.COARSE_AUTO, "pcg": sem.COARSE_PCG, "direct": sem.COARSE_DIRECT}[a.coarse]

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def make(prec, fdm_prec=None, geom_prec=sem.F32):
        opts = sem.make_opts(schedule=sched, smoother=sem.SMOOTH_RAS, cheb_order=2,
                             smoother_prec=prec, krylov=sem.KRYLOV_FCG, coarse_tol=a.coarse_tol,
                             coarse_solver=coarse, fdm_prec=fdm_prec if fdm_prec else prec,
                             geom_prec=geom_prec)
        t0 = time.perf_counter()
        s = sem.Solver(n, n, n, xyz, 1, p, opts=opts)
        torch.cuda.synchronize()
        return s, time.perf_counter() - t0

    mixed, t_setup = make(sem.F32)
    X = mixed.coords(0)
    fl = torch.as_tensor(f(*(X.cpu().numpy())), dtype=torch.float64).cuda()
    b = mixed.rhs(fl)
    del X, fl
    L0 = mixed.levels[0]
    note(f"setup {t_setup:.2f}s  E={L0.E} p={p} n_unique={L0.nglobal} local={L0.nlocal}")

    for _ in range(a.warmup):
        mixed.solve(b, rtol=1e-8, maxit=200)
    torch.cuda.synchronize()
    # the timed steps record HIP events around the roofline's kernel classes
    # only (Ax and FDM: 12 launches per iteration); the other classes are timed
    # in extra steps afterwards, outside the timed region
    timed_kinds = ("ax64", "ax32", "fdm")
    mixed.profile(True, kinds=timed_kinds)
    infos = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        x, info = mixed.solve(b, rtol=1e-8, maxit=200)
        infos.append(info)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    prof = mixed.profile_read()
    mixed.profile(True, kinds=tuple(k for k in sem.PROF_NAMES if k not in timed_kinds))
    for _ in range(max(1, min(a.steps, 3))):
        mixed.solve(b, rtol=1e-8, maxit=200)
    prof.update({k: v for k, v in mixed.profile_read().items() if k not in timed_kinds})
    mixed.profile(False)
    ms_step = 1e3 * t_total / a.steps
    value = L0.nglobal / (t_total / a.steps) / 1e9
    iters = [i.iters for i in infos]
    coarse_used = "direct" if infos[-1].coarse_iters == 0 else "pcg"
    lam_tilde = [infos[-1].lambda_tilde[l] for l in range(len(sched) - 1)]
    note(f"mixed solve {ms_step:.2f} ms/step iters={iters} true_rel_res={infos[-1].true_rel_res:.2e}")
    sols = {"mixed": (x.cpu().numpy(), infos[-1], ms_step)}
    mixed.close()
    del mixed, x

    # per-kernel rooflines from the event timings of the timed steps
    kern = {}
    for k in ("ax64", "ax32", "fdm", "gs32", "gs64"):
        ms, cnt = prof[k]
        if cnt == 0:
            continue
        avg = ms / cnt
        byt = algorithmic_bytes(k, L0)
        kern[k] = {"avg_us": 1e3 * avg, "launches": cnt, "total_ms": ms,
                   "bytes_per_launch": byt, "GBs": byt / (avg * 1e-3) / 1e9}
        if k == "fdm":
            kern[k]["TFLOPs"] = fdm_flops(L0) / (avg * 1e-3) / 1e12
    for k in ("coarse", "vcycle"):
        ms, cnt = prof[k]
        if cnt:
            kern[k] = {"avg_us": 1e3 * ms / cnt, "launches": cnt, "total_ms": ms}
    # dominant finest-level kernel of the timed solves (by total time)
    dom = max((k for k in kern if "bytes_per_launch" in kern[k]), key=lambda k: kern[k]["total_ms"])
    d = kern[dom]
    traffic = TRAFFIC_32CUBE_P7.get(dom) if (n, p) == (32, 7) else None
    if dom == "fdm":   # FP32 contractions on the matrix cores
        roofline = {"bound": "mfma", "kernel": dom, "achieved": round(d["TFLOPs"], 2),
                    "peak": FP32_MATRIX_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(d["TFLOPs"] / FP32_MATRIX_PEAK_TFLOPS, 4),
                    "traffic": traffic, "hbm_GBs": round(d["GBs"], 1)}
    else:
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(d["GBs"], 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(d["GBs"] / HBM_PEAK_GBS, 4),
                    "traffic": traffic}
    ax = kern.get("ax64")
    ax_gdofs = L0.nglobal / (ax["avg_us"] * 1e-6) / 1e9 if ax else None
    fdm_k = kern.get("fdm")
    fdm_roof = None
    if fdm_k:
        fdm_roof = {"bound": "mfma", "achieved": round(fdm_k["TFLOPs"], 2),
                    "peak": FP32_MATRIX_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(fdm_k["TFLOPs"] / FP32_MATRIX_PEAK_TFLOPS, 4),
                    "traffic": TRAFFIC_32CUBE_P7.get("fdm") if (n, p) == (32, 7) else None}

    # plain FP64 solve, the FDM contractions in FP16 / BF16 on the matrix cores,
    # the smoother's A reading FP16 geometric factors, and both FP16 options
    if not a.no_fp64:
        for name, prec, fp, gp in (("fp64", sem.F64, None, sem.F32),
                                   ("fp16_fdm", sem.F32, sem.F16, sem.F32),
                                   ("bf16_fdm", sem.F32, sem.BF16, sem.F32),
                                   ("fp16_geom", sem.F32, None, sem.F16),
                                   ("fp16_fdm_geom", sem.F32, sem.F16, sem.F16)):
            sm, _ = make(prec, fp, gp)
            sm.solve(b, rtol=1e-8, maxit=200)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            xm, im = sm.solve(b, rtol=1e-8, maxit=200)
            torch.cuda.synchronize()
            tm = 1e3 * (time.perf_counter() - t1)
            sols[name] = (xm.cpu().numpy(), im, tm)
            note(f"{name} solve {tm:.2f} ms iters={im.iters}")
            sm.close()
            del sm, xm
    solves = {}
    x64 = sols["fp64"][0] if "fp64" in sols else None
    for name, (xs, info, tms) in sols.items():
        rec = {"ms": round(tms, 2), "iters": info.iters, "true_rel_res": info.true_rel_res}
        if x64 is not None and name != "fp64":
            rec["rel_diff_vs_fp64_gpu"] = float(np.linalg.norm(xs - x64) / np.linalg.norm(x64))
            rec["speedup_vs_fp64"] = round(sols["fp64"][2] / tms, 3)
        solves[name] = rec

    ctx = {}
    if not a.no_config2:
        ctx["config2"] = config2_run(a)
        note(f"config2 {ctx['config2']}")
    if not a.no_batch:
        ctx["batch"] = batch_run(SimpleNamespace(nprob=64, no_tune=False), oracle_lanes=not a.no_oracle)
        note(f"batch {ctx['batch']['batched_s']} s, x{ctx['batch']['speedup_batched_vs_sequential_fp64']}"
             " vs sequential FP64")
    torch.cuda.synchronize()

    # the FP64 oracle on the host: residual of every solution, and the CPU baseline
    osolver = None
    if not a.no_oracle or not a.no_cpu_baseline:
        osolver, t_osetup = oracle_solver_shift(n, p, sched, lam_tilde)
        note(f"oracle set up in {t_osetup:.1f} s")
    if not a.no_oracle:
        Lo = osolver.fine
        bo = oracle_rhs(Lo, f, Lo.X)
        for name, (xs, info, _) in sols.items():
            solves[name]["oracle_rel_res"] = oracle_rel_res(Lo, bo, xs)
            note(f"oracle residual of the {name} solution: {solves[name]['oracle_rel_res']:.3e}")
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline_sample(osolver, f, L0.nglobal, int(np.median(iters)), a.cpu_iters)
        cpu["sample"] += f"; oracle set up in {t_osetup:.0f} s (untimed)"
        note(f"cpu baseline {cpu}")

    out = {
        "metric": "Ax GDOF/s + %HBM roofline at p=7; time-to-1e-8 mixed vs FP64 solve",
        "value": round(value, 4),
        "unit": "GDOF/s",
        "value_note": "unique DOF per second of the whole timed step: one mixed-precision solve "
                      "from x = 0 to 1e-8 (the metric's Ax rate is ax64_gdof_s)",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer / f32 smoother",
        "data": "synthetic",
        "config": {"workload": f"layer-shift box {n}^3 hex, p={p}, Dirichlet, sin RHS; "
                               f"FCG + pMG{sched} Cheby-RAS(2) FP32, coarse p=1 "
                               + ("exact block-tridiagonal solve" if coarse_used == "direct"
                                  else f"Jacobi-PCG {a.coarse_tol:g}") + ", tol 1e-8",
                   "coarse_solver": coarse_used,
                   "elements": int(L0.E), "p": p, "n_unique": int(L0.nglobal),
                   "n_local": int(L0.nlocal), "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "iters": iters,
        "true_rel_res": infos[-1].true_rel_res,
        "lambda_tilde": [round(v, 4) for v in lam_tilde],
        "setup_s": round(t_setup, 3),
        "ax64_gdof_s": round(ax_gdofs, 3) if ax_gdofs else None,
        "ax64_hbm_frac": round(ax["GBs"] / HBM_PEAK_GBS, 4) if ax else None,
        "fdm_roofline": fdm_roof,
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "solves": solves,
        "speedup_mixed_vs_fp64": solves["mixed"].get("speedup_vs_fp64"),
        **ctx,
    }
    print(json.dumps(out), flush=True)


def oracle_solver_shift(n, p, sched, lam_tilde):
    """The oracle's pMG solver on the layer-shift mesh, with the GPU's lambda~
    per level (the same Chebyshev bounds) and a Jacobi-PCG coarse solve to 1e-10."""
    from oracle.hierarchy import Solver as OSolver
    from paper_2110_07663_amd import workloads as wl
    t0 = time.perf_counter()
    o = OSolver(n, n, n, wl.layer_shift_vertices(n, seed=3), 1, sched, smoother="ras", cheb_order=2,
                lambda_override=list(lam_tilde) + [0.0], coarse_tol=1e-10)
    return o, time.perf_counter() - t0


def cpu_baseline_sample(o, f, nglobal, gpu_iters, iters):
    """The oracle (plain NumPy FP64) timed on the host: `iters` FCG iterations
    of the same solve with all the host's threads available to it, scaled to
    the GPU's iteration count (same algorithm, same Chebyshev bounds)."""
    from threadpoolctl import threadpool_limits
    hi = host_info()
    Lo = o.fine
    bo = oracle_rhs(Lo, f, Lo.X)
    t_ax = {}
    for th in (1, hi["threads_all"]):
        with threadpool_limits(limits=th):
            t0 = time.perf_counter()
            Lo.apply_A(bo)
            t_ax[str(th)] = round(time.perf_counter() - t0, 3)
    with threadpool_limits(limits=hi["threads_all"]):
        t0 = time.perf_counter()
        o.solve(bo, tol=1e-30, maxit=iters)
        t_it = (time.perf_counter() - t0) / iters
    t_solve = t_it * gpu_iters
    return {"value": round(nglobal / t_solve / 1e9, 7), "unit": "GDOF/s",
            "cores": hi["threads_all"], "kind": "oracle",
            "sample": f"NumPy FP64 oracle, same mesh and bounds (GPU lambda~), coarse Jacobi-PCG "
                      f"1e-10 instead of the GPU's exact solve: {iters} FCG iteration(s) timed "
                      f"({t_it:.1f} s each) with {hi['threads_all']} threads allowed, scaled to the "
                      f"GPU's {gpu_iters} iterations",
            "host": hi["cpu_model"], "nproc": hi["nproc"],
            "apply_A_s_by_threads": t_ax}


def cpu_mode(a):
    """The oracle timed on the host, as the measurement protocol asks: apply_A
    at the 16^3 and 32^3 p = 7 workloads, the full 4^3 p = 3 Jacobi-PCG solve
    and the full 16^3 p = 7 pMG solve, and three FCG iterations of the 32^3
    p = 7 workload, each at 1 thread and at all threads."""
    from threadpoolctl import threadpool_limits
    from oracle.hierarchy import Solver as OSolver
    from oracle import gll as ogll
    from paper_2110_07663_amd import workloads as wl
    hi = host_info()
    res = {"mode": "cpu", **hi, "runs": {}}

    def log(k, v):
        res["runs"][k] = v
        print(f"[cpu] {k}: {v}", file=sys.stderr, flush=True)

    f, _ = wl.sinusoid(1, 1, 1)
    for th in (1, hi["threads_all"]):
        with threadpool_limits(limits=th):
            # config 1: 4^3 undeformed cube, p = 3, Jacobi-PCG to 1e-10
            t0 = time.perf_counter()
            o1 = OSolver(4, 4, 4, wl.box_vertices(4, 4, 4), 1, (3,))
            bo = o1.rhs(f(*o1.fine.X))
            t1 = time.perf_counter()
            r1 = o1.jacobi_pcg(bo, 1e-10, 500)
            log(f"config1_solve_t{th}", {"setup_s": round(t1 - t0, 3),
                                         "solve_s": round(time.perf_counter() - t1, 3),
                                         "iters": r1.iters})
            # config 2: 16^3 sine map, p = 7, pMG (7,3,1) Cheby-Jacobi(2), coarse PCG 1e-10
            xyz = wl.sampled_mesh(16, 16, 16, ogll.gll_nodes_weights(7)[0], wl.sin_map(0.05))
            t0 = time.perf_counter()
            o2 = OSolver(16, 16, 16, xyz, 7, (7, 3, 1), smoother="jacobi", coarse_tol=1e-10)
            bo = o2.rhs(f(*o2.fine.X))
            t1 = time.perf_counter()
            o2.fine.apply_A(bo)
            t2 = time.perf_counter()
            print(f"[cpu] config2_t{th}: set up in {t1 - t0:.1f} s, apply_A {t2 - t1:.2f} s",
                  file=sys.stderr, flush=True)
            r2 = o2.solve(bo, tol=1e-8, maxit=300, krylov="pcg")
            log(f"config2_t{th}", {"setup_s": round(t1 - t0, 2), "apply_A_s": round(t2 - t1, 3),
                                   "solve_s": round(time.perf_counter() - t2, 2), "iters": r2.iters})
            del o2
            # config 3: 32^3 layer shift, p = 7, Cheby-RAS(2) (7,3,1); 3 FCG iterations
            t0 = time.perf_counter()
            o3 = OSolver(32, 32, 32, wl.layer_shift_vertices(32, seed=3), 1, (7, 3, 1),
                         smoother="ras", lambda_override=[26.4181, 20.1744, 0.0], coarse_tol=1e-10)
            bo = o3.rhs(f(*o3.fine.X))
            t1 = time.perf_counter()
            o3.fine.apply_A(bo)
            t2 = time.perf_counter()
            print(f"[cpu] config3_t{th}: set up in {t1 - t0:.1f} s, apply_A {t2 - t1:.2f} s",
                  file=sys.stderr, flush=True)
            its = []
            for k in range(3):  # one FCG iteration (one V-cycle and one A) at a time
                t3 = time.perf_counter()
                o3.solve(bo, tol=1e-30, maxit=1)
                its.append(time.perf_counter() - t3)
                print(f"[cpu] config3_t{th}: FCG iteration {k + 1}: {its[-1]:.1f} s", file=sys.stderr,
                      flush=True)
            log(f"config3_t{th}", {"setup_s": round(t1 - t0, 2), "apply_A_s": round(t2 - t1, 3),
                                   "fcg_iteration_s": round(float(np.mean(its)), 2),
                                   "solve_52_iterations_s_extrapolated": round(float(np.mean(its)) * 52, 1)})
            del o3
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
