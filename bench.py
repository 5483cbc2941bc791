"""Benchmark: DOFs/s to a 1e-10 relative residual, 3D Poisson 256^3.

Workload: -Lap u = f on the unit cube, 256^3 cell-centred grid, zero
Dirichlet boundary, f = sum of 8 seeded sine modes (seed 0), V(2,2) cycles
with weighted Jacobi (omega = 2/3), 8-cell restriction, trilinear
prolongation, 4^3 exact coarsest solve.  One step = one complete solve from
x = 0 to ||f - A x||_2 / ||f||_2 <= 1e-10, inputs resident in HBM.

Paths: mixed-precision refinement with FP32 inner cycles (the headline
`value`), the same with BF16 storage, and plain FP64 V-cycles; all three are
timed and reported.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 256
TOL = 1e-10
SWEEP_REPS = 50
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_path(B, fg, xg, h, prec, steps, warmup):
    """Wall time of `steps` solves (graph-replayed cycles, no per-kernel events)."""
    import torch
    for _ in range(warmup):
        B.mg_poisson_solve(fg, xg, h, B.BC_DIRICHLET0, tol=TOL, smooth_prec=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(steps):
        _, stats = B.mg_poisson_solve(fg, xg, h, B.BC_DIRICHLET0, tol=TOL, smooth_prec=prec)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats


def kernel_times(B, fg, xg, h, prec, steps):
    """Per-kind duration of the finest-level kernels over `steps` solves, each launch
    bracketed by HIP events on the stream it runs on (graph replay is off while timing)."""
    import torch
    out = {}
    kinds = (("sweep", B.PROF_JACOBI), ("sweep_zero", B.PROF_SWEEP_ZERO), ("restrict", B.PROF_RESTRICT),
             ("prolong", B.PROF_PROLONG),
             ("refine", B.PROF_REFINE), ("fused_down", B.PROF_DOWN), ("fused_down_zero", B.PROF_DOWN_ZERO),
             ("fused_up", B.PROF_UP))
    for name, mask in kinds:
        B.np_prof_enable(mask)
        for _ in range(steps):
            B.mg_poisson_solve(fg, xg, h, B.BC_DIRICHLET0, tol=TOL, smooth_prec=prec)
        torch.cuda.synchronize()
        n, ms, by = B.np_prof_read()
        B.np_prof_enable(0)
        if n:
            out[name] = dict(launches=n, avg_us=1e3 * ms / n, bytes_per_launch=by / n,
                             gbs=(by / n) / (ms / n * 1e-3) / 1e9)
    return out


def copy_bandwidth(reps=5):
    """Measured device copy rate (torch's copy kernel, 512 MiB read + 512 MiB write)."""
    import torch
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return 2 * a.numel() * 8 / dt / 1e9


SOLVER_PROFILE = os.path.join(ROOT, "profiles", "mg_level_kernels_poisson3d_256.md")

# source region of each finest-level kernel whose counter traffic the profile records:
# (file under csrc/, first line, line after the region)
KERNEL_SOURCES = {
    "refine": ("mg_level.h", "// Refinement step of the mixed path on the z-marching tiles",
               "// x += P ec on the z-marching tiles"),
    "sweep": ("mg_zfused.h", "template <class S> struct Z2Cfg {", "// The down-leg of a large 3D level"),
    "fused_up": ("mg_zfused.h", "template <class S> struct Z2Cfg {", "// The down-leg of a large 3D level"),
    "fused_down_zero": ("mg_zfused.h", "// The down-leg of a large 3D level", "}  // namespace np"),
    "fused_down": ("mg_zfused.h", "// k_down2z on two cells per thread", "}  // namespace np"),
    "restrict": ("mg_level.h", "// Residual + restriction on the z-marching tiles",
                 "// Refinement step of the mixed path on the z-marching tiles"),
}


def kernel_source_hash(kind):
    """Hash of a finest-level kernel's source, which the counter summary records with
    its traffic: counters taken on other code are not reported."""
    import hashlib
    fname, first, after = KERNEL_SOURCES[kind]
    src = open(os.path.join(ROOT, "paper_2402_17913_amd", "csrc", fname)).read()
    body = src[src.index(first):src.index(after, src.index(first))]
    # the z-marching tile shape (cells per thread) that every one of these kernels takes
    lvl = open(os.path.join(ROOT, "paper_2402_17913_amd", "csrc", "mg_level.h")).read()
    cfg = lvl[lvl.index("template <class S> struct ZCfg {"):lvl.index("};", lvl.index("template <class S> struct ZCfg {"))]
    return hashlib.sha256((cfg + body).encode()).hexdigest()[:16]


def measured_traffic(kernel, head):
    """HBM bytes per launch of the dominant kernel at the finest level from the
    committed rocprofv3 counter summary, if the kernel's source is unchanged since
    the counters were taken."""
    import re
    if kernel not in KERNEL_SOURCES or not os.path.exists(SOLVER_PROFILE):
        return None
    txt = open(SOLVER_PROFILE).read()
    m1 = re.search(r"^traffic_%s_%s_bytes_per_launch: (\d+)" % (kernel, head), txt, re.M)
    m2 = re.search(r"^traffic_%s_source_sha256_16: (\w+)" % kernel, txt, re.M)
    if not (m1 and m2) or kernel_source_hash(kernel) != m2.group(1):
        return None
    return int(m1.group(1))


def host_threads():
    """Host threads the oracle may use: OMP_NUM_THREADS when set (the CPU share of
    the process), else the CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else len(os.sched_getaffinity(0))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(f, h, gpu_x):
    """The oracle on the host cores.  All cores: its OpenMP timing build (-O3, the
    solve's cell loops in parallel) runs full solves of the same 256^3 problem to
    1e-10, one untimed then the median of three.  One core: the same build on a
    bounded sample, two V-cycles with the residual evaluation around them, scaled to
    the cycle count of a full solve.  The untimed solve's converged x is the FP64
    oracle solution that each GPU path's result (gpu_x: name -> host array) is
    compared with: max |x - x_oracle| / max |x_oracle|."""
    import numpy as np

    import oracle
    threads = host_threads()
    ref = oracle.mg_solve(f, h, oracle.BC_DIRICHLET0, tol=TOL, threads=threads)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        res = oracle.mg_solve(f, h, oracle.BC_DIRICHLET0, tol=TOL, threads=threads)
        times.append(time.perf_counter() - t0)
    t_all = sorted(times)[1]
    sample_cycles = 2
    t0 = time.perf_counter()
    oracle.mg_solve(f, h, oracle.BC_DIRICHLET0, fixed_cycles=sample_cycles, threads=1)
    t_one = (time.perf_counter() - t0) / sample_cycles * res.cycles
    scale = float(np.abs(ref.x).max())
    err = {name: float(np.abs(x - ref.x).max()) / scale for name, x in gpu_x.items()}
    base = dict(value=f.size / t_all, unit="DOF/s", cores=threads, kind="oracle",
                sample="full solves of the %d^3 workload to 1e-10 (%d cycles, rel_res %.2e) by the oracle's "
                       "OpenMP timing build on %d threads: median of 3 after 1 untimed, %.2f s each"
                       % (f.shape[0], res.cycles, res.rel_res, threads, t_all),
                cpu_model=cpu_model(), seconds_per_solve=t_all, seconds_per_solve_runs=times,
                single_thread=dict(value=f.size / t_one, unit="DOF/s", cores=1,
                                   sample="%d oracle V(2,2) cycles with their residual checks on the same "
                                          "problem, scaled to the %d cycles of a full solve (%.1f s)"
                                          % (sample_cycles, res.cycles, t_one)),
                note="the oracle is plain unfused C loops (a reference, not a tuned CPU multigrid)")
    return base, dict(norm="max|x - x_oracle| / max|x_oracle|, x_oracle the oracle's FP64 solve to 1e-10",
                      oracle_cycles=ref.cycles, oracle_rel_res=ref.rel_res, **err)


def timed(fn, steps, warmup):
    """Wall time of `steps` calls of fn after `warmup` untimed ones (device synced
    on both sides); returns (seconds, last result)."""
    import torch
    out = None
    for _ in range(warmup):
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def leg_c1(B, inputs, steps, warmup):
    """2D Poisson 128^2, Dirichlet-0, manufactured sin(pi x) sin(pi y) + 8 modes, FP64."""
    import torch
    g = inputs.manufactured_2d(128, seed=0)
    f = torch.from_numpy(g["f"]).cuda()
    x = torch.zeros_like(f)
    dt, (_, st) = timed(lambda: B.mg_poisson_solve(f, x, g["h"], B.BC_DIRICHLET0, tol=TOL), steps, warmup)
    return dict(workload="poisson2d_128sq_dirichlet_manufactured_seed0_fp64", dofs=f.numel(),
                dofs_per_s=f.numel() * steps / dt, ms_per_solve=1e3 * dt / steps, cycles=st["cycles"],
                rel_res=st["rel_res"])


def leg_c2(B, inputs, nsteps=100):
    """2D NS projection steps, 1024^2 periodic, nu = 1e-3, 100 steps from the seeded
    divergence-free field; pressure increment from zero, and from the previous step's."""
    import torch
    n = 1024
    g = inputs.divfree_velocity(2, n, seed=0)
    out = {}
    for name, ws in (("zero_guess", 0), ("previous_dp_guess", 2)):
        B.np_release_all()
        u, v = [torch.from_numpy(c).cuda() for c in g["q"]]
        p = torch.zeros_like(u)
        # untimed: one step on a copy of the state allocates the workspaces and captures the
        # graphs; then the previous increment is cleared, so the timed run starts from zero
        uw, vw = u.clone(), v.clone()
        B.ns_projection_step(uw, vw, None, p.clone(), g["h"], g["dt"], 1e-3, tol=TOL, warm_start=ws)
        uw.zero_()
        vw.zero_()
        B.ns_projection_step(uw, vw, None, torch.zeros_like(p), g["h"], g["dt"], 1e-3, tol=TOL, warm_start=0)
        del uw, vw
        ke0 = float(0.5 * (u.square().sum() + v.square().sum())) * g["h"] ** 2
        cyc = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            _, st = B.ns_projection_step(u, v, None, p, g["h"], g["dt"], 1e-3, tol=TOL, warm_start=ws)
            cyc.append(st["cycles"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ke = float(0.5 * (u.square().sum() + v.square().sum())) * g["h"] ** 2
        cfl = g["dt"] * (float(u.abs().max()) + float(v.abs().max())) / g["h"]
        out[name] = dict(cell_steps_per_s=n * n * nsteps / dt, ms_per_step=1e3 * dt / nsteps,
                         mean_cycles=sum(cyc) / len(cyc), max_cycles=max(cyc), kinetic_energy=[ke0, ke],
                         final_cfl=cfl)
        log("  C2 %s: %.2f ms/step, %.1f cycles/step" % (name, 1e3 * dt / nsteps, sum(cyc) / len(cyc)))
    return dict(workload="ns2d_1024sq_periodic_divfree_seed0_nu1e-3_100steps_fp64", steps=nsteps, **out)


def leg_c4(B, inputs, steps, warmup):
    """512 batched 2D Dirichlet solves, sizes drawn by seed 0 from {64..1024}^2, RHS
    seed 1000 + i; FP32 inner cycles with FP64 refinement, autotuned inner count."""
    import torch
    sizes = inputs.batched_sizes(512, seed=0)
    fs = [torch.from_numpy(inputs.sine_rhs(2, n, seed=1000 + i)["f"]).cuda() for i, n in enumerate(sizes)]
    xs = [torch.zeros_like(f) for f in fs]
    hs = [1.0 / n for n in sizes]
    dofs = sum(n * n for n in sizes)
    t0 = time.perf_counter()
    B.mg_poisson_solve_batched(fs, xs, hs, smooth_prec=B.FP32, inner_cycles=0)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    inner, tune_ms = B.np_last_autotune()
    settings = B.np_last_batched_settings()
    dt, (_, stats) = timed(lambda: B.mg_poisson_solve_batched(fs, xs, hs, smooth_prec=B.FP32, inner_cycles=0),
                           steps, warmup)
    worst = max(s["rel_res"] for s in stats)

    def solo():
        for f, x, h in zip(fs, xs, hs):
            B.mg_poisson_solve(f, x, h, B.BC_DIRICHLET0, tol=TOL, smooth_prec=B.FP32)
    dts, _ = timed(solo, 1, 1)
    hist = {str(c): sizes.count(c) for c in sorted(set(sizes))}
    return dict(workload="batched_poisson2d_512_sizes64-1024_seed0_fp32+fp64", problems=len(sizes), dofs=dofs,
                size_histogram=hist, dofs_per_s=dofs * steps / dt, ms_per_batch=1e3 * dt / steps,
                first_call_s=setup, autotune_ms=tune_ms, autotuned_settings=settings, worst_rel_res=worst,
                one_at_a_time_dofs_per_s=dofs / dts, batched_over_one_at_a_time=(dofs * steps / dt) / (dofs / dts))


def leg_c5(B, inputs, nsteps=10):
    """3D projection steps, 256^3 periodic, nu = 1e-3, seed 0 (held out from the
    network's training seeds 1..20): pressure increment from zero, from the previous
    step's increment, and from the learned warm start; FP64, FP32-inner and BF16-inner solves."""
    import torch
    from paper_2402_17913_amd import learned
    n = 256
    wpath = os.path.join(ROOT, "paper_2402_17913_amd", "weights", "ns3d_periodic_256_in128_L4.npcnn")
    g = inputs.divfree_velocity(3, n, seed=0)
    out = {}
    for prec_name, prec in (("fp64", B.FP64), ("fp32", B.FP32), ("bf16", B.BF16)):
        variants = [("zero_guess", 0, 0), ("previous_dp_guess", 2, 0), ("learned_guess", 1, 0)]
        if prec == B.FP64:  # the learned coarse-grid correction runs on FP64 V-cycles
            variants += [("learned_cgc_first_cycle", 0, 1), ("learned_cgc_every_cycle", 0, 256),
                         ("previous_dp_guess_and_learned_cgc_first_cycle", 2, 1)]
        for name, ws, cgc in variants:
            B.np_cnn_load(wpath if ws == 1 or cgc > 0 else None)
            q = [torch.from_numpy(c).cuda() for c in g["q"]]
            p = torch.zeros_like(q[0])
            # untimed: one step from a copy of the state warms workspaces, graphs and
            # the network for this grid; one step of a zero field then leaves a zero
            # increment behind, so the first timed step starts from zero under every
            # variant (there is no previous increment before the first step)
            qw = [c.clone() for c in q]
            B.ns_projection_step(qw[0], qw[1], qw[2], p.clone(), g["h"], g["dt"], 1e-3, tol=TOL,
                                 warm_start=1 if ws == 1 else 0, smooth_prec=prec, cnn_cgc=cgc)
            for c in qw:
                c.zero_()
            B.ns_projection_step(qw[0], qw[1], qw[2], torch.zeros_like(p), g["h"], g["dt"], 1e-3, tol=TOL,
                                 warm_start=0, smooth_prec=prec)
            del qw
            cyc, fb, kept = [], 0, 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(nsteps):
                _, st = B.ns_projection_step(q[0], q[1], q[2], p, g["h"], g["dt"], 1e-3, tol=TOL,
                                             warm_start=ws, smooth_prec=prec, cnn_cgc=cgc)
                cyc.append(st["cycles"])
                fb += st["used_fallback"]
                kept += st["cgc_accepted"]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            out["%s_%s" % (prec_name, name)] = dict(ms_per_step=1e3 * dt / nsteps, cycles=cyc,
                                                    fallbacks=fb if ws == 1 else None,
                                                    coarse_corrections_kept=kept if cgc else None)
            log("  C5 %s %s: %.2f ms/step, cycles %s" % (prec_name, name, 1e3 * dt / nsteps, cyc))
    B.np_cnn_load(None)
    net = B.Cnn(path=wpath)
    xin = torch.randn((net.n_in,) * 3, dtype=torch.float32, device="cuda")
    y = torch.empty_like(xin)
    dt, _ = timed(lambda: net.forward(xin, y), 10, 2)
    # one training step (forward, backward, Adam) on a batch of 4 synthetic pairs at the
    # network's input size, on a copy of the trained weights
    xb = [torch.randn((net.n_in,) * 3, dtype=torch.float32, device="cuda") for _ in range(4)]
    tb = [torch.randn((net.n_in,) * 3, dtype=torch.float32, device="cuda") for _ in range(4)]
    dts, _ = timed(lambda: net.train_step(xb, tb, 1e-4), 5, 1)
    net.close()
    meta = json.load(open(os.path.splitext(wpath)[0] + ".json"))
    return dict(workload="ns3d_256cube_periodic_divfree_seed0_nu1e-3_%dsteps" % nsteps, steps=nsteps,
                network=dict(n_in=meta["n_in"], levels=meta["levels"], pairs=meta["pairs"],
                             training_seeds=meta["seeds"], epochs=meta["epochs"],
                             training_s=meta["training_s"], pair_generation_s=meta["pair_generation_s"],
                             forward_ms=1e3 * dt / 10, train_step_ms_batch4=1e3 * dts / 5),
                **out)


def leg_c5_zero(B, inputs, nsteps=3):
    """The 3D projection step of C5 (256^3 periodic, seed 0) from a zero pressure
    increment only, FP64 and BF16-inner solves, no network: a short run for kernel
    profiles of the momentum stages, the divergence, the correction and the solves."""
    import torch
    n = 256
    g = inputs.divfree_velocity(3, n, seed=0)
    out = {}
    for prec_name, prec in (("fp64", B.FP64), ("bf16", B.BF16)):
        q = [torch.from_numpy(c).cuda() for c in g["q"]]
        p = torch.zeros_like(q[0])
        B.ns_projection_step(q[0].clone(), q[1].clone(), q[2].clone(), p.clone(), g["h"], g["dt"], 1e-3, tol=TOL,
                             smooth_prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            B.ns_projection_step(q[0], q[1], q[2], p, g["h"], g["dt"], 1e-3, tol=TOL, smooth_prec=prec)
        torch.cuda.synchronize()
        out[prec_name] = dict(ms_per_step=1e3 * (time.perf_counter() - t0) / nsteps)
        log("  C5 zero-guess %s: %.2f ms/step" % (prec_name, out[prec_name]["ms_per_step"]))
    return dict(workload="ns3d_256cube_periodic_divfree_seed0_nu1e-3_%dsteps_zero_guess" % nsteps, **out)


def leg_sawtooth(B, inputs, steps, warmup):
    """The paper's sawtooth cycle against V(2,2): as printed (alpha = 1, one Jacobi
    step, copying prolongation) and damped (alpha = 2/3, two steps, linear
    prolongation), on the 2D 128^2 manufactured source and the 3D 256^3 sine
    source (Dirichlet, FP64, tol 1e-10): measured contraction per cycle, cycles
    and time per solve."""
    import torch
    out = {}
    cases = (("2d_128", inputs.manufactured_2d(128, seed=0)), ("3d_256", inputs.sine_rhs(3, 256, seed=0)))
    variants = (("v22", dict()),
                ("sawtooth_printed", dict(cycle=B.CYCLE_SAWTOOTH, prolong=B.PROLONG_COPY, nu1=0, nu2=1, omega=1.0,
                                          max_cycles=40)),
                ("sawtooth_damped_linear", dict(cycle=B.CYCLE_SAWTOOTH, nu1=0, nu2=2, omega=2.0 / 3.0)))
    for name, g in cases:
        f = torch.from_numpy(g["f"]).cuda()
        x = torch.zeros_like(f)
        res = {}
        for vn, kw in variants:
            dt, (st, stats) = timed(lambda: B.mg_poisson_solve(f, x, g["h"], B.BC_DIRICHLET0, tol=TOL, check=False,
                                                               **kw), max(1, steps // 2), 1)
            hist = [v for v in stats["hist"][:stats["cycles"] + 1] if v > 0]
            tail = hist[-6:]
            rho = (tail[-1] / tail[0]) ** (1.0 / (len(tail) - 1)) if len(tail) > 1 else None
            res[vn] = dict(status="converged" if st == 0 else "not converged (status %d)" % st,
                           cycles=stats["cycles"], rel_res=stats["rel_res"], rho_last5=rho,
                           ms_per_solve=1e3 * dt / max(1, steps // 2))
            log("  sawtooth leg %s %s: %s, %d cycles, rho %.3f, %.2f ms" % (
                name, vn, res[vn]["status"], stats["cycles"], rho or -1, res[vn]["ms_per_solve"]))
        out[name] = res
        del f, x
    return dict(workload="sawtooth_vs_v22_dirichlet_fp64_tol1e-10", **out)


def ad_level_live(B, T0, h, op):
    """Finest-level kernels of the advection-diffusion solve timed live: SWEEP_REPS
    back-to-back launches of the solver's own kernel and launch shape between HIP
    events on the library stream (np_ad_prof_level), against HBM peak."""
    import torch
    d, n = T0.dim(), T0.shape[0]
    m = T0.numel()
    x = torch.randn_like(T0)
    y = torch.zeros_like(T0)
    yc = torch.zeros((n // 2,) * d, dtype=torch.float64, device=T0.device)
    out = {}
    for kname, kind, nbytes in (("sweep", B.PROF_LEVEL_SWEEP, 24 * m), ("restrict", B.PROF_LEVEL_RESTRICT,
                                                                         16 * m + 8 * m // 2 ** d),
                                ("prolong", B.PROF_LEVEL_PROLONG, 16 * m + 8 * m // 2 ** d)):
        ms = B.np_ad_prof_level(kind, T0, x, y if kind == B.PROF_LEVEL_SWEEP else yc, h, B.BC_DIRICHLET0, op,
                                reps=SWEEP_REPS)
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[kname] = dict(avg_us=1e3 * ms, bytes_per_launch=nbytes, gbs=gbs, frac=gbs / HBM_PEAK_GBS)
    return out


def leg_ad(B, inputs, steps, warmup):
    """Implicit advection-diffusion multigrid (Section 2.2 backward Euler, Section 3.2
    experiment): the paper's case (128^2, Dirichlet, u = v = 1, nu = 2, dt = 50, dx = 1,
    Gaussian gamma = 10 at the centre, upwind, zero first estimate) with the paper's
    L1 change gauge for V(2,2) and the sawtooth variants, then the same per-cell
    coefficients at 4096^2 (gamma 320) and 256^3 (gamma 20): time to 1e-10 and the
    finest-level kernels against HBM."""
    import torch
    out = {}
    T0 = torch.from_numpy(inputs.gaussian_2d(128, gamma=10.0)).cuda()
    x = torch.zeros_like(T0)
    op = B.ad_op(50.0, 2.0, [1.0, 1.0], 0)
    paper = {}
    variants = (("v22", dict()),
                ("sawtooth_printed", dict(cycle=B.CYCLE_SAWTOOTH, prolong=B.PROLONG_COPY, nu1=0, nu2=1, omega=1.0)),
                ("sawtooth_linear", dict(cycle=B.CYCLE_SAWTOOTH, nu1=0, nu2=1, omega=1.0)),
                ("sawtooth_damped_linear", dict(cycle=B.CYCLE_SAWTOOTH, nu1=0, nu2=2, omega=2.0 / 3.0)))
    for vn, kw in variants:
        # the paper's gauge over 256 cycles: the change at 50 cycles and the first cycle whose
        # change falls below its tolerance 1e-5
        st, sg = B.np_ad_implicit_solve(T0, x, 1.0, B.BC_DIRICHLET0, op, check=False, l1=True, fixed_cycles=256,
                                        **kw)
        l1 = sg["l1_change"][:50]
        below = [k + 1 for k, v in enumerate(sg["l1_change"]) if v < 1e-5]
        dt, (st, stats) = timed(lambda: B.np_ad_implicit_solve(T0, x, 1.0, B.BC_DIRICHLET0, op, tol=TOL, check=False,
                                                               max_cycles=100, **kw), max(1, steps // 2), 1)
        paper[vn] = dict(l1_change_first=l1[0], l1_change_50=l1[-1], l1_reduction_50=l1[-1] / l1[0],
                         first_cycle_l1_below_1e5=below[0] if below else None,
                         status="converged" if st == 0 else "not converged (status %d)" % st,
                         cycles_to_tol=stats["cycles"], rel_res=stats["rel_res"],
                         ms_per_solve=1e3 * dt / max(1, steps // 2))
        log("  ad paper %s: L1 change %.3g -> %.3g in 50 cycles, below 1e-5 from cycle %s; tol 1e-10: %s, %d "
            "cycles, %.2f ms" % (vn, l1[0], l1[-1], paper[vn]["first_cycle_l1_below_1e5"], paper[vn]["status"],
                                 stats["cycles"], paper[vn]["ms_per_solve"]))
    out["paper_2d_128"] = paper
    del T0, x
    out.update(ad_large(B, inputs, steps, warmup))
    return dict(workload="ad_implicit_dirichlet_upwind_C50_nu_dt100_gaussian_tol1e-10_fp64", **out)


def ad_large(B, inputs, steps, warmup):
    """The advection-diffusion solve at 4096^2 (gamma 320) and 256^3 (gamma 20): time
    to 1e-10 and the finest-level kernels against HBM (the same coefficients as the
    paper's 128^2 case)."""
    import torch
    out = {}
    for name, d, n, gamma in (("2d_4096", 2, 4096, 320.0), ("3d_256", 3, 256, 20.0)):
        T0 = torch.from_numpy(inputs.gaussian_2d(n, gamma=gamma) if d == 2 else
                              inputs.gaussian_3d(n, gamma=gamma)).cuda()
        x = torch.zeros_like(T0)
        opd = B.ad_op(50.0, 2.0, [1.0] * d, 0)
        solve = lambda: B.np_ad_implicit_solve(T0, x, 1.0, B.BC_DIRICHLET0, opd, tol=TOL)
        dt, (st, stats) = timed(solve, steps, warmup)
        ker = ad_level_live(B, T0, 1.0, opd)
        out[name] = dict(dofs=T0.numel(), dofs_per_s=T0.numel() * steps / dt, ms_per_solve=1e3 * dt / steps,
                         cycles=stats["cycles"], rel_res=stats["rel_res"], rho=stats["rho_est"],
                         finest_level_kernels=ker)
        log("  ad %s: %.2f ms, %d cycles, %.3g DOF/s; sweep %.1f us (%.2f of HBM peak)" % (
            name, out[name]["ms_per_solve"], stats["cycles"], out[name]["dofs_per_s"],
            ker.get("sweep", {}).get("avg_us", -1), ker.get("sweep", {}).get("frac", -1)))
        del T0, x
    return out


def leg_explicit(B, inputs, steps, warmup):
    """Explicit advection-diffusion step with the paper's filter families (Section 2.1,
    Appendix A): central, upwind and finite element, on 4096^2 (rotation) and 256^3
    (divergence-free field), Dirichlet-0.  Throughput in cell-steps/s and the step's
    algorithmic bytes (predictor: T and a read, T~ and a copy of T written; corrector:
    the copy, T~ and a read, T written) against HBM peak."""
    import torch
    out = {}
    for name, d, n in (("2d_4096", 2, 4096), ("3d_256", 3, 256)):
        T, a, h, dt, nu = inputs.explicit_ad_case(d, n)
        Tg = torch.from_numpy(T).cuda()
        ag = [torch.from_numpy(c).cuda() for c in a]
        m = Tg.numel()
        nbytes = m * (8 * (1 + d + 2) + 8 * (2 + d + 1))  # predictor writes T~ and a copy of T
        res = {}
        for sname, scheme in (("central", 0), ("upwind", 1), ("finite_element", 2)):
            dt_s, _ = timed(lambda: B.np_ad_explicit_step(Tg, h, dt, nu, B.BC_DIRICHLET0, a=ag, scheme=scheme),
                            steps, warmup)
            ms = 1e3 * dt_s / steps
            gbs = nbytes / (ms * 1e-3) / 1e9
            res[sname] = dict(ms_per_step=ms, cell_steps_per_s=m / (ms * 1e-3), bytes_per_step=nbytes, gbs=gbs,
                              frac=gbs / HBM_PEAK_GBS)
            log("  explicit %s %s: %.3f ms/step, %.3g cell-steps/s, %.0f GB/s (%.2f of HBM peak)" % (
                name, sname, ms, m / (ms * 1e-3), gbs, gbs / HBM_PEAK_GBS))
        out[name] = res
        del Tg, ag
    return dict(workload="explicit_ad_step_dirichlet_gaussian_C0.1_fp64", **out)


def leg_collocated(B, inputs, nsteps=20):
    """The projection step with the paper's collocated nodes and finite-element filters
    (and the central family for comparison), periodic, from the seeded divergence-free
    field: 2D 1024^2 and 3D 256^3, nu = 1e-3, pressure increment from zero to 1e-10.
    Reports time per step, pressure cycles and how much divergence each projection
    leaves (the approximate projection's signature)."""
    import torch
    out = {}
    for name, d, n, steps in (("2d_1024", 2, 1024, nsteps), ("3d_256", 3, 256, max(2, nsteps // 4))):
        g = inputs.divfree_velocity(d, n, seed=0)
        res = {}
        for sname, scheme in (("finite_element", 2), ("central", 0)):
            B.np_release_all()
            q = [torch.from_numpy(c).cuda() for c in g["q"]]
            p = torch.zeros_like(q[0])
            w = q[2] if d == 3 else None
            cyc = []
            div = torch.zeros_like(p)

            def div_rms():  # rms of the scheme's divergence, in units of (velocity rms / h)
                B.np_nsc_divergence(q[0], q[1], w, div, g["h"], scheme=scheme)
                vel = sum(float(c.square().mean()) for c in q) ** 0.5
                return float(div.square().mean()) ** 0.5 * g["h"] / vel

            div0 = div_rms()
            B.ns_collocated_step(q[0], q[1], w, p, g["h"], g["dt"], 1e-3, scheme=scheme, tol=TOL)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                _, st = B.ns_collocated_step(q[0], q[1], w, p, g["h"], g["dt"], 1e-3, scheme=scheme, tol=TOL)
                cyc.append(st["cycles"])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res[sname] = dict(ms_per_step=1e3 * dt / steps, cell_steps_per_s=q[0].numel() * steps / dt,
                              mean_cycles=sum(cyc) / len(cyc), steps=steps + 1,
                              divergence_rms_scaled=[div0, div_rms()])
            log("  collocated %s %s: %.2f ms/step, %.1f cycles/step, divergence rms (x h / |q|) %.2e -> %.2e" % (
                name, sname, 1e3 * dt / steps, sum(cyc) / len(cyc), *res[sname]["divergence_rms_scaled"]))
            del q, p, w, div
        out[name] = res
    return dict(workload="ns_collocated_periodic_divfree_seed0_nu1e-3_fp64", **out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--legs", default="c1,c2,c4,c5,sawtooth,ad,explicit,collocated",
                    help="other workloads to run after the headline (comma list, '' for none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2402_17913_amd import binding as B
    from paper_2402_17913_amd import inputs

    torch.cuda.set_device(0)
    g = inputs.sine_rhs(3, N, seed=0)
    f, h = g["f"], g["h"]
    fg = torch.from_numpy(f).cuda()
    xg = torch.zeros_like(fg)
    dofs = f.size
    copy_gbs = copy_bandwidth()
    log("device copy: %.0f GB/s" % copy_gbs)
    res, gpu_x = {}, {}
    for name, prec in (("fp64", B.FP64), ("fp32", B.FP32), ("bf16", B.BF16)):
        dt, stats = time_path(B, fg, xg, h, prec, args.steps, args.warmup)
        gpu_x[name] = xg.cpu().numpy()
        prof = kernel_times(B, fg, xg, h, prec, max(1, min(args.steps, 3)))
        res[name] = dict(seconds=dt, stats=stats, prof=prof, dofs_per_s=dofs * args.steps / dt)
        log("  kernels: " + ", ".join("%s %.1f us %.0f GB/s" % (k, v["avg_us"], v["gbs"])
                                      for k, v in prof.items()))
        log("%s: %.3f ms/solve, %d cycles, %d outer, rel_res %.3e, %.3e DOF/s" % (
            name, 1e3 * dt / args.steps, stats["cycles"], stats["outer_iters"], stats["rel_res"],
            res[name]["dofs_per_s"]))

    # the headline is the faster of the two mixed-precision paths
    head = "bf16" if res["bf16"]["dofs_per_s"] > res["fp32"]["dofs_per_s"] else "fp32"
    kt = res[head]["prof"]
    # dominant finest-level kernel of the headline path: largest total time
    dom = max(kt, key=lambda k: kt[k]["launches"] * kt[k]["avg_us"])
    # live duration of the finest-level sweep: HIP events around back-to-back
    # launches on the library's stream, on this workload's fields
    level_live = {}
    for name, prec, dt in (("fp64", B.FP64, torch.float64), ("fp32", B.FP32, torch.float32),
                           ("bf16", B.BF16, torch.bfloat16)):
        fl, xl = fg.to(dt), (0.5 * fg).to(dt)
        if dt == torch.bfloat16:
            fl, xl = fl.view(torch.int16), xl.view(torch.int16)
        yl = torch.empty_like(xl)
        cl = torch.zeros((N // 2,) * 3, dtype=xl.dtype, device="cuda")
        sz = {"fp64": 8, "fp32": 4, "bf16": 2}[name]
        level_live[name] = {}
        for kind, kname, nbytes, y in ((B.PROF_LEVEL_SWEEP, "sweep", 3 * dofs * sz, yl),
                                       (B.PROF_LEVEL_RESTRICT, "restrict", (2 * dofs + dofs // 8) * sz, cl),
                                       (B.PROF_LEVEL_PROLONG, "prolong", (2 * dofs + dofs // 8) * sz, cl)):
            # median over 5 rounds of SWEEP_REPS back-to-back launches (each round: mean launch time)
            rounds = sorted(B.np_prof_level(kind, fl, xl if kind != B.PROF_LEVEL_PROLONG else yl, y, h,
                                            B.BC_DIRICHLET0, prec, reps=SWEEP_REPS) for _ in range(5))
            ms = rounds[2]
            level_live[name][kname] = dict(avg_us=1e3 * ms, bytes_per_launch=nbytes,
                                           gbs=nbytes / (ms * 1e-3) / 1e9,
                                           frac=nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
        del fl, xl, yl, cl
    for name, v in level_live.items():
        log("  live %s: " % name + ", ".join("%s %.1f us %.0f GB/s" % (k, w["avg_us"], w["gbs"])
                                             for k, w in v.items()))
    # the dominant kernel's own launches in the timed solves, each bracketed by HIP events
    avg_us, nbytes = kt[dom]["avg_us"], kt[dom]["bytes_per_launch"]
    achieved = nbytes / (avg_us * 1e-6) / 1e9
    line = {
        "metric": "DOFs/s to 1e-10 rel. residual (MG V-cycle), learned/mixed vs plain FP64",
        "value": res[head]["dofs_per_s"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * res[head]["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32+f64", "bf16": "bf16(f32 arith)+f64"}[head],
        "data": "synthetic",
        "config": {
            "workload": "poisson3d_256cube_dirichlet_sine8_seed0_tol1e-10",
            "dofs": dofs,
            "path": {"fp32": "mixed-precision refinement: FP32 inner V(2,2) cycles, FP64 residual/update/coarsest",
                     "bf16": "mixed-precision refinement: inner V(2,2) cycles on BF16 storage with FP32 "
                             "arithmetic, FP64 residual/update/coarsest"}[head],
            "cycles": res[head]["stats"]["cycles"],
            "outer_iters": res[head]["stats"]["outer_iters"],
            "rel_res": res[head]["stats"]["rel_res"],
            "plain_fp64_dofs_per_s": res["fp64"]["dofs_per_s"],
            "plain_fp64_cycles": res["fp64"]["stats"]["cycles"],
            "plain_fp64_ms_per_solve": 1e3 * res["fp64"]["seconds"] / args.steps,
            "fp32_mixed_dofs_per_s": res["fp32"]["dofs_per_s"],
            "fp32_mixed_cycles": res["fp32"]["stats"]["cycles"],
            "fp32_mixed_outer_iters": res["fp32"]["stats"]["outer_iters"],
            "bf16_mixed_dofs_per_s": res["bf16"]["dofs_per_s"],
            "bf16_mixed_cycles": res["bf16"]["stats"]["cycles"],
            "bf16_mixed_outer_iters": res["bf16"]["stats"]["outer_iters"],
            "mixed_over_plain": res[head]["dofs_per_s"] / res["fp64"]["dofs_per_s"],
        },
        "roofline": {
            "kernel": {"sweep": "k_sweep2z: two weighted-Jacobi sweeps of a nonzero iterate in one pass, "
                                "finest level (z-marching)",
                       "sweep_zero": "k_sweep3: first two sweeps from a zero iterate, finest level",
                       "restrict": "k_restrict3: residual + restriction, finest level",
                       "prolong": "k_prolong3: prolongation + correction, finest level",
                       "refine": "k_ir_resid3: FP64 update + residual of the refinement",
                       "fused_down": "k_down2z2: two sweeps of a nonzero iterate + residual + restriction "
                                     "in one pass, finest level (z-marching)",
                       "fused_down_zero": "k_down0z1: two sweeps from zero + residual + restriction in one "
                                          "pass, finest level (z-marching)",
                       "fused_up": "k_sweep2z: prolongation + correction and two sweeps in one pass, "
                                   "finest level (z-marching)"}[dom] +
                      (" (%s correction and residual, %s per thread)" % (
                          head.upper(), "two cells" if B.np_get_tuning("ir_cpt") == 2 else "one cell")
                       if dom == "refine" else
                       " (%s storage, two cells per thread)" % head.upper()),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom, head),
            "avg_us": avg_us,
            "bytes_per_launch": nbytes,
            "timing": "HIP events around each launch of the kernel in the timed solves, on the library stream",
            "copy_measured_gbs": copy_gbs,
            "finest_level_live": level_live,
            "level0_kernels_event_bracketed": {p: res[p]["prof"] for p in res},
        },
        "cpu_baseline": None,
    }
    line["config"]["error_vs_fp64_oracle"] = None
    if not args.no_cpu:
        log("timing the oracle on the host ...")
        line["cpu_baseline"], line["config"]["error_vs_fp64_oracle"] = cpu_baseline(f, h, gpu_x)
        log("  oracle: %.3g DOF/s on %d threads; error vs oracle %s" % (
            line["cpu_baseline"]["value"], line["cpu_baseline"]["cores"],
            {k: v for k, v in line["config"]["error_vs_fp64_oracle"].items() if k in gpu_x}))
    del gpu_x
    legs = [l for l in args.legs.split(",") if l]
    others = {}
    for leg in legs:
        log("workload %s ..." % leg)
        if leg == "c1":
            others["c1"] = leg_c1(B, inputs, args.steps, args.warmup)
        elif leg == "c2":
            others["c2"] = leg_c2(B, inputs)
        elif leg == "c4":
            others["c4"] = leg_c4(B, inputs, max(1, args.steps // 3), 1)
        elif leg == "c5":
            others["c5"] = leg_c5(B, inputs)
        elif leg == "sawtooth":
            others["sawtooth"] = leg_sawtooth(B, inputs, args.steps, args.warmup)
        elif leg == "ad":
            others["ad"] = leg_ad(B, inputs, args.steps, args.warmup)
        elif leg == "c5_zero":  # the 3D projection steps from zero only (kernel profiles)
            others["c5_zero"] = leg_c5_zero(B, inputs)
        elif leg == "ad_large":  # the large advection-diffusion solves only (kernel profiles)
            others["ad_large"] = ad_large(B, inputs, args.steps, args.warmup)
        elif leg == "explicit":
            others["explicit"] = leg_explicit(B, inputs, args.steps, args.warmup)
        elif leg == "collocated":
            others["collocated"] = leg_collocated(B, inputs)
        else:
            sys.exit("unknown leg %s" % leg)
        B.np_release_all()
        torch.cuda.empty_cache()
    if others:
        line["workloads"] = others
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
