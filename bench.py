#!/usr/bin/env python3
"""Benchmark of the rigid-multiblob mobility solver on one MI355X.

Timed step (the whole hot path, inputs resident in HBM): one mobility solve
of 1000 x 15-blob boomerangs above a no-slip wall (15,000 blobs), right-
preconditioned GMRES with the block-diagonal preconditioner, FP32-pair
products inside FP64 iterative refinement to an FP64 relative residual of
1e-8 with the body velocities' error also bounded by 1e-8 (the solver
tightens its residual target by the error amplification it measures).
`value` = blob-pair interactions evaluated per second over the timed solves
(every FP32 and FP64 mobility product counts Nb^2 pairs).

Also reported (outside the timed region): the plain FP64 solve of the same
system; the 196,608-blob monolayer mobility product in both precisions; a
serving run of 256 wall-bounded requests (Poisson arrivals at 50/s, p50/p99
latency, and the saturated solves/s against the same requests solved one at
a time in plain FP64); the roofline of the dominant kernel (FP32 wall pair
kernel) from HIP events recorded around its launches; and the CPU oracle's
pair rate on a bounded sample.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Flop counts of the pair arithmetic (FMA = 2, add/mul = 1, reciprocal
# square root = 1, compares/selects/conversions = 0), counted once from the
# first implemented form of each kernel and held fixed as the unit of work
# (the current forms execute fewer: lengths in units of a, shared wall
# polynomials):
#  one-sided kernel, per ordered pair;
#  symmetric kernel, per unordered off-diagonal pair (coefficients once, both
#  contractions) and per ordered pair of its diagonal tiles.
FLOPS_PER_PAIR = {"pair_f32_wall": 130, "pair_f32_free": 42, "pair_f64_wall": 145, "pair_f64_free": 50}
FLOPS_SYM = {"pair_f32_wall": (155, 122), "pair_f32_free": (60, 42), "pair_f64_wall": (171, 138),
             "pair_f64_free": (68, 50)}


def product_flops(rmb, kernel, nb):
    """Algorithmic flops of one mobility product of nb blobs."""
    sym, blk = rmb.pair_plan(nb)
    if not sym:
        return FLOPS_PER_PAIR[kernel] * nb * nb
    sizes = [blk] * (nb // blk) + ([nb % blk] if nb % blk else [])
    diag = sum(b * b for b in sizes)
    off = (nb * nb - diag) // 2
    f_off, f_diag = FLOPS_SYM[kernel]
    return f_off * off + f_diag * diag
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}  # MI355X published vector peaks
METRIC = "blob-pair interactions/s (wall RPY matvec); solves/s + p50/p99 latency @1e-8 vs FP64"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM traffic of the dominant kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs scaled by the same counters on a plain copy of known size.  It is
# reported only while the kernel source still hashes to what was profiled.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_sym_f32_wall_boomerangs15000_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1602_02170_amd", "csrc", f)
                  for f in ("rmb_pair_sym.hip", "rmb_common.h")]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, None
    if t.get("source_sha256") != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    return t["hbm_bytes_per_launch"], t


def copy_calibration(torch, mib):
    """A plain device copy of `mib` MiB, three times (reference for the
    FETCH_SIZE / WRITE_SIZE counters: each dispatch reads and writes exactly
    mib MiB)."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"  copy calibration: 3 x {mib} MiB device-to-device copies")


def solve_leg(rmb, torch, ctx, sysd, FT, precision, steps, warmup, tol=1e-8, u_tol=1e-8):
    for _ in range(warmup):
        rmb.solve_mobility(ctx, sysd, FT, tol=tol, u_tol=u_tol, precision=precision)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, _, info = rmb.solve_mobility(ctx, sysd, FT, tol=tol, u_tol=u_tol, precision=precision)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = {k: ctx.kernel_time(k) for k in ("pair_f32_wall", "pair_f64_wall")}
    ctx.set_timing(False)
    return dt, infos, kt


def matvec_leg(rmb, torch, ctx, S, reps=20):
    """Wall mobility products of prefixes of the 128 x 128 icosahedron
    monolayer (1024 ... 16384 bodies, 12,288 ... 196,608 blobs): median of
    `reps` launches after a warm-up, each launch timed with its own events.
    The FP32 leg takes float32 forces and returns float32 velocities
    (rmb_mobility_matvec_f32), the FP64 leg float64 ones."""
    res = {"workload": "wall RPY mobility product, 16384 x 12-blob icosahedra monolayer (196,608 blobs) and "
                       "prefixes of it", "forces": {"fp32": "float32 in, float32 out", "fp64": "float64"},
           "sweep": []}
    for n_bodies in (1024, 2048, 4096, 8192, 16384):
        sus, lam = S.icosahedra_monolayer(n_bodies=n_bodies)
        sysd = rmb.System.from_suspension(sus)
        lt = torch.tensor(lam, dtype=torch.float64, device="cuda")
        out = torch.empty_like(lt)
        lt32 = torch.tensor(lam.astype(np.float32), device="cuda")
        out32 = torch.empty_like(lt32)
        row = {"n_blobs": sus.n_blobs}
        for prec in ("fp32", "fp64"):
            def product():
                if prec == "fp32":
                    rmb.mobility_matvec_f32(ctx, sysd, lt32, out32)
                else:
                    rmb.mobility_matvec(ctx, sysd, lt, prec, out)
            product()
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for e0, e1 in ev:
                e0.record()
                product()
                e1.record()
            torch.cuda.synchronize()
            ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
            k = "pair_f32_wall" if prec == "fp32" else "pair_f64_wall"
            row[f"{prec}_ms"] = round(ms, 4)
            row[f"{prec}_pairs_per_s"] = sus.n_blobs ** 2 / (ms * 1e-3)
            row[f"{prec}_tflops"] = product_flops(rmb, k, sus.n_blobs) / (ms * 1e-3) / 1e12
            log(f"  matvec {sus.n_blobs} blobs {prec}: {ms:.3f} ms, {row[f'{prec}_pairs_per_s']:.3e} pairs/s, "
                f"{row[f'{prec}_tflops']:.1f} TFLOP/s")
        res["sweep"].append(row)
        del lt, out, lt32, out32
    full = res["sweep"][-1]
    for k in ("fp32_ms", "fp32_pairs_per_s", "fp32_tflops", "fp64_ms", "fp64_pairs_per_s", "fp64_tflops"):
        res[k] = full[k]
    return res


def flow_leg(rmb, torch, ctx, S, reps=5):
    """Flow field of the 16384 x 12-blob monolayer (appendix on computing
    flow fields): every blob split into 12 tracer blobs (radius a/10) on a
    sphere of radius 0.4 a, i.e. 2,359,296 sources, evaluated on a 128 x 128
    plane of points at z = 2.5.  One-sided pair kernel; median of `reps`
    calls, each timed with its own events, plus the pair kernel's own
    event-timed share."""
    sus, lam = S.icosahedra_monolayer()
    u = S.icosahedron()
    offs = 0.4 * u / np.linalg.norm(u, axis=1, keepdims=True)
    lo, hi = sus.pos[:, :2].min(0), sus.pos[:, :2].max(0)
    gx, gy = np.meshgrid(np.linspace(lo[0], hi[0], 128), np.linspace(lo[1], hi[1], 128))
    T = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 2.5)], 1)
    sysd = rmb.System.from_suspension(sus)
    lt = torch.tensor(lam, dtype=torch.float64, device="cuda")
    tt = torch.tensor(T, dtype=torch.float64, device="cuda")
    out = torch.empty_like(tt)
    ns, nt = sus.n_blobs * len(offs), len(T)
    res = {"workload": f"flow field, {sus.n_blobs} wall blobs x {len(offs)} tracer blobs = {ns} sources, "
                       f"{nt} targets", "pairs": ns * nt}
    for prec in ("fp32", "fp64"):
        k = "pair_f32_wall" if prec == "fp32" else "pair_f64_wall"
        rmb.flow_field(ctx, sysd, lt, offs, 0.1 * sus.a, tt, prec, out)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record()
            rmb.flow_field(ctx, sysd, lt, offs, 0.1 * sus.a, tt, prec, out)
            e1.record()
        torch.cuda.synchronize()
        kms, kn = ctx.kernel_time(k)
        ctx.set_timing(False)
        ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
        kavg = kms / max(kn, 1)
        tf = FLOPS_PER_PAIR[k] * ns * nt / (kavg * 1e-3) / 1e12
        res[prec] = {"ms": round(ms, 3), "pairs_per_s": ns * nt / (ms * 1e-3), "kernel_ms": round(kavg, 3),
                     "kernel_tflops": round(tf, 2), "kernel_frac": round(tf / PEAK_TFLOPS[prec], 4)}
        log(f"  flow field {prec}: {ms:.2f} ms per call, pair kernel {kavg:.2f} ms, {tf:.1f} TFLOP/s "
            f"({tf / PEAK_TFLOPS[prec]:.1%} of peak)")
    return res


def factor_leg(rmb, torch, ctx, S, reps=3):
    """Batched per-body factorisation: 512 x 162-blob shells above the wall
    (486 x 486 blocks, padded to 512), all blocks in one launch, then the
    preconditioner applied to 8 right-hand sides."""
    sus, rhs = S.shells_wall()
    sysd = rmb.System.from_suspension(sus)
    r = torch.tensor(rhs, dtype=torch.float64, device="cuda")
    pc = rmb.Precond(ctx, sysd)  # first build also tunes the panel width
    pc.close()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        pc = rmb.Precond(ctx, sysd)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
        if _ < reps - 1:
            pc.close()
    out = pc.apply(r)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pc.apply(r, out)
    e1.record()
    torch.cuda.synchronize()
    apply_ms = e0.elapsed_time(e1) / reps
    pc.close()
    Mp = 512
    m = 3 * 162  # the method's block size; the padding to Mp is not counted
    flops = sus.n_bodies * (m ** 3 / 3 + 6 * m ** 2 + 36 * m)  # Cholesky + L^-1 K + Y^T Y
    ms = min(ts) * 1e3
    res = {"workload": "512 x 162-blob shells (486 x 486 wall-RPY blocks, padded to 512): assembly, Cholesky, "
                       "L^-1 K, Schur factor; apply to 8 right-hand sides",
           "flops": flops, "flops_counted": "per body m^3/3 + 6 m^2 + 36 m with m = 486 (padding not counted)",
           "factor_ms": ms, "factor_tflops": flops / (ms * 1e-3) / 1e12,
           "factor_frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"],
           "apply_8rhs_ms": apply_ms, "panel_width": ctx.tuned_panel(Mp),
           "autotune": [t for t in ctx.tune_log() if t["padded_dim"] == Mp]}
    log(f"  batched factor: {ms:.2f} ms ({res['factor_tflops']:.2f} TFLOP/s), apply 8 rhs {apply_ms:.2f} ms, "
        f"panel width {res['panel_width']}")
    for t in res["autotune"]:
        log(f"    shape panel {t['panel']} row tiles {t['row_tiles']} chunk {t['chunk']}: {t['ms']:.2f} ms"
            f"{'  (chosen)' if t['chosen'] else ''}")
    return res


def shared_leg(rmb, torch, ctx, S, reps=5):
    """One factorisation per reference shape, rotated per body (free-space
    blocks; for these wall problems the approximate preconditioner that
    neglects the wall): (1) the 512 x 162-blob shells, factor and apply to 8
    right-hand sides; (2) the 1000-boomerang solve to 1e-8 (FP32 pairs, FP64
    refinement) with prebuilt shared blocks, against the wall blocks built
    inside every solve."""
    res = {}
    sus, rhs = S.shells_wall()
    sysd = rmb.System.from_suspension(sus)
    shell = S.sphere_shell(162)
    shapes = [shell - shell.mean(axis=0)]
    idx = np.zeros(sus.n_bodies, np.int32)
    qd = torch.tensor(sus.quat, dtype=torch.float64, device="cuda")
    r = torch.tensor(rhs, dtype=torch.float64, device="cuda")
    ts = []
    for k in range(reps):
        t = time.perf_counter()
        pc = rmb.Precond.from_shapes(ctx, sysd, shapes, idx, qd)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
        if k < reps - 1:
            pc.close()
    out = pc.apply(r)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pc.apply(r, out)
    e1.record()
    torch.cuda.synchronize()
    pc.close()
    res["shells"] = {"factor_ms": min(ts) * 1e3, "apply_8rhs_ms": e0.elapsed_time(e1) / reps}
    log(f"  shared shells: factor {res['shells']['factor_ms']:.3f} ms, apply 8 rhs "
        f"{res['shells']['apply_8rhs_ms']:.3f} ms")

    sus = S.boomerangs_wall()
    sysd = rmb.System.from_suspension(sus)
    boo = S.boomerang()
    qd = torch.tensor(sus.quat, dtype=torch.float64, device="cuda")
    FT = torch.tensor(sus.FT, dtype=torch.float64, device="cuda")
    t = time.perf_counter()
    pc = rmb.Precond.from_shapes(ctx, sysd, [boo - boo.mean(axis=0)], np.zeros(sus.n_bodies, np.int32), qd)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t) * 1e3
    rmb.solve_mobility(ctx, sysd, FT, precond=pc, tol=1e-8, precision="fp32")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        _, _, info = rmb.solve_mobility(ctx, sysd, FT, precond=pc, tol=1e-8, precision="fp32")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) / reps * 1e3
    _, _, iw = rmb.solve_mobility(ctx, sysd, FT, tol=1e-8, precision="fp32")
    pc.close()
    res["boomerangs"] = {"build_ms": build_ms, "ms_per_solve": ms, "iterations": info["iterations"],
                         "iterations_wall_blocks": iw["iterations"], "rel_residual": info["rel_residual"],
                         "status": info["status"]}
    log(f"  shared boomerangs: build {build_ms:.2f} ms, solve {ms:.2f} ms, {info['iterations']} iterations "
        f"({iw['iterations']} with the wall blocks)")
    return res


def resistance_leg(rmb, torch, ctx, S, reps=3):
    """Resistance problem (M lambda = K U, F = K^T lambda) on the
    1000-boomerang suspension with seeded random body velocities, FP32 pairs
    with FP64 refinement to 1e-8; the mobility solve's iteration count on the
    same system for comparison."""
    sus = S.boomerangs_wall()
    sysd = rmb.System.from_suspension(sus)
    U = torch.tensor(np.random.default_rng(8).standard_normal((sus.n_bodies, 6)), dtype=torch.float64,
                     device="cuda")
    rmb.solve_resistance(ctx, sysd, U, tol=1e-8, precision="fp32")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        _, _, info = rmb.solve_resistance(ctx, sysd, U, tol=1e-8, precision="fp32")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) / reps * 1e3
    res = {"workload": "resistance problem, 1000 x 15-blob boomerangs, random U, FP32 pairs + FP64 refinement "
                       "to 1e-8", "ms_per_solve": ms, "iterations": info["iterations"],
           "fp32_products": info["matvecs_fp32"], "fp64_products": info["matvecs_fp64"],
           "rel_residual": info["rel_residual"], "status": info["status"]}
    log(f"  resistance solve: {ms:.2f} ms, {info['iterations']} iterations")
    return res


def serving_leg(rmb, torch, ctx, S, n_req, rate, precision="fp32", extra_precisions=("relaxed",)):
    t_gen = time.perf_counter()
    reqs = [S.mixed_wall_request(i) for i in range(n_req)]
    arrivals = S.poisson_arrivals(n_req, rate)
    systems = [rmb.System.from_suspension(r) for r in reqs]
    FTs = [torch.tensor(r.FT, dtype=torch.float64, device="cuda") for r in reqs]
    torch.cuda.synchronize()
    nb = np.array([r.n_blobs for r in reqs])
    log(f"  serving: generated {n_req} requests ({nb.sum()} blobs, max {nb.max()}) "
        f"in {time.perf_counter() - t_gen:.1f}s")
    opts = dict(tol=1e-8, u_tol=1e-8, precision=precision)
    # warm-up of the server path
    srv = rmb.Server(ctx)
    srv.submit(0, systems[0], FTs[0], **opts)
    while not srv.poll():
        srv.step()
    srv.close()

    def run(arr, opts=opts):
        srv = rmb.Server(ctx)
        done = {}
        nxt = 0
        t0 = time.perf_counter()
        ticks = 0
        while len(done) < n_req:
            now = time.perf_counter() - t0
            while nxt < n_req and arr[nxt] <= now:
                srv.submit(nxt, systems[nxt], FTs[nxt], **opts)
                nxt += 1
            a, q = srv.step()
            ticks += 1
            for tag, U, lam, info in srv.poll():
                done[tag] = (time.perf_counter() - t0, info)
            if a == 0 and q == 0 and nxt < n_req:
                time.sleep(max(0.0, arr[nxt] - (time.perf_counter() - t0)))
        srv.close()
        comp = np.array([done[i][0] for i in range(n_req)])
        infos = [done[i][1] for i in range(n_req)]
        return comp, infos, ticks

    comp, infos, ticks = run(arrivals)
    lat = comp - arrivals
    ok = sum(1 for i in infos if i["status"] == 0 and i["rel_residual"] <= 1e-8)
    res = {
        "workload": f"{n_req} wall suspensions, 10-4000 mixed icosahedra/boomerangs, Poisson {rate:g}/s, "
                    f"{'FP32 pairs + FP64 refinement' if precision == 'fp32' else 'relaxed-precision GMRES'} to a "
                    f"relative residual of 1e-8 with the velocity error bounded by 1e-8",
        "precision": precision,
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "solves_per_s": n_req / (comp.max() - arrivals.min()),
        "converged": ok,
        "ticks": ticks,
    }
    log(f"  serving Poisson: p50 {res['p50_latency_ms']:.1f} ms p99 {res['p99_latency_ms']:.1f} ms, "
        f"{res['solves_per_s']:.1f} solves/s, {ok}/{n_req} converged")
    comp_sat, infos_sat, _ = run(np.zeros(n_req))
    res["saturated_solves_per_s"] = n_req / comp_sat.max()
    res["u_err_est_max"] = max(i["u_err_est"] for i in infos_sat)
    for p in extra_precisions:
        c, inf, _ = run(np.zeros(n_req), dict(opts, precision=p))
        res[f"saturated_solves_per_s_{p}"] = n_req / c.max()
        log(f"  serving saturated, {p}: {n_req / c.max():.1f} solves/s")
    # plain FP64 GPU path, unbatched: the same requests one at a time
    torch.cuda.synchronize()
    service = np.zeros(n_req)
    for i in range(n_req):
        t = time.perf_counter()
        rmb.solve_mobility(ctx, systems[i], FTs[i], tol=1e-8, u_tol=1e-8, precision="fp64")
        torch.cuda.synchronize()
        service[i] = time.perf_counter() - t
    res["fp64_unbatched_solves_per_s"] = n_req / service.sum()
    # the same Poisson stream through a FIFO of one-at-a-time FP64 solves
    fin = np.zeros(n_req)
    tcur = 0.0
    for i in range(n_req):
        tcur = max(tcur, arrivals[i]) + service[i]
        fin[i] = tcur
    lat64 = fin - arrivals
    res["fp64_unbatched_p50_latency_ms"] = float(np.percentile(lat64, 50) * 1e3)
    res["fp64_unbatched_p99_latency_ms"] = float(np.percentile(lat64, 99) * 1e3)
    res["speedup_vs_fp64_unbatched"] = res["saturated_solves_per_s"] / res["fp64_unbatched_solves_per_s"]
    log(f"  serving saturated: {res['saturated_solves_per_s']:.1f} solves/s; FP64 unbatched "
        f"{res['fp64_unbatched_solves_per_s']:.1f} solves/s (x{res['speedup_vs_fp64_unbatched']:.2f})")
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(S, sus):
    """The CPU oracle solving the same system (plain FP64 GMRES with the
    block-diagonal preconditioner, FP64 Kahan-summed pair products): blob-pair
    interactions evaluated per second over the whole solve."""
    import oracle
    calls = [0]

    def apply_A(v):
        calls[0] += 1
        return oracle.saddle_apply(sus, v)

    t = time.perf_counter()
    P = oracle.BlockPreconditioner(sus)
    b = oracle.rhs(sus, sus.FT, None)
    _, it, hist = oracle.gmres(apply_A, P.apply, b, tol=1e-8, restart=100, maxiter=1000)
    dt = time.perf_counter() - t
    pairs = calls[0] * sus.n_blobs ** 2
    return {"value": pairs / dt, "unit": "blob-pair interactions/s", "cores": oracle.num_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"the oracle's full FP64 solve of the same 1000-boomerang system to 1e-8: {it} iterations, "
                      f"{calls[0]} products of {sus.n_blobs}^2 pairs, {dt:.1f} s",
            "other_workloads": _cpu_other_workloads(S, oracle)}


def _cpu_other_workloads(S, oracle):
    """Part of the CPU-baseline leg: the oracle on bounded samples of the
    other workloads, beside the GPU figures: the product over a 24,576-blob
    prefix of the 196,608-blob monolayer, and a few small requests of the
    serving stream solved one at a time (FP64 GMRES to 1e-8)."""
    mono, lam = S.icosahedra_monolayer()
    n = 24576  # a prefix of the monolayer, one of the GPU sweep's sizes
    t = time.perf_counter()
    oracle.matvec(mono.pos[:n], lam[:n], mono.a, mono.eta, mono.wall)
    dtm = time.perf_counter() - t
    ids = [0, 1, 8, 9]
    reqs = [S.mixed_wall_request(i) for i in ids]
    t = time.perf_counter()
    for r in reqs:
        oracle.solve_mobility(r, r.FT, tol=1e-8)
    dts = time.perf_counter() - t
    nb = [r.n_blobs for r in reqs]
    return {
        "c3_matvec": {"value": n * n / dtm, "unit": "blob-pair interactions/s",
                      "cores": oracle.num_threads(), "kind": "oracle",
                      "sample": f"the full FP64 wall product over the first {n} blobs of the {mono.n_blobs}-blob "
                                f"monolayer, {dtm:.2f} s"},
        "c5_serial": {"value": len(reqs) / dts, "unit": "solves/s", "cores": oracle.num_threads(), "kind": "oracle",
                      "sample": f"requests {ids} of the serving stream ({min(nb)}-{max(nb)} blobs) solved one at a "
                                f"time, {dts:.2f} s"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--no-matvec", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-factor", action="store_true")
    ap.add_argument("--no-flow", action="store_true")
    ap.add_argument("--prewarm", type=int, default=300, help="untimed products before anything is timed")
    ap.add_argument("--serve-precision", default="fp32", choices=["fp32", "relaxed"])
    ap.add_argument("--serve-budget-gib", type=int, default=0, help="server context budget (0: 16 GiB)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-step", action="store_true", help="timed solves only (for profiling)")
    ap.add_argument("--only-factor", action="store_true",
                    help="the batched large-body factorisation leg only (for profiling); prints its results")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the mobility product would shard "
              "by target rows with one all-gather of lambda per product); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1602_02170_amd as rmb
    import suspensions as S

    ctx = rmb.Context(0)
    if args.only_factor:
        res = factor_leg(rmb, torch, ctx, S)
        if args.calib_copy:
            copy_calibration(torch, args.calib_copy)
        ctx.close()
        print(json.dumps({"batched_factor": res}), flush=True)
        return
    sus = S.boomerangs_wall()
    sysd = rmb.System.from_suspension(sus)
    FT = torch.tensor(sus.FT, dtype=torch.float64, device="cuda")
    nb = sus.n_blobs
    log(f"workload: {sus.name}, {nb} blobs")

    # bring the GPU clocks up before anything is timed: the first ~100
    # products of a fresh process run up to 15% slower (about 0.1 s here)
    lam_w = torch.ones((nb, 3), dtype=torch.float64, device="cuda")
    vel_w = torch.empty_like(lam_w)
    for _ in range(args.prewarm):
        rmb.mobility_matvec(ctx, sysd, lam_w, "fp32", vel_w)
    torch.cuda.synchronize()
    del lam_w, vel_w

    dt, infos, kt = solve_leg(rmb, torch, ctx, sysd, FT, "fp32", args.steps, args.warmup)
    pairs = sum((i["matvecs_fp32"] + i["matvecs_fp64"]) * nb * nb for i in infos)
    bad = [i for i in infos if i["status"] != 0 or i["rel_residual"] > 1e-8 or not 0 < i["u_err_est"] <= 1e-8]
    value = pairs / dt
    ms_step = dt / args.steps * 1e3
    log(f"  refined solve: {ms_step:.2f} ms/solve, {value:.3e} pairs/s, iterations "
        f"{infos[-1]['iterations']}, fp32/fp64 products {infos[-1]['matvecs_fp32']}/{infos[-1]['matvecs_fp64']}, "
        f"internal tol {infos[-1]['tol_internal']:.2e}, velocity error estimate {infos[-1]['u_err_est']:.2e}")
    k_ms, k_n = kt["pair_f32_wall"]
    avg_ms = k_ms / max(k_n, 1)
    flops = product_flops(rmb, "pair_f32_wall", nb)
    achieved = flops / (avg_ms * 1e-3) / 1e12
    sym, blk = rmb.pair_plan(nb)
    roofline = {"bound": "alu", "kernel": f"pair_sym_kernel<f32, B={blk}, wall>" if sym else "pair_f32_kernel<wall>",
                "achieved": achieved, "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS["fp32"], "traffic": None,
                "flops_per_launch": flops, "interactions_per_launch": nb * nb, "avg_launch_ms": avg_ms,
                "launches": k_n}
    log(f"  pair f32 wall kernel ({'symmetric B=%d' % blk if sym else 'one-sided'}): {avg_ms:.4f} ms avg "
        f"over {k_n} launches, {achieved:.1f} TFLOP/s")
    traffic, detail = measured_traffic()
    roofline["traffic"] = traffic
    if isinstance(detail, dict):
        roofline["traffic_detail"] = {k: detail[k] for k in ("fetch_bytes_per_launch", "write_bytes_per_launch",
                                                              "copy_factor_fetch", "copy_factor_write", "profile")}
    elif detail:
        roofline["traffic_detail"] = detail
    if args.calib_copy:
        copy_calibration(torch, args.calib_copy)

    line = {"metric": METRIC, "value": value, "unit": "blob-pair interactions/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 pairs, f32 sums over each group of 64 sources, f64 accumulation across groups and "
                     "tiles, f64 residual/refinement",
            "data": "synthetic (seeded boomerang suspension; no dataset)",
            "config": {"workload": "wall RPY mobility solve, 1000 x 15-blob boomerangs (15,000 blobs), "
                                   "block-diagonal preconditioned GMRES, FP32 pairs + FP64 refinement to "
                                   "FP64 relative residual 1e-8 and velocity error 1e-8",
                       "n_blobs": nb, "n_bodies": sus.n_bodies, "tol": 1e-8, "u_tol": 1e-8,
                       "parallelism": "single GPU"},
            "roofline": roofline,
            "solve": {"ms_per_solve": ms_step, "solves_per_s": 1e3 / ms_step,
                      "iterations": infos[-1]["iterations"], "fp32_products": infos[-1]["matvecs_fp32"],
                      "fp64_products": infos[-1]["matvecs_fp64"], "rel_residual": infos[-1]["rel_residual"],
                      "tol_internal": infos[-1]["tol_internal"], "gamma": infos[-1]["gamma"],
                      "u_err_est": infos[-1]["u_err_est"], "failed": len(bad)}}
    if not args.only_step:
        dt64, infos64, kt64 = solve_leg(rmb, torch, ctx, sysd, FT, "fp64", args.steps, 1)
        ms64 = dt64 / args.steps * 1e3
        line["solve"]["fp64_ms_per_solve"] = ms64
        line["solve"]["fp64_iterations"] = infos64[-1]["iterations"]
        line["solve"]["fp64_tol_internal"] = infos64[-1]["tol_internal"]
        line["solve"]["speedup_vs_fp64"] = ms64 / ms_step
        k64 = kt64["pair_f64_wall"]
        line["solve"]["pair_f64_wall_avg_launch_ms"] = k64[0] / max(k64[1], 1)
        log(f"  plain FP64 solve: {ms64:.2f} ms/solve ({infos64[-1]['iterations']} iterations)")
        dtr, infosr, _ = solve_leg(rmb, torch, ctx, sysd, FT, "relaxed", args.steps, 1)
        msr = dtr / args.steps * 1e3
        line["solve"]["relaxed"] = {"ms_per_solve": msr, "iterations": infosr[-1]["iterations"],
                                    "fp32_products": infosr[-1]["matvecs_fp32"],
                                    "fp64_products": infosr[-1]["matvecs_fp64"],
                                    "rel_residual": infosr[-1]["rel_residual"],
                                    "failed": len([i for i in infosr if i["status"] != 0 or i["rel_residual"] > 1e-8])}
        log(f"  relaxed-precision solve: {msr:.2f} ms/solve ({infosr[-1]['iterations']} iterations, fp32/fp64 "
            f"products {infosr[-1]['matvecs_fp32']}/{infosr[-1]['matvecs_fp64']})")
        # the residual bound alone (no velocity bound), as the paper's solves stop
        res_only = {}
        for p in ("fp32", "fp64"):
            d, inf, _ = solve_leg(rmb, torch, ctx, sysd, FT, p, args.steps, 1, u_tol=0.0)
            res_only[p] = {"ms_per_solve": d / args.steps * 1e3, "iterations": inf[-1]["iterations"]}
        line["solve"]["residual_only"] = res_only
        log(f"  residual bound only: fp32 {res_only['fp32']['ms_per_solve']:.2f} ms, fp64 "
            f"{res_only['fp64']['ms_per_solve']:.2f} ms")
        if not args.no_matvec:
            line["matvec"] = matvec_leg(rmb, torch, ctx, S)
        line["resistance"] = resistance_leg(rmb, torch, ctx, S)
        if not args.no_flow:
            line["flow_field"] = flow_leg(rmb, torch, ctx, S)
        if not args.no_factor:
            line["batched_factor"] = factor_leg(rmb, torch, ctx, S)
            line["shared_precond"] = shared_leg(rmb, torch, ctx, S)
        if not args.no_serving:
            sctx = rmb.Context(0, args.serve_budget_gib << 30) if args.serve_budget_gib else ctx
            line["serving"] = serving_leg(rmb, torch, sctx, S, args.requests, args.rate, args.serve_precision)
            line["serving"]["device_budget_gib"] = args.serve_budget_gib or 16
            if sctx is not ctx:
                sctx.close()
        if not args.no_cpu:
            line["cpu_baseline"] = cpu_baseline(S, sus)
            log(f"  cpu oracle: {line['cpu_baseline']['value']:.3e} pairs/s on {line['cpu_baseline']['cores']} threads")
            ow = line["cpu_baseline"]["other_workloads"]
            log(f"  cpu oracle, other workloads: monolayer prefix {ow['c3_matvec']['value']:.3e} pairs/s; "
                f"small requests {ow['c5_serial']['value']:.2f} solves/s")
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
