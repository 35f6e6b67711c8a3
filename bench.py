#!/usr/bin/env python
"""Benchmark: FMM-BEM matrix-vector products per second on one MI355X.

Workload: the L-shaped room (boxes 6x5x3 m and 4x3x3 m) with a 7 cm baffle slab and a 1x2 m
doorway patch (beta = 1), f = 2.5 kHz (k = 45.8 1/m), meshed at 1.908 cm (N = 1,009,576 flat
triangles), per-face admittance beta ~ U[0.05, 0.3]; direct BIE (Eq. dbem4).  One step is one
full FMM matrix-vector product A x (densities, P2P + near table, P2M, M2M, M2L, L2L, L2P +
combine) on a seeded complex vector already resident in HBM.

Also reported: the roofline position of the dominant kernel (device time from HIP events on the
library stream over the timed region), the time of flexible GMRES to relative residual 1e-4,
and the CPU oracle timed on a bounded sample of rows (whose values also check the GPU product).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"fp64": 78.6e12, "fp32": 157.3e12, "hbm": 8.0e12}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_lroom_1M_fp64.json")
# tile shapes of the run whose counters TRAFFIC_FILE holds: replayed by default on that workload, so
# that the timed launches are the counted ones (the autotuner's near ties may fall either way)
SHAPES_FILE = os.path.join(ROOT, "profiles", "tile_shapes_lroom_1M_fp64.json")


def measured_traffic(kernel, launches_per_product):
    """HBM bytes per launch of `kernel` from the committed counter summary (two rocprofv3 --pmc
    passes, calibrated on a device copy), or None when the summary is missing, the sources it
    was taken with have changed since, or its run put a different number of batches on the
    kernel (the tile-shape autotuner chose otherwise there), so that a launch there is not the
    launch timed here."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    for fn, digest in t.get("source_sha256", {}).items():
        with open(os.path.join(ROOT, "paper_2103_16073_amd", "csrc", fn), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != digest:
                return None
    for name, v in t.get("kernels", {}).items():
        if name.replace("<1>", "") == kernel:
            if abs(v.get("launches_per_product", -1) - launches_per_product) > 1e-9:
                return None
            return v["hbm_bytes_per_launch"]
    return None


# kernels whose arithmetic runs on the matrix cores (the others use the vector ALUs)
MFMA_KERNELS = ("k_tq_rcr", "k_tq_lds", "k_tf_trans", "k_tm_")


def kernel_roofline(st, steps, counted):
    """Roofline position of one kernel class from the library's per-launch algorithmic work: the
    method's flops (rotation, coaxial step and back rotation of every translation job; pair kernel
    evaluations) and its compulsory HBM bytes (each distinct input expansion and table once, targets
    once).  The bound is the one the kernel's intensity (flops / compulsory bytes) reaches first
    against the FP64 ridge point (peak FP64 flops / peak HBM bandwidth); achieved = the bound's
    quantity per launch / the average launch time (HIP events on the launch's own stream).
    `traffic` is the measured HBM bytes per launch (committed counter summary) when those counters
    were taken on these very launches; its excess over the compulsory bytes is what the
    implementation adds (work rows between kernels, re-reads)."""
    avg_s = st["ms"] / st["launches"] * 1e-3
    fl = st["flops"] / st["launches"]
    by = st["bytes"] / st["launches"]
    ridge = PEAKS["fp64"] / PEAKS["hbm"]
    intensity = fl / by if by > 0 else float("inf")
    if intensity >= ridge:
        bound = "mfma" if st["name"].startswith(MFMA_KERNELS) else "alu"
        rl = {"kernel": st["name"], "bound": bound, "achieved": fl / avg_s / 1e12, "peak": PEAKS["fp64"] / 1e12,
              "unit": "TFLOP/s", "frac": fl / avg_s / PEAKS["fp64"]}
    else:
        rl = {"kernel": st["name"], "bound": "hbm", "achieved": by / avg_s / 1e9, "peak": PEAKS["hbm"] / 1e9,
              "unit": "GB/s", "frac": by / avg_s / PEAKS["hbm"]}
    traffic = measured_traffic(st["name"], st["launches"] / steps) if counted else None
    rl.update({"traffic": traffic,
               "traffic_GBps": None if traffic is None else traffic / avg_s / 1e9,
               "traffic_over_compulsory": None if traffic is None else traffic / by,
               "algorithmic_flops_per_launch": fl, "compulsory_bytes_per_launch": by,
               "intensity_flop_per_byte": intensity, "fp64_ridge_flop_per_byte": ridge,
               "achieved_TFLOPs": fl / avg_s / 1e12, "compulsory_GBps": by / avg_s / 1e9,
               "avg_launch_ms": 1e3 * avg_s, "launches_per_step": st["launches"] / steps,
               "formula": "frac = algorithmic_flops_per_launch / (avg_launch_ms * 1e-3) / (peak * 1e12)"
               if rl["unit"] == "TFLOP/s" else
               "frac = compulsory_bytes_per_launch / (avg_launch_ms * 1e-3) / (peak * 1e9)"})
    return rl


def one_core_rows(workload, R):
    """Seconds the oracle takes for R seeded rows of the workload's product on one OpenMP thread (a
    child process, so that the parent's thread pool is untouched); None if the child fails."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "import numpy as np\n"
            "from oracle import bem\n"
            "from paper_2103_16073_amd import synth\n"
            "room, k = synth.config_room(%d)\n"
            "x = synth.complex_normal(room.n, 11)\n"
            "rc = bem.near_cutoff(room.vertices, room.triangles)\n"
            "rows = np.random.default_rng(6).choice(room.n, %d, replace=False)\n"
            "bem.direct_matvec_rows(room.vertices, room.triangles, k, room.beta, rc, x, rows[:2])\n"
            "t = time.perf_counter()\n"
            "bem.direct_matvec_rows(room.vertices, room.triangles, k, room.beta, rc, x, rows)\n"
            "print(time.perf_counter() - t)\n") % (ROOT, workload, R)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
        return float(r.stdout.strip().splitlines()[-1])
    except Exception as e:  # noqa: BLE001 -- a baseline that failed is reported as missing
        log(f"one-core oracle run failed: {e}")
        return None


def sweep_workload(args):
    """The frequency sweep of one room: the L-room at 64 frequencies log-spaced over 100 Hz - 2 kHz,
    each meshed at 7 elements per wavelength (its own N, octree depth and truncation numbers:
    N = 1,922 ... 612,540) with 4 source positions, 256 FGMRES solves to relative residual 1e-4
    (mixed-precision products, FP32 Krylov vectors, FP64 restart and final residuals, near-field
    leaf blocks).  The contexts, sorted by N, are solved in waves of at most `sweep_wave_n` elements
    by fmmbem_solve_many: every system of a wave in flight from this one thread (the 4 sources of a
    frequency in lock step with 4-vector products, the frequencies advancing in turn on their own
    streams).  A few solutions are checked against the oracle's rows of Eq. dbem4."""
    import numpy as np
    from paper_2103_16073_amd import fmmbem as F
    from paper_2103_16073_amd import synth
    fs = [100.0 * 20.0 ** (i / 63.0) for i in range(64)]
    rooms, ctxs = [], []
    t_setup = 0.0
    for f in fs:
        room = synth.lroom(synth.SOUND_SPEED / (7.0 * f))
        rs, _ = synth.source_and_receivers(room, 4, nsrc=4)
        ctx = F.Context(0, autotune=0)
        ctx.fmmbem_set_mesh(room.vertices, room.triangles)
        ctx.fmmbem_set_wavenumber(synth.wavenumber(f))
        ctx.fmmbem_set_admittance(room.beta)
        ctx.fmmbem_set_sources(rs)
        t0 = time.perf_counter()
        ctx.fmmbem_setup()
        t_setup += time.perf_counter() - t0
        rooms.append((room, rs, f))
        ctxs.append(ctx)
    log(f"sweep: 64 contexts set up in {t_setup:.1f} s, N = {rooms[0][0].n} ... {rooms[-1][0].n}")
    kw = dict(tol=1e-4, restart=args.sweep_restart, maxit=2 * args.sweep_restart, precision=F.FMMBEM_MIXED,
              precond=F.FMMBEM_PC_NEARBLOCK)
    waves, cur, ncur = [], [], 0
    for i, (room, _, _) in enumerate(rooms):
        if cur and ncur + room.n > args.sweep_wave_n:
            waves.append(cur)
            cur, ncur = [], 0
        cur.append(i)
        ncur += room.n
    waves.append(cur)
    sols, reports, t_solve = {}, {}, 0.0
    for w in waves:
        sc = [ctxs[i] for i in w for _ in range(4)]
        ss = [s for _ in w for s in range(4)]
        torch_sync()
        t0 = time.perf_counter()
        xs, reps, status, rc = F.fmmbem_solve_many(sc, ss, **kw)
        dt = time.perf_counter() - t0
        t_solve += dt
        for q, (i, s) in enumerate(zip([i for i in w for _ in range(4)], ss)):
            sols[(i, s)] = xs[q]
            reports[(i, s)] = (status[q], reps[q].iters, reps[q].rel_res)
        log(f"  wave of {len(w)} frequencies (N {rooms[w[0]][0].n}..{rooms[w[-1]][0].n}): {dt:.2f} s, "
            f"iterations {min(r.iters for r in reps)}..{max(r.iters for r in reps)}, code {rc}")
        for i in w:
            ctxs[i].fmmbem_release_workspace()
    # one wave of the small frequencies again, one context after another (fmmbem_solve_batch), for
    # the gain of keeping several contexts in flight
    w0 = waves[0]
    for _ in range(2):  # the second round of each, with the work arrays already in place
        torch_sync()
        t0 = time.perf_counter()
        for i in w0:
            ctxs[i].fmmbem_solve_batch([0, 1, 2, 3], **kw)
        t_seq0 = time.perf_counter() - t0
        torch_sync()
        t0 = time.perf_counter()
        F.fmmbem_solve_many([ctxs[i] for i in w0 for _ in range(4)], [s for _ in w0 for s in range(4)], **kw)
        t_many0 = time.perf_counter() - t0
    log(f"first wave ({len(w0)} frequencies): one context at a time {t_seq0:.2f} s, all in flight {t_many0:.2f} s")
    checks = []
    if not args.no_cpu_baseline:
        from oracle import bem
        for i, s in ((0, 0), (31, 1), (63, 2)):
            room, rs, f = rooms[i]
            k = synth.wavenumber(f)
            rc = bem.near_cutoff(room.vertices, room.triangles)
            rows = np.random.default_rng(20 + i).choice(room.n, min(256, room.n), replace=False)
            ax = bem.direct_matvec_rows(room.vertices, room.triangles, k, room.beta, rc, sols[(i, s)], rows)
            b = bem.direct_rhs_rows(room.vertices, room.triangles, k, room.beta, rs[s], rc, rows)
            r = float(np.linalg.norm(ax - b) / np.linalg.norm(b))
            checks.append({"f_hz": f, "n": room.n, "source": s, "oracle_rows": int(len(rows)),
                           "rel_residual_on_rows": r, "rel_residual_fp64_fmm": reports[(i, s)][2]})
            log(f"  oracle rows, {f:.0f} Hz N {room.n} source {s}: |A x - b| / |b| = {r:.2e} "
                f"(FMM FP64 residual {reports[(i, s)][2]:.2e})")
    its = [v[1] for v in reports.values()]
    ok = sum(1 for v in reports.values() if v[0] == 0)
    result = {"metric": "FGMRES sweep: 64 frequencies x 4 sources to rel. residual 1e-4",
              "value": t_solve, "unit": "s", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
              "dtype": "f64 residuals, f32 products", "data": "synthetic",
              "config": {"workload": "L-room 6x5x3 + 4x3x3 m, baffle slab + doorway; 64 frequencies 100 Hz - 2 kHz "
                                     "log-spaced, 7 elements per wavelength, 4 sources, direct BIE",
                         "n_min": rooms[0][0].n, "n_max": rooms[-1][0].n, "n_total": sum(r[0].n for r in rooms),
                         "restart": args.sweep_restart, "wave_n": args.sweep_wave_n, "waves": len(waves)},
              "solves": len(reports), "converged": ok, "iterations": {"min": min(its), "max": max(its),
                                                                       "mean": sum(its) / len(its)},
              "setup_s": t_setup, "first_wave": {"frequencies": len(w0), "one_context_at_a_time_s": t_seq0,
                                                 "all_in_flight_s": t_many0},
              "oracle_checks": checks}
    for c in ctxs:
        c.close()
    print(json.dumps(result))


def ir_workload(args):
    """Impulse responses of Section 4.1: the 8 x 6 x 3 m shoebox with impedance zeta = 9 on every wall,
    a monopole at (3, 2, 1.75) m, the total field on a receiver plane at z = 1.75 m over the whole
    floor area for 128 frequencies 20, 40, ..., 2560 Hz (T = 50 ms), turned into pressure on 256 time
    steps of T / 256 by the pulse of Eq. (an3) and one inverse FFT per receiver.  Meshes per octave
    band (320, 640, 1280, 2560 Hz tops) at 6.7 elements per wavelength at the band's top frequency,
    the paper's resolution criterion; FGMRES to 1e-4 per frequency.  The image-source solution
    (Eq. an2, R = 0.8, images within c T) is compared on a sample of the plane's receivers in the
    frequency and the time domain."""
    import numpy as np
    from paper_2103_16073_amd import ir, synth
    L, zeta, rs = (8.0, 6.0, 3.0), 9.0, np.array([3.0, 2.0, 1.75])
    df, nf, nt = 20.0, args.ir_freqs, 256
    freqs = df * np.arange(1, nf + 1)
    rec, (nx, ny) = ir.receiver_plane(L[0], L[1], 1.75, args.ir_spacing)
    bands = [b for b in (320.0, 640.0, 1280.0, 2560.0) if b < freqs[-1]] + [float(freqs[-1])]
    log(f"impulse responses: {nf} frequencies {freqs[0]:.0f}-{freqs[-1]:.0f} Hz, plane of {nx} x {ny} = "
        f"{len(rec)} receivers, bands {bands}")
    torch_sync()
    t0 = time.perf_counter()
    H, iters, summary = ir.sweep_plane(L, zeta, rs, freqs, rec, bands, tol=1e-4, wave_n=args.sweep_wave_n, log=log)
    T = 1.0 / df
    dt = T / nt
    spec = ir.an3_spectrum(freqs, dt)
    p = ir.synthesize_fft(H, spec, nt)  # nt x receivers
    t_total = time.perf_counter() - t0
    log(f"sweep + synthesis {t_total:.1f} s, iterations {iters.min()}..{iters.max()}")
    checks = {}
    if not args.no_cpu_baseline:
        from oracle import analytic
        R = (zeta - 1.0) / (zeta + 1.0)
        rng = np.random.default_rng(41)
        # receivers at least 0.3 m from the walls and 0.2 m from the source
        ok = np.where((rec[:, 0] > 0.3) & (rec[:, 0] < L[0] - 0.3) & (rec[:, 1] > 0.3) & (rec[:, 1] < L[1] - 0.3)
                      & (np.linalg.norm(rec - rs, axis=1) > 0.2))[0]
        pick = rng.choice(ok, min(args.ir_check, len(ok)), replace=False)
        t1 = time.perf_counter()
        Hi = np.stack([analytic.image_sum_box(L, rs, rec[pick], 2 * np.pi * f / synth.SOUND_SPEED, R,
                                              r_max=synth.SOUND_SPEED * T) for f in freqs])
        ef = np.linalg.norm(H[:, pick] - Hi, axis=1) / np.linalg.norm(Hi, axis=1)
        pi = ir.synthesize_fft(Hi, spec, nt)
        pb = p[:, pick]
        times = np.arange(nt) * dt
        out = {}
        for name, sel in (("first_25ms", times < T / 2), ("all_50ms", times < T)):
            a, b = pb[sel], pi[sel]
            out[name] = {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                         "correlation": float(np.sum(a * b) / np.sqrt(np.sum(a * a) * np.sum(b * b)))}
        checks = {"receivers": int(len(pick)), "image_method_s": time.perf_counter() - t1,
                  "freq_rel_diff_median": float(np.median(ef)), "freq_rel_diff_max": float(ef.max()),
                  "freq_rel_diff_by_band": {f"{s['band_hz'][0]:.0f}-{s['band_hz'][1]:.0f}":
                                            float(np.median(ef[(freqs >= s['band_hz'][0]) & (freqs <= s['band_hz'][1])]))
                                            for s in summary},
                  "time_domain": out}
        log(f"image sources on {len(pick)} receivers: per-frequency relative difference median "
            f"{checks['freq_rel_diff_median']:.3f}; time domain first 25 ms: rel L2 {out['first_25ms']['rel_l2']:.3f}, "
            f"correlation {out['first_25ms']['correlation']:.4f}; 50 ms: rel L2 {out['all_50ms']['rel_l2']:.3f}, "
            f"correlation {out['all_50ms']['correlation']:.4f}")
    result = {"metric": f"impulse responses: {nf} frequency solves + receiver-plane fields + FFT synthesis",
              "value": t_total, "unit": "s", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
              "dtype": "f64 residuals, f32 products", "data": "synthetic",
              "config": {"workload": "shoebox 8x6x3 m, zeta = 9, source (3, 2, 1.75) m, receiver plane z = 1.75 m",
                         "frequencies": nf, "df_hz": df, "time_steps": nt, "dt_ms": 1e3 * dt,
                         "receivers": int(len(rec)), "plane_grid": [nx, ny], "spacing_m": args.ir_spacing,
                         "elements_per_wavelength": 6.7},
              "bands": summary, "iterations": {"min": int(iters.min()), "max": int(iters.max()),
                                               "mean": float(iters.mean())},
              "image_source_checks": checks}
    if args.ir_out:  # FP32 pressure frames and transfer functions
        np.savez_compressed(args.ir_out, freqs=freqs, receivers=rec.astype(np.float32), plane=np.array([nx, ny]),
                            H=H.astype(np.complex64), p=p.astype(np.float32), dt=dt)
    print(json.dumps(result))


def torch_sync():
    import torch
    torch.cuda.synchronize()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=3,
                    help="named room: 1, 2, 3 or 5 (products and solves; 5: the 6M room at 5 kHz, fixed tile "
                         "rule, the inner-outer solve only); 4: the 64-frequency, 4-source sweep; 6: the impulse "
                         "responses of the shoebox (frequency sweep, receiver plane, pulse, FFT)")
    ap.add_argument("--ir-freqs", type=int, default=128, help="frequencies of the impulse-response sweep (20 Hz apart)")
    ap.add_argument("--ir-spacing", type=float, default=0.05, help="receiver-plane grid spacing (m)")
    ap.add_argument("--ir-check", type=int, default=400, help="plane receivers compared with the image sources")
    ap.add_argument("--ir-out", default=None, help="write H, the receivers and the pressure frames (.npz)")
    ap.add_argument("--sweep-restart", type=int, default=120, help="Krylov dimension of the sweep's solves")
    ap.add_argument("--sweep-wave-n", type=int, default=1000000,
                    help="elements per wave of the sweep (contexts solved together by fmmbem_solve_many)")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--maxit", type=int, default=1200, help="FGMRES iteration cap (= Krylov dimension)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner solve")
    ap.add_argument("--no-coarse-inner", action="store_true",
                    help="skip the solve preconditioned by an inner GMRES on a coarser FMM")
    ap.add_argument("--no-batched-solve", action="store_true", help="skip the 4-source batched solve")
    ap.add_argument("--outer", type=int, default=0,
                    help="Krylov dimension (= iteration cap) of the inner-outer solve (0: 200, 400 for workload 5)")
    ap.add_argument("--inner-steps", type=int, default=0,
                    help="GMRES steps of the inner solve on the coarse FMM (0: 10, 20 for workload 5)")
    ap.add_argument("--batch-restart", type=int, default=850, help="Krylov dimension of the batched solve")
    ap.add_argument("--no-autotune", action="store_true", help="fixed tile-shape rule instead of measured shapes")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run 4 device copies of 512 MiB (calibration of the FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--train-maxit", type=int, default=300, help="iteration cap of the reference solve for training")
    ap.add_argument("--lds-budget", type=int, default=0, help="LDS bytes per translation tile (0 = library default)")
    ap.add_argument("--mfma", type=int, default=1, help="matrix-core tiles: 0 never, 1 library rule/autotuner, 2 every lane batch")
    ap.add_argument("--fused", type=int, default=1, help="fused LDS-resident translation tiles for p <= 16: 0 never, 1 allowed")
    ap.add_argument("--shapes-out", default=None, help="write the batches' tile shapes (JSON) after setup")
    ap.add_argument("--shapes-in", default=None,
                    help="replay tile shapes written by --shapes-out (the same launches as that run); default on the "
                         "L-room: the shapes of the committed counter run")
    ap.add_argument("--fresh-shapes", action="store_true",
                    help="keep this run's autotuned shapes instead of replaying the committed ones")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(frequency/source sharding across GPUs is a design note only)", file=sys.stderr)
        sys.exit(2)
    if args.workload == 4:
        sweep_workload(args)
        return
    if args.workload == 6:
        ir_workload(args)
        return

    import numpy as np
    import torch

    from paper_2103_16073_amd import fmmbem as F
    from paper_2103_16073_amd import synth

    room, k = synth.config_room(args.workload)
    rs, rec = synth.source_and_receivers(room, 64, nsrc=4)
    n = room.n
    log(f"workload {args.workload}: N={n} k={k:.3f}")
    shapes_in = args.shapes_in
    if (shapes_in is None and args.workload == 3 and not args.fresh_shapes and not args.no_autotune
            and os.path.exists(SHAPES_FILE)):
        shapes_in = SHAPES_FILE
    # autotuned even when shapes are replayed: the coarser context of the inner-outer solve
    # inherits the options and tunes its own batches
    # the 6M room (workload 5) runs the fixed tile rule: timing every candidate shape of its
    # batches would take longer than the benchmark
    big = args.workload == 5
    ctx = F.Context(0, lds_budget=args.lds_budget, autotune=0 if (args.no_autotune or big) else 1,
                    mfma=args.mfma, fused=args.fused)
    ctx.fmmbem_set_mesh(room.vertices, room.triangles)
    ctx.fmmbem_set_wavenumber(k)
    ctx.fmmbem_set_admittance(room.beta)
    ctx.fmmbem_set_sources(rs)
    t0 = time.perf_counter()
    ctx.fmmbem_setup()
    t_setup = time.perf_counter() - t0
    info = ctx.fmmbem_get_info()
    ps = [info.p[l] for l in range(info.depth + 1)]
    log(f"setup {t_setup:.2f}s depth {info.depth} leaves {info.nleaf} p {ps} near_nnz {info.near_nnz} "
        f"lds_max {info.lds_max}")
    shapes_src = "autotuned" if not args.no_autotune else "fixed rule"
    if shapes_in:
        with open(shapes_in) as fh:
            want = json.load(fh)
        try:
            ctx.fmmbem_set_batch_shapes(want)
            shapes_src = "replayed from " + os.path.relpath(shapes_in, ROOT)
            log(f"tile shapes {shapes_src}")
        except F.FmmbemError as e:
            if args.shapes_in:
                raise
            log(f"committed tile shapes do not fit this tree ({e}); keeping the autotuned ones")
    shapes = ctx.fmmbem_batch_shapes()
    if args.shapes_out:
        with open(args.shapes_out, "w") as fh:
            json.dump(shapes, fh)
    for s in shapes:
        log(f"  tiles L{s['level']} {s['kind']}: {(('mfma', 'fused', 'fused-reg', 'fused-lds')[s['mfma'] - 1] if s['mfma'] else 'lane') if s['lane'] else ('whole' if s['whole'] else 'degree')} "
            f"JT {s['jt']} jobs {s['jobs']} {s['ms']:.3f} ms")

    dev = torch.device("cuda:0")
    x_h = synth.complex_normal(n, 11)
    x = torch.from_numpy(x_h).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream
    for _ in range(args.warmup):
        ctx.fmmbem_matvec_dev(x.data_ptr(), y.data_ptr(), stream=sp)
    torch.cuda.synchronize()
    log("warmup done")
    if args.copy_calib:
        a = torch.empty(512 * 2 ** 20 // 4, dtype=torch.float32, device=dev)
        c = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(4):
            c.copy_(a)
        torch.cuda.synchronize()
        del a, c
        log("copy calibration: 4 x 512 MiB device copies")

    # timed region: K products as a caller runs them (captured HIP graph, two streams)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.fmmbem_matvec_dev(x.data_ptr(), y.data_ptr(), stream=sp)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms_per_step = 1e3 * t / args.steps
    value = args.steps / t
    log(f"timed {args.steps} matvecs: {ms_per_step:.2f} ms/step, {value:.3f} matvec/s")
    # second timed region, the same K products with HIP events around every kernel on its own
    # stream (eager launches; the events cost ~1.7 ms per product and stop the two streams from
    # overlapping): per-kernel durations for the phase table and the roofline
    ctx.fmmbem_profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.fmmbem_matvec_dev(x.data_ptr(), y.data_ptr(), stream=sp)
    torch.cuda.synchronize()
    t_prof = time.perf_counter() - t0
    stats = ctx.fmmbem_kernel_stats()
    ctx.fmmbem_profile(False)
    log(f"profiled {args.steps} matvecs: {1e3 * t_prof / args.steps:.2f} ms/step")

    # per-phase breakdown and the dominant kernel
    phases = {}
    for s in stats:
        phases[s["name"]] = round(s["ms"] / args.steps, 4)
        log(f"  {s['name']:16s} {s['ms'] / args.steps:9.3f} ms/step  {s['launches'] / args.steps:5.1f} launches  "
            f"{s['flops'] / max(s['ms'], 1e-9) / 1e9:8.2f} TFLOP/s")
    dom = max(stats, key=lambda s: s["ms"])
    roofline = kernel_roofline(dom, args.steps, args.workload == 3 and not args.no_autotune)
    log(f"dominant kernel {dom['name']}: {roofline['avg_launch_ms']:.3f} ms/launch, "
        f"{roofline['achieved_TFLOPs']:.3f} TFLOP/s of the method's flops, "
        f"{roofline['compulsory_GBps']:.0f} GB/s of its compulsory bytes: {roofline['bound']} bound, "
        f"frac {roofline['frac']:.3f}")
    p2p = next((s for s in stats if s["name"] == "k_p2p"), None)
    p2p_line = None
    if p2p is not None:
        t = p2p["ms"] / p2p["launches"] * 1e-3
        p2p_traffic = (measured_traffic("k_p2p", p2p["launches"] / args.steps)
                       if (args.workload == 3 and not args.no_autotune) else None)
        p2p_line = {"kernel": "k_p2p", "avg_launch_ms": 1e3 * t, "pairs_per_s": info.p2p_pairs / t,
                    "algorithmic_bytes_per_launch": p2p["bytes"] / p2p["launches"],
                    "achieved_GBps": p2p["bytes"] / p2p["launches"] / t / 1e9,
                    "hbm_frac": p2p["bytes"] / p2p["launches"] / t / PEAKS["hbm"],
                    "traffic": p2p_traffic,
                    "traffic_GBps": None if p2p_traffic is None else p2p_traffic / t / 1e9,
                    "traffic_hbm_frac": None if p2p_traffic is None else p2p_traffic / t / PEAKS["hbm"],
                    "alu_TFLOPs": p2p["flops"] / p2p["launches"] / t / 1e12,
                    "alu_frac": p2p["flops"] / p2p["launches"] / t / PEAKS["fp64"]}
        log(f"P2P: {p2p_line['pairs_per_s']:.3e} pairs/s, {p2p_line['achieved_GBps']:.0f} GB/s algorithmic "
            f"({p2p_line['hbm_frac']:.3f} of HBM), {p2p_line['alu_TFLOPs']:.2f} TFLOP/s")

    y_h = y.cpu().numpy()

    # the same product in mixed precision (FP32 near field and translations)
    ym = torch.empty_like(x)
    for _ in range(args.warmup):
        ctx.fmmbem_matvec_dev(x.data_ptr(), ym.data_ptr(), precision=F.FMMBEM_MIXED, stream=sp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.fmmbem_matvec_dev(x.data_ptr(), ym.data_ptr(), precision=F.FMMBEM_MIXED, stream=sp)
    torch.cuda.synchronize()
    tm = time.perf_counter() - t0
    ctx.fmmbem_profile(True)
    for _ in range(args.steps):
        ctx.fmmbem_matvec_dev(x.data_ptr(), ym.data_ptr(), precision=F.FMMBEM_MIXED, stream=sp)
    stats_m = ctx.fmmbem_kernel_stats()
    ctx.fmmbem_profile(False)
    ym_h = ym.cpu().numpy()
    mixed = {"ms_per_step": 1e3 * tm / args.steps, "value": args.steps / tm,
             "rel_l2_vs_fp64_product": float(np.linalg.norm(ym_h - y_h) / np.linalg.norm(y_h)),
             "phases_ms": {s["name"]: round(s["ms"] / args.steps, 4) for s in stats_m}}
    log(f"mixed: {mixed['ms_per_step']:.2f} ms/step, {mixed['value']:.3f} matvec/s, "
        f"rel L2 vs FP64 product {mixed['rel_l2_vs_fp64_product']:.2e}")
    for s in stats_m:
        log(f"  {s['name']:20s} {s['ms'] / args.steps:9.3f} ms/step")

    # several vectors per product (the batched solves' products): 4 seeded vectors at once
    batched = {}
    if big:
        args.no_batched_solve = True
    X4 = torch.from_numpy(synth.complex_normal(n, 31, count=4)).to(dev)
    Y4 = torch.empty_like(X4)
    for name, prec in ((("fp64", F.FMMBEM_FP64), ("mixed", F.FMMBEM_MIXED)) if not big else ()):
        for _ in range(max(1, args.warmup)):
            ctx.fmmbem_matvec_dev(X4.data_ptr(), Y4.data_ptr(), nrhs=4, precision=prec, stream=sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.fmmbem_matvec_dev(X4.data_ptr(), Y4.data_ptr(), nrhs=4, precision=prec, stream=sp)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        # check against single-vector products
        y1 = torch.empty_like(X4[0])
        ctx.fmmbem_matvec_dev(X4[3].data_ptr(), y1.data_ptr(), nrhs=1, precision=prec, stream=sp)
        torch.cuda.synchronize()
        d = float(torch.linalg.norm(Y4[3] - y1) / torch.linalg.norm(y1))
        batched[name] = {"vectors": 4, "ms_per_product": 1e3 * tb / args.steps,
                         "vector_products_per_s": 4 * args.steps / tb, "rel_diff_vs_single": d}
        log(f"4-vector products {name}: {1e3 * tb / args.steps:.2f} ms, {4 * args.steps / tb:.2f} vector products/s, "
            f"diff vs single {d:.1e}")
    del X4, Y4
    ctx.fmmbem_release_workspace()

    result = {
        "metric": "FMM-BEM matvecs/s at N=1M" if args.workload == 3 else f"FMM-BEM matvecs/s at N={n}",
        "value": value,
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "profiled_ms_per_step": 1e3 * t_prof / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("L-room 6x5x3 + 4x3x3 m, baffle slab + doorway, %.1f kHz, direct BIE"
                                % (k * synth.SOUND_SPEED / (2e3 * 3.141592653589793)))
                   if args.workload in (3, 5) else f"named room {args.workload}",
                   "n": n, "k": k, "depth": info.depth, "p_per_level": ps, "leaves": info.nleaf,
                   "near_nnz": info.near_nnz, "m2l_pairs": [info.m2l_pairs[l] for l in range(info.depth + 1)],
                   "parallelism": "single GPU"},
        "setup_s": t_setup,
        "tile_shapes": shapes,
        "tile_shapes_source": shapes_src,
        "phases_ms": phases,
        "roofline": roofline,
        "p2p": p2p_line,
        "mixed_precision": mixed,
        "four_vector_products": batched,
    }

    if not args.no_solve:
        # FGMRES to relative residual 1e-4 (FP64 FMM operator, checked at the end), near-field
        # leaf-block preconditioner, Krylov basis kept whole (restart = maxit): plain FP64
        # products, then mixed-precision products with the FP64 final residual.
        # Gram-Schmidt: the library default (a second pass when the first removed most of the
        # vector), then one pass ("_one_pass"; the final FP64 residual decides either way)
        fg = {}
        # the 6M room keeps its Krylov memory bounded: only the inner-outer solve (outer dimension 200)
        plain = () if big else (("fp64", F.FMMBEM_FP64, 1), ("mixed", F.FMMBEM_MIXED, 1),
                                ("fp64_one_pass", F.FMMBEM_FP64, 0), ("mixed_one_pass", F.FMMBEM_MIXED, 0))
        if big:
            args.no_learned = True
        for name, prec, reorth in plain:
            torch.cuda.synchronize()
            xs, rep, rc = ctx.fmmbem_solve(0, tol=1e-4, restart=args.maxit, maxit=args.maxit,
                                           precond=F.FMMBEM_PC_NEARBLOCK, precision=prec, reorth=reorth)
            fg[name] = {"status": rc, "iters": rep.iters, "rel_res_fp64": rep.rel_res, "t_solve_s": rep.t_solve_s,
                        "matvecs_fp64": rep.matvecs_fp64, "matvecs_mixed": rep.matvecs_mixed,
                        "krylov_storage": "fp32" if prec == F.FMMBEM_MIXED else "fp64",
                        "gram_schmidt": "one pass" if reorth == 0 else "second pass when needed"}
            log(f"FGMRES {name}: status {rc} iters {rep.iters} rel_res {rep.rel_res:.3e} t {rep.t_solve_s:.2f}s")
            ctx.fmmbem_release_workspace()
        if not args.no_coarse_inner:
            # the paper's inner-outer scheme: FGMRES (mixed products, Krylov dimension 200) whose
            # preconditioner is 10 GMRES steps (tolerance 0.1) on a second FMM with p_min 4 and
            # excess 0 (p = ceil(k d) per level), itself preconditioned by the leaf blocks
            ctx.fmmbem_release_workspace()
            outer = args.outer if args.outer > 0 else (400 if big else 200)
            ni = args.inner_steps if args.inner_steps > 0 else (20 if big else 10)
            xs, rep, rc = ctx.fmmbem_solve(0, tol=1e-4, restart=outer, maxit=outer, precond=F.FMMBEM_PC_NEARBLOCK,
                                           precision=F.FMMBEM_MIXED, inner_iters=ni, inner_tol=0.1,
                                           inner_p_min=4, inner_p_excess=0.0)
            fg["mixed_coarse_inner"] = {"status": rc, "iters": rep.iters, "inner_iters": rep.inner_iters,
                                        "rel_res_fp64": rep.rel_res, "t_solve_s": rep.t_solve_s,
                                        "t_setup_coarse_s": rep.t_setup_s, "matvecs_fp64": rep.matvecs_fp64,
                                        "matvecs_mixed": rep.matvecs_mixed, "matvecs_coarse": rep.matvecs_coarse,
                                        "inner": {"iters": ni, "tol": 0.1, "p_min": 4, "p_excess": 0.0},
                                        "restart": outer}
            log(f"FGMRES mixed + coarse inner GMRES: status {rc} outer {rep.iters} inner {rep.inner_iters} "
                f"rel_res {rep.rel_res:.3e} t {rep.t_solve_s:.2f}s (coarse setup {rep.t_setup_s:.2f}s)")
            ctx.fmmbem_release_workspace()
        if not args.no_learned:
            # learned preconditioner trained on another source position, mixed products
            ctx.fmmbem_release_workspace()
            trep = ctx.fmmbem_learned_train(1, restart=8, maxit=args.train_maxit, tol=1e-3, max_pairs=12,
                                            epochs=20, batch=4096)
            log(f"learned PC trained: samples {trep.samples} pairs {trep.pairs} loss zero {trep.loss_zero:.3e} "
                f"first {trep.loss_first:.3e} last {trep.loss_last:.3e} data {trep.t_data_s:.1f}s "
                f"train {trep.t_train_s:.1f}s")
            ctx.fmmbem_release_workspace()
            xs, rep, rc = ctx.fmmbem_solve(0, tol=1e-4, restart=args.maxit, maxit=args.maxit,
                                           precond=F.FMMBEM_PC_LEARNED, precision=F.FMMBEM_MIXED)
            fg["mixed_learned"] = {"status": rc, "iters": rep.iters, "rel_res_fp64": rep.rel_res,
                                   "t_solve_s": rep.t_solve_s, "matvecs_fp64": rep.matvecs_fp64,
                                   "matvecs_mixed": rep.matvecs_mixed, "guard_fallback_at": rep.pc_fallback_at,
                                   "training": {"source": 1, "samples": trep.samples, "pairs": trep.pairs,
                                                "loss_zero": trep.loss_zero, "loss_first": trep.loss_first,
                                                "loss_last": trep.loss_last, "t_data_s": trep.t_data_s,
                                                "t_train_s": trep.t_train_s}}
            log(f"FGMRES mixed+learned: status {rc} iters {rep.iters} rel_res {rep.rel_res:.3e} "
                f"t {rep.t_solve_s:.2f}s fallback at {rep.pc_fallback_at}")
        if not args.no_batched_solve:
            # four source positions solved together: one 4-vector mixed product per step
            ctx.fmmbem_release_workspace()
            xs4, reps, rc = ctx.fmmbem_solve_batch([0, 1, 2, 3], tol=1e-4, restart=args.batch_restart,
                                                   maxit=args.maxit, precond=F.FMMBEM_PC_NEARBLOCK,
                                                   precision=F.FMMBEM_MIXED)
            tb = reps[0].t_solve_s
            fg["mixed_batched_4_sources"] = {
                "status": rc, "iters": [r.iters for r in reps], "rel_res_fp64": [r.rel_res for r in reps],
                "t_solve_s_total": tb, "t_solve_s_per_source": tb / 4, "restart": args.batch_restart,
                "matvecs_mixed": reps[0].matvecs_mixed, "matvecs_fp64": reps[0].matvecs_fp64}
            log(f"FGMRES mixed, 4 sources batched: status {rc} iters {[r.iters for r in reps]} "
                f"rel_res {[f'{r.rel_res:.2e}' for r in reps]} t {tb:.2f}s ({tb / 4:.2f}s per source)")
            ctx.fmmbem_release_workspace()
        fg["precond"] = "near-field leaf blocks"
        fg["restart"] = args.maxit
        f64 = fg.get("fp64", {})
        if f64.get("status") == 0 and fg["mixed"]["status"] == 0:
            fg["speedup_mixed_vs_fp64"] = fg["fp64"]["t_solve_s"] / fg["mixed"]["t_solve_s"]
        if f64.get("status") == 0 and fg["mixed_one_pass"]["status"] == 0:
            fg["speedup_mixed_one_pass_vs_fp64"] = fg["fp64"]["t_solve_s"] / fg["mixed_one_pass"]["t_solve_s"]
        if f64.get("status") == 0 and fg.get("mixed_coarse_inner", {}).get("status") == 0:
            fg["speedup_coarse_inner_vs_fp64"] = fg["fp64"]["t_solve_s"] / fg["mixed_coarse_inner"]["t_solve_s"]
        result["fgmres_to_1e-4"] = fg

    if not args.no_cpu_baseline:
        from oracle import bem
        rng = np.random.default_rng(5)
        cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
        # calibrate on a few rows, then run a bounded sample of about cpu_seconds
        rc = bem.near_cutoff(room.vertices, room.triangles)
        assert abs(rc - info.rc) <= 1e-14 * rc, (rc, info.rc)
        probe = rng.choice(n, 16, replace=False)
        tp = time.perf_counter()
        bem.direct_matvec_rows(room.vertices, room.triangles, k, room.beta, rc, x_h, probe)
        per_row = (time.perf_counter() - tp) / 16
        R = int(min(8192, max(32, args.cpu_seconds / max(per_row, 1e-6))))
        rows = rng.choice(n, R, replace=False)
        tc = time.perf_counter()
        ref = bem.direct_matvec_rows(room.vertices, room.triangles, k, room.beta, rc, x_h, rows)
        tcpu = time.perf_counter() - tc
        t_matvec = tcpu * n / R
        # the same oracle on one core (a child process with one OpenMP thread), on a smaller sample
        R1 = max(4, min(R, int(R / max(1, cores))))
        one = one_core_rows(args.workload, R1)
        err = float(np.linalg.norm(y_h[rows] - ref) / np.linalg.norm(ref))
        mixed["rel_l2_vs_oracle_on_sample"] = float(np.linalg.norm(ym_h[rows] - ref) / np.linalg.norm(ref))
        result["cpu_baseline"] = {"value": 1.0 / t_matvec, "unit": "matvec/s", "cores": cores, "kind": "oracle",
                                  "sample": f"{R} seeded rows x all {n} columns in {tcpu:.1f} s, "
                                            f"scaled by N/R",
                                  "cpu_model": cpu_model(),
                                  "value_1core": None if one is None else 1.0 / (one * n / R1),
                                  "sample_1core": None if one is None else
                                  f"{R1} seeded rows x all {n} columns in {one:.1f} s on 1 thread, scaled by N/R"}
        result["gpu_vs_oracle_rel_l2_on_sample"] = err
        log(f"oracle: {R} rows in {tcpu:.1f}s -> {1.0 / t_matvec:.3e} matvec/s; GPU vs oracle rel L2 {err:.3e}")

    ctx.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
