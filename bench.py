"""Benchmark: grid-point updates/s of the split-step Crank-Nicolson step on one MI355X.

Workload: the real-time quench on a 512x480x448 grid (dx = 0.05, nu = (1, 1.4142, 1.7321),
g = 100 -> 50, dt = 0.01 dx^2).  The state is prepared by a short imaginary-time run from
the Gaussian, g is quenched, W untimed real-time steps run, then K timed real-time steps.
A step is one full pass of the hot path: potential/nonlinear step + x sweep, y sweep,
z sweep.  psi is resident in HBM when the timed region starts.

The headline (`value`, `dtype` f64) is complex128, the precision of the paper's programs;
`precision_form` holds the same measurement for complex64 storage and sweeps with FP64
reductions.  Each carries a roofline object for its dominant kernel: algorithmic bytes per
launch (one read and one write of psi: 2 x 16 B or 2 x 8 B per point) over its mean
duration from HIP events recorded on the library's stream during the timed region;
`traffic` is the HBM bytes per launch from the committed counter runs
(profiles/traffic.json) when they were taken on the same mapping.  The practical ceiling
is the library's own streaming copy (16-byte buffer loads and stores, like the sweeps' rows).
Line mappings come from a private copy of the committed autotuner cache
(results/autotune_gfx950.txt), which a run never modifies.  cpu_baseline times the CPU
FP64 oracle on host cores on bounded samples: the quench grid, the 48x40x32 run in full and
the 384^3 grid, with all host threads and with one.  Sub-objects: `halo_truncated` (the
truncated-inverse step variants on the quench grid against the exact sweeps), `batched`
(256 uneven grids advanced by shared launches vs one solver after another) and
`time_to_ground_state` (512 held-out problems: Gaussian starts serial and batched, learned
warm starts batched).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12  # MI355X HBM3E, bytes/s
KINDS = ("x_sweep", "y_sweep", "z_sweep", "norm_finalize", "other")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prep", type=int, default=200, help="imaginary-time preparation steps")
    ap.add_argument("--precision", choices=("c128", "c64"), default="c128",
                    help="precision of the headline (the other one is reported beside it)")
    ap.add_argument("--only", action="store_true", help="measure the headline precision only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default line mapping")
    ap.add_argument("--mapping", default=None,
                    help="mx,swx,my,swy,segz,mz: use this line mapping instead of autotuning")
    ap.add_argument("--autotune-cache", default=os.path.join(ROOT, "results", "autotune_gfx950.txt"),
                    help="autotuner cache, read through a private copy (a miss tunes and appends to the copy)")
    ap.add_argument("--autotune-steps", type=int, default=8)
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB copy with the library's copy kernel (HBM counter calibration)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--no-trunc", action="store_true", help="skip the halo-truncated inverse measurement")
    ap.add_argument("--trunc-steps", type=int, default=50)
    ap.add_argument("--batch-n", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--batch-serial-steps", type=int, default=400)
    ap.add_argument("--no-ttgs", action="store_true", help="skip the time-to-ground-state measurement")
    ap.add_argument("--ttgs-n", type=int, default=512)
    ap.add_argument("--weights", default=os.path.join(ROOT, "results", "warmstart_weights.npy"))
    ap.add_argument("--paper-scale", action="store_true",
                    help="instead of the default run: 1000 iterations on each of the paper's large "
                         "grids (1920x1600x1280 imaginary, 1600x1280x960 real time)")
    ap.add_argument("--paper-precision", choices=("c64", "c128", "both"), default="both")
    ap.add_argument("--paper-iterations", type=int, default=1000,
                    help="timed iterations per grid in --paper-scale (the paper's runs: 1000)")
    ap.add_argument("--paper-no-trunc", action="store_true",
                    help="--paper-scale: skip the halo-truncated repeat of each run")
    return ap.parse_args()


def private_cache(path):
    """A temporary copy of the committed autotuner cache: hits read it, misses append to
    the copy, so a run never changes the committed file."""
    import shutil
    import tempfile
    fd, tmp = tempfile.mkstemp(prefix="gpsscn_tune_", suffix=".txt")
    os.close(fd)
    if path and os.path.exists(path):
        shutil.copyfile(path, tmp)
    return tmp


def run_precision(torch, gp, inputs, w, prec, args):
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    npts = nx * ny * nz
    dtype = torch.complex64 if prec == gp.GP_C64 else torch.complex128
    # Thomas-Fermi-like seed is not needed for throughput; the Gaussian of the trap is the
    # documented starting state of the preparation run.
    psi0 = inputs.gaussian_psi(nx, ny, nz, w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"],
                               dtype=np.complex64 if prec == gp.GP_C64 else np.complex128)
    psi = torch.from_numpy(psi0).to("cuda", dtype=dtype)
    del psi0
    prm = dict(w, dt=w["dt_imag"])
    s_imag = gp.Solver.from_workload(psi, prm)
    log(f"[bench] prep: {args.prep} imaginary steps ({'c64' if prec == gp.GP_C64 else 'c128'})")
    s_imag.step_imag(args.prep)
    e, mu = s_imag.energy_mu()
    s_imag.close()
    log(f"[bench] prepared state: mu={mu:.6f} E={e:.6f}")
    s = gp.Solver.from_workload(psi, w)
    s.set_g(w["g_quench"])
    if args.mapping:
        s.set_mapping(*(int(v) for v in args.mapping.split(",")))
        log(f"[bench] mapping set: {s.get_mapping()}")
    elif not args.no_autotune:
        log(f"[bench] autotune: {s.autotune('real', steps=args.autotune_steps, cache_path=args.tune_cache)}")
    n0 = s.norm()
    s.step_real(args.warmup)
    torch.cuda.synchronize()
    s.set_timing(True)
    torch.cuda.synchronize()
    log(f"[bench] timed: {args.steps} real-time steps")
    t0 = time.perf_counter()
    s.step_real(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, n = s.get_timing()
    s.set_timing(False)
    n1 = s.norm()
    rms = s.rms()
    mapping = s.get_mapping()
    s.close()
    del psi
    torch.cuda.empty_cache()
    wall = t1 - t0
    esz = 8 if prec == gp.GP_C64 else 16
    per_kernel = {}
    for k, name in enumerate(KINDS[:3]):
        if n[k]:
            per_kernel[name] = dict(ms=float(ms[k]), launches=int(n[k]),
                                    algorithmic_GBps=2 * esz * npts / (ms[k] * 1e-3) / 1e9)
    return dict(npts=npts, wall=wall, ms=ms, n=n, per_kernel=per_kernel, esz=esz,
                norm_drift=abs(n1 - n0) / n0, rms=rms.tolist(), mapping=mapping)


def run_batch(torch, gp, inputs, args):
    """Batched form: 256 instances drawn by inputs.draw_batch(seed 0) (dims over
    {32, 40, ..., 96} per axis, dx = 0.2, nu ~ U[0.5, 4]^3, g log-uniform [1, 1000],
    dt = 0.004), complex64 with FP64 reductions, Gaussian starts, `batch_steps`
    imaginary-time steps through the batched launches (graph-captured), against the
    same instances advanced one after another by single-grid contexts."""
    ws = inputs.draw_batch(0, args.batch_n)
    sizes = [w["nx"] * w["ny"] * w["nz"] for w in ws]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    total = int(sum(sizes))
    host = np.empty(total, dtype=np.complex64)
    for w, o, n in zip(ws, offs, sizes):
        host[o:o + n] = inputs.gaussian_psi(w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"], w["nux"],
                                            w["nuy"], w["nuz"], dtype=np.complex64).reshape(-1)
    psi0 = torch.from_numpy(host).to("cuda")
    del host
    psi = psi0.clone()
    b = gp.Batch(psi, ws, offs)
    tuned = None
    if not args.no_autotune:
        tuned = b.autotune("imag", steps=4, cache_path=args.tune_cache)
        log(f"[bench] batch autotune: {tuned}")
    b.step_imag(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] batch timed: {args.batch_steps} imaginary steps, {len(ws)} instances, {total} points")
    t0 = time.perf_counter()
    b.step_imag(args.batch_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e, mu = b.energy_mu()
    # per-kernel durations in a short separate eager run
    b.set_timing(True)
    b.step_imag(20)
    ms, nl = b.get_timing()
    b.set_timing(False)
    mapping = b.get_mapping()
    fusion = b.get_yz_fusion()
    b.close()
    # serial per-instance launches: one single-grid context per instance, default mapping
    psi.copy_(psi0)
    views = [psi[o:o + n].view(w["nx"], w["ny"], w["nz"]) for w, o, n in zip(ws, offs, sizes)]
    solvers = [gp.Solver.from_workload(v, w) for v, w in zip(views, ws)]
    for s in solvers:
        s.step_imag(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] serial timed: {args.batch_serial_steps} imaginary steps per instance")
    t0 = time.perf_counter()
    for s in solvers:
        s.step_imag(args.batch_serial_steps)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    for s in solvers:
        s.close()
    del psi, psi0, views
    torch.cuda.empty_cache()
    rate_b = total * args.batch_steps / wall
    rate_s = total * args.batch_serial_steps / wall_s
    kern = {}
    for k, name in enumerate(KINDS[:4]):
        if nl[k]:
            kern[name] = dict(ms=float(ms[k]), launches=int(nl[k]),
                              algorithmic_GBps=(2 * 8 * total / (ms[k] * 1e-3) / 1e9) if k < 3 else None)
    return {"workload": f"batch{len(ws)}_imag_dims32-96_dx0.2_seed0", "instances": len(ws), "points": total,
            "steps": args.batch_steps, "value": rate_b, "unit": "grid-point updates/s",
            "ms_per_step": wall / args.batch_steps * 1e3, "serial_value": rate_s,
            "serial_steps": args.batch_serial_steps, "speedup_vs_serial": rate_b / rate_s,
            "algorithmic_frac_of_hbm_peak": rate_b * 3 * 2 * 8 / PEAK_HBM, "mapping": mapping,
            "yz_fusion": {"enabled": fusion[0], "fused_instances": fusion[1]},
            "kernels": kern, "mu_range": [float(np.min(mu)), float(np.max(mu))]}


def run_truncated(torch, gp, inputs, w, args, main):
    """The halo-truncated inverse (gp_set_truncation) on the quench grid, per precision:
    imaginary time in the exact sweeps (mode 0), the streaming x and y sweeps (mode 1) and
    the exact x sweep followed by one fused pass of the truncated y sweep and the z sweep
    (mode 2), each `trunc_steps` steps from the same Gaussian start after 5 untimed ones,
    with the largest difference from mode 0's final state relative to max|psi|; real time
    in mode 1 only, against the headline's own timed exact steps (`main`).  The exact
    real-time kernels (and mode 2's exact x sweep, the same kernel) are not launched here,
    so the kernel statistics of a default run hold only the timed region's calls of them.
    ms per step and the algorithmic fraction of the HBM peak (6 psi transfers per step in
    modes 0 and 1, 4 in mode 2)."""
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    npts = nx * ny * nz
    K = args.trunc_steps
    out = {"workload": "quench_512x480x448", "steps": K}
    for prec in (gp.GP_C128, gp.GP_C64):
        tag = "c64" if prec == gp.GP_C64 else "c128"
        esz = 8 if prec == gp.GP_C64 else 16
        ndt = np.complex64 if prec == gp.GP_C64 else np.complex128
        psi0 = torch.from_numpy(inputs.gaussian_psi(nx, ny, nz, w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"],
                                                    w["nuz"], dtype=ndt)).to("cuda")
        psi = torch.empty_like(psi0)
        for kind, modes in (("imag", (0, 1, 2)), ("real", (1,))):
            prm = dict(w, dt=w["dt_imag"]) if kind == "imag" else dict(w)
            ref = None
            for mode in modes:
                psi.copy_(psi0)
                with gp.Solver.from_workload(psi, prm) as s:
                    if not args.no_autotune:   # the exact sweeps' mapping (z in mode 1, x in mode 2)
                        s.autotune(kind, steps=args.autotune_steps, cache_path=args.tune_cache)
                    s.set_truncation(mode)
                    step = s.step_imag if kind == "imag" else s.step_real
                    step(5)
                    torch.cuda.synchronize()
                    s.set_timing(True)
                    t0 = time.perf_counter()
                    step(K)
                    torch.cuda.synchronize()
                    wall = time.perf_counter() - t0
                    ms, n = s.get_timing()
                    s.set_timing(False)
                    hlen = s.get_truncation()[1][0 if kind == "imag" else 1]
                torch.cuda.synchronize()
                if kind == "real":
                    diff = None   # no exact reference from this start (tests cover the accuracy)
                elif mode == 0:
                    ref = psi.clone()
                    diff = 0.0
                else:
                    diff = float((psi - ref).abs().max() / ref.abs().max())
                moves = 4 if mode == 2 else 6
                r = dict(ms_per_step=wall / K * 1e3, updates_per_s=npts * K / wall,
                         algorithmic_frac_of_hbm_peak=npts * K / wall * moves * esz / PEAK_HBM,
                         kernel_ms={KINDS[q]: float(ms[q]) for q in range(3) if n[q]},
                         halo=hlen if mode else None, max_rel_diff_vs_exact=diff)
                if kind == "real" and prec in main:
                    m = main[prec]
                    r["exact_ms_per_step"] = m["ms_per_step"]
                    r["speedup_vs_exact"] = m["ms_per_step"] / r["ms_per_step"]
                out[f"{tag}_{kind}_mode{mode}"] = r
                log(f"[bench] truncation {tag} {kind} mode {mode}: {r['ms_per_step']:.3f} ms/step"
                    + ("" if diff is None else f", diff vs exact {diff:.2e}"))
            del ref
        del psi, psi0
        torch.cuda.empty_cache()
    return out


def stream_copy_gbps(torch, gp, nbytes=1 << 30, reps=5):
    """Practical HBM ceilings: the library's streaming copy kernel (16-byte buffer loads and
    stores, as the sweeps' rows) and torch's device copy, read + write bytes over HIP-event
    time (both run on torch's current stream)."""
    a = torch.empty(nbytes // 8, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    out = {}
    for name, fn in (("library_copy_GBps", lambda: gp.stream_copy(a, b)), ("torch_copy_GBps", lambda: b.copy_(a))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = 2 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


def run_ttgs(torch, args):
    """Time to ground state at mu tolerance 1e-7 on 512 held-out problems of the learned
    warm-start workload (64^3, dx = 0.25, dt = 0.00625, nu ~ U[0.5, 4]^3, g log-uniform
    on [1, 1000], seed 2): Gaussian starts one solver after another, Gaussian starts
    batched, and network starts (trained weights from results/, inference and residual
    gate inside the clock) batched, all in complex128 (complex64's own rounding floor puts
    some of these ground states up to 7e-7 from the FP64 mu).  Reference mu: the same
    scheme in complex128 until the stopping rule holds at 1e-12."""
    from paper_1601_04641_amd import inputs, nn, warmstart as ws
    prm = inputs.draw_nn_params(2, args.ttgs_n)
    _, mu_ref, _, _ = ws.ground_states(torch, prm, 1e-12, tag="ttgs reference (complex128)", complex128=True)
    with nn.Net(dx=ws.DX, max_batch=16) as net:
        net.set_params(np.load(args.weights))
        r = ws.time_to_ground_state(torch, net, prm, 1e-7, 0.5, 16, mu_ref, serial=True, complex128=True)
    torch.cuda.empty_cache()
    r["workload"] = f"warmstart_64cube_dx0.25_{len(prm)}_heldout_seed2"
    r["tol"] = 1e-7
    return r


def cpu_baseline(inputs):
    """The FP64 CPU oracle on bounded samples, with all host threads and with one: the
    quench grid (real time, the headline workload), the 48x40x32 imaginary-time run in
    full (500 steps) and the 384^3 grid of the precision form (imaginary time, seed 0).
    Each leg is timed around its step loop; about 20-30 s in all."""
    import oracle
    nproc = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    q = dict(inputs.WORKLOADS["quench_512x480x448"])
    q["g"] = q["g_quench"]
    c1 = dict(inputs.WORKLOADS["imag_48x40x32"])
    (nux, nuy, nuz), g3 = inputs.draw_trap(0)
    c3 = dict(inputs.WORKLOADS["imag_384cube"], nux=nux, nuy=nuy, nuz=nuz, g=g3)
    legs = []
    states = {}
    for threads in (nproc, 1):
        oracle.set_threads(threads)
        for name, w, imag, steps in (("quench_512x480x448_real_time", q, False, 5 if threads > 1 else 1),
                                     ("imag_48x40x32_500_steps", c1, True, 500),
                                     ("imag_384cube_seed0", c3, True, 5 if threads > 1 else 1)):
            if name not in states:
                states[name] = inputs.gaussian_psi(w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"], w["nux"],
                                                   w["nuy"], w["nuz"])
            o = oracle.Oracle.from_params(w, states[name])
            t0 = time.perf_counter()
            (o.step_imag if imag else o.step_real)(steps)
            el = time.perf_counter() - t0
            o.close()
            npts = w["nx"] * w["ny"] * w["nz"]
            legs.append(dict(workload=name, threads=threads, steps=steps, seconds=el, value=npts * steps / el))
            log(f"[bench] cpu oracle {name}, {threads} threads: {steps} steps in {el:.2f} s")
    head = legs[0]
    return dict(value=head["value"], unit="grid-point updates/s", cores=head["threads"], kind="oracle",
                sample=f"{head['steps']} real-time steps of the 512x480x448 quench workload, complex128 FP64 "
                       f"oracle, OpenMP over lines, {head['seconds']:.1f} s; further legs (1 thread, the "
                       f"48x40x32 run in full, the 384^3 grid) in `legs`",
                legs=legs)


def max_rel_diff(torch, a, b, chunk=1 << 26):
    """max|a - b| / max|b| over flat views, in chunks (no psi-sized temporaries)."""
    fa, fb = a.reshape(-1), b.reshape(-1)
    num = den = 0.0
    for o in range(0, fa.numel(), chunk):
        num = max(num, float((fa[o:o + chunk] - fb[o:o + chunk]).abs().max()))
        den = max(den, float(fb[o:o + chunk].abs().max()))
    return num / den


def run_paper_scale(torch, gp, inputs, args):
    """The paper's large runs on one device: 1000 imaginary-time iterations on 1920x1600x1280
    and 1000 real-time iterations on 1600x1280x960 from the trap's Gaussian, in complex128
    (the paper's precision; 63 and 31 GB) and complex64 storage and sweeps with FP64
    reductions (31.5 and 15.7 GB), psi resident in HBM, autotuned line mapping.  Each run
    is repeated from the same start with the halo-truncated inverse's streaming x and y
    sweeps (gp_set_truncation mode 1; `halo_truncated_mode1`, with the largest difference
    of its final state from the exact run's) unless --paper-no-trunc."""
    out = {}
    precs = {"c64": [gp.GP_C64], "c128": [gp.GP_C128], "both": [gp.GP_C128, gp.GP_C64]}[args.paper_precision]
    for prec in precs:
        tag = "c64" if prec == gp.GP_C64 else "c128"
        esz = 8 if prec == gp.GP_C64 else 16
        cdt, ndt = (torch.complex64, np.complex64) if prec == gp.GP_C64 else (torch.complex128, np.complex128)
        for name, imag in (("paper_imag_1920x1600x1280", True), ("paper_real_1600x1280x960", False)):
            w = dict(inputs.WORKLOADS[name])
            nx, ny, nz, K = w["nx"], w["ny"], w["nz"], args.paper_iterations
            npts = nx * ny * nz
            f = [torch.from_numpy(v.astype(ndt)).to("cuda")
                 for v in inputs.gaussian_factors(nx, ny, nz, w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"],
                                                  w["nuz"])]
            psi = torch.empty((nx, ny, nz), dtype=cdt, device="cuda")
            ref = None
            mapping = None
            for trunc in ((0,) if args.paper_no_trunc else (0, 1)):
                torch.mul(f[0][:, None, None] * f[1][None, :, None], f[2][None, None, :], out=psi)
                s = gp.Solver.from_workload(psi, w)
                step = s.step_imag if imag else s.step_real
                if trunc == 0:
                    log(f"[bench] {name} {tag}: {npts * esz / 1e9:.1f} GB, default mapping {s.get_mapping()}")
                    if args.mapping:
                        s.set_mapping(*(int(v) for v in args.mapping.split(",")))
                    elif not args.no_autotune:
                        s.autotune("imag" if imag else "real", steps=3, cache_path=args.tune_cache)
                    mapping = s.get_mapping()
                else:
                    s.set_mapping(*mapping)
                    s.set_truncation(1)
                label = "exact" if trunc == 0 else "halo-truncated mode 1"
                log(f"[bench] {name} {tag} {label}: mapping {s.get_mapping()}; warmup")
                step(args.warmup)
                n0 = s.norm()
                torch.cuda.synchronize()
                s.set_timing(True)
                log(f"[bench] {name} {tag} {label}: timed {K} iterations")
                t0 = time.perf_counter()
                step(K)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                ms, n = s.get_timing()
                s.set_timing(False)
                e, mu = s.energy_mu()
                n1 = s.norm()
                r = dict(grid=[nx, ny, nz], precision=tag, mode="imaginary" if imag else "real", iterations=K,
                         seconds=wall, ms_per_step=wall / K * 1e3, updates_per_s=npts * K / wall,
                         algorithmic_frac_of_hbm_peak=npts * K / wall * 6 * esz / PEAK_HBM,
                         kernels={KINDS[q]: dict(ms=float(ms[q]), GBps=2 * esz * npts / (ms[q] * 1e-3) / 1e9)
                                  for q in range(3) if n[q]},
                         mapping=s.get_mapping(), mu=mu, energy=e,
                         norm=n1 if imag else None, norm_drift=None if imag else abs(n1 - n0) / n0)
                if trunc:
                    r["halo"] = s.get_truncation()[1][0 if imag else 1]
                s.close()
                log(f"[bench] {name} {tag} {label}: {wall:.1f} s for {K} iterations ({r['ms_per_step']:.2f} ms/step)")
                torch.cuda.synchronize()
                if trunc == 0:
                    out[f"{name}_{tag}"] = r
                    if not args.paper_no_trunc:
                        ref = psi.clone()
                else:
                    r["max_rel_diff_vs_exact"] = max_rel_diff(torch, psi, ref)
                    out[f"{name}_{tag}"]["halo_truncated_mode1"] = r
                    log(f"[bench] {name} {tag}: final states differ by {r['max_rel_diff_vs_exact']:.2e}")
            del f, psi, ref
            torch.cuda.empty_cache()
            # the practical ceiling at this footprint: a copy of psi's size
            out[f"{name}_{tag}"].update(stream_copy_gbps(torch, gp, nbytes=npts * esz, reps=3))
            r = out[f"{name}_{tag}"]
            log(f"[bench] {name} {tag}: copies of {npts * esz / 1e9:.1f} GB: "
                f"{r['library_copy_GBps']:.0f} (library), {r['torch_copy_GBps']:.0f} (torch) GB/s")
    return out


def roofline(gp, r, prec, traffic_json, copy):
    """Roofline object of the dominant (slowest) sweep of one precision's timed run."""
    pk = r["per_kernel"]
    dom = max(pk, key=lambda k: pk[k]["ms"])
    achieved = pk[dom]["algorithmic_GBps"]
    key = "c64" if prec == gp.GP_C64 else "c128"
    traffic = None
    if os.path.exists(traffic_json):
        try:
            tj = json.load(open(traffic_json)).get(key, {})
            # counters hold for the kernels they were taken on: same workload and mapping
            if list(tj.get("mapping", [])) == list(r["mapping"]):
                traffic = tj.get(dom)
        except (ValueError, OSError):
            traffic = None
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": achieved / (PEAK_HBM / 1e9), "traffic": traffic,
            "measured_GBps": (traffic / (pk[dom]["ms"] * 1e-3) / 1e9) if traffic else None,
            "library_copy_GBps": copy["library_copy_GBps"], "torch_copy_GBps": copy["torch_copy_GBps"],
            "frac_of_library_copy": achieved / copy["library_copy_GBps"]}


def main():
    args = parse()
    if args.gpus != 1:
        log("bench.py runs on one GPU only: this library has no multi-GPU decomposition "
            "(each GPU would hold an x-slab); use --gpus 1")
        sys.exit(2)
    import torch

    from paper_1601_04641_amd import gp, inputs
    gp.load()
    args.tune_cache = private_cache(args.autotune_cache)
    if args.paper_scale:
        ps = run_paper_scale(torch, gp, inputs, args)
        print(json.dumps({"metric": "seconds for 1000 iterations on the paper's large grids",
                          "n_gpus": 1, "dtype": "f64" if args.paper_precision == "c128" else "mixed",
                          "data": "synthetic", "runs": ps}), flush=True)
        return
    w = dict(inputs.WORKLOADS["quench_512x480x448"])
    head = gp.GP_C128 if args.precision == "c128" else gp.GP_C64
    precs = [head] if args.only else [head, gp.GP_C64 if head == gp.GP_C128 else gp.GP_C128]
    res = {prec: run_precision(torch, gp, inputs, w, prec, args) for prec in precs}
    if args.calib_copy:
        n = 1 << 27  # 2^27 complex64 = 1 GiB
        a = torch.empty(n, dtype=torch.complex64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        gp.stream_copy(a, b)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy (gpk::k_stream_copy): {n * 8} bytes read, {n * 8} bytes written")
        del a, b
    copy = stream_copy_gbps(torch, gp)
    log(f"[bench] 1 GiB copies: {copy['library_copy_GBps']:.0f} (library), {copy['torch_copy_GBps']:.0f} (torch) GB/s")
    K = args.steps

    def summary(prec):
        r = res[prec]
        return dict(value=r["npts"] * K / r["wall"], ms_per_step=r["wall"] / K * 1e3,
                    roofline=roofline(gp, r, prec, args.traffic_json, copy),
                    algorithmic_frac_of_hbm_peak=r["npts"] * K / r["wall"] * 6 * r["esz"] / PEAK_HBM,
                    kernels=r["per_kernel"], norm_drift=r["norm_drift"], mapping=r["mapping"])

    main_r = summary(head)
    out = {
        "metric": "grid-point updates/s per SSCN step (% HBM roofline); time-to-ground-state at mu tol 1e-7",
        "value": main_r["value"],
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == gp.GP_C64 else "f64",
        "data": "synthetic",
        "config": {"workload": "quench_512x480x448_real_time", "grid": [w["nx"], w["ny"], w["nz"]],
                   "precision": "complex64 storage+sweeps, FP64 reductions" if head == gp.GP_C64
                   else "complex128", "dx": w["dx"], "nu": [w["nux"], w["nuy"], w["nuz"]],
                   "g": [w["g"], w["g_quench"]], "dt": w["dt"], "split": "lie",
                   "prep_imag_steps": args.prep, "mapping": main_r["mapping"]},
        "roofline": main_r["roofline"],
        "algorithmic_frac_of_hbm_peak": main_r["algorithmic_frac_of_hbm_peak"],
        "kernels": main_r["kernels"],
        "norm_drift": main_r["norm_drift"],
    }
    if len(precs) > 1:
        other = precs[1]
        sub = summary(other)
        sub["dtype"] = "f32" if other == gp.GP_C64 else "f64"
        sub["precision"] = ("complex64 storage+sweeps, FP64 reductions" if other == gp.GP_C64 else "complex128")
        out["precision_form" if other == gp.GP_C64 else "complex128"] = sub
    if not args.no_trunc:
        out["halo_truncated"] = run_truncated(torch, gp, inputs, w, args,
                                              {p: summary(p) for p in precs})
    if not args.no_batch:
        out["batched"] = run_batch(torch, gp, inputs, args)
    if not args.no_ttgs and os.path.exists(args.weights):
        log("[bench] time to ground state (512 held-out problems, three starts)")
        out["time_to_ground_state"] = run_ttgs(torch, args)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: the oracle on bounded samples")
        out["cpu_baseline"] = cpu_baseline(inputs)
    os.unlink(args.tune_cache)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
