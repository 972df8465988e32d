"""Long GPU runs of the paper's workloads, each printing one JSON document.

    python -m paper_1601_04641_amd.experiments quench    [--prec c64|c128] [--out F]
    python -m paper_1601_04641_amd.experiments precision [--seeds 0,1,2,3,4] [--out F]
    python -m paper_1601_04641_amd.experiments strang    [--out F]

quench: the real-time quench workload (512x480x448, dx = 0.05, nu = (1, 1.4142, 1.7321)):
imaginary time (dt = 0.1 dx^2) from the trap's Gaussian until mu changes by at most
`tol` relative over 0.25 time units, then g -> g/2 and 1000 real-time steps
(dt = 0.01 dx^2) with the norm and rms sizes recorded every `every` steps (the time
propagation of program summary (ii), with the observables of calcrms).

precision: the complex64 form (complex64 storage, FP32 sweeps and phase step, FP64
norm / energy / mu / rms sums and renormalisation scale) against the complex128 GPU path
on 384^3 grids (dx = 0.08, dt = 0.1 dx^2, nu ~ U[0.5, 4]^3 and g ~ U[0, 500] drawn per
seed), 20000 imaginary-time steps from the Gaussian: relative error of mu and E and the
largest point difference relative to max|psi|.  The complex128 path itself is compared
with the FP64 CPU reference by the test suite.

Every step runs in the library's HIP kernels; these drivers only sequence calls and read
observables.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import gp, inputs


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _dtype(torch, prec):
    return torch.complex64 if prec == gp.GP_C64 else torch.complex128


def imag_until(s, dt, tol, check_time=0.25, max_steps=200000, tag=""):
    """Imaginary time in chunks of ceil(check_time/dt) steps until the relative change of
    mu over one chunk is at most tol.  Returns (steps, mu history)."""
    k = max(1, math.ceil(check_time / dt))
    steps, hist = 0, []
    prev = s.energy_mu()[1]
    t0 = time.perf_counter()
    while steps < max_steps:
        s.step_imag(k)
        steps += k
        mu = s.energy_mu()[1]
        hist.append(mu)
        rel = abs(mu - prev) / abs(mu)
        log(f"[{tag}] {steps} imaginary steps, mu {mu:.12f}, rel change {rel:.2e}, "
            f"{time.perf_counter() - t0:.1f} s")
        if rel <= tol:
            break
        prev = mu
    return steps, hist


def quench(prec=gp.GP_C64, tol=1e-9, real_steps=1000, every=50):
    import torch
    gp.load()
    w = dict(inputs.WORKLOADS["quench_512x480x448"])
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    psi0 = inputs.gaussian_psi(nx, ny, nz, w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"],
                               dtype=np.complex64 if prec == gp.GP_C64 else np.complex128)
    psi = torch.from_numpy(psi0).to("cuda")
    del psi0
    tag = "c64" if prec == gp.GP_C64 else "c128"
    t0 = time.perf_counter()
    with gp.Solver.from_workload(psi, dict(w, dt=w["dt_imag"])) as s:
        nimag, hist = imag_until(s, w["dt_imag"], tol, tag=tag + " prep")
        e0, mu0 = s.energy_mu()
        rms0 = s.rms().tolist()
    t_prep = time.perf_counter() - t0
    series = []
    with gp.Solver.from_workload(psi, w) as s:
        s.set_g(w["g_quench"])
        n0 = s.norm()
        e_q, mu_q = s.energy_mu()
        series.append(dict(step=0, t=0.0, norm=n0, rms=s.rms().tolist()))
        t0 = time.perf_counter()
        for k in range(every, real_steps + 1, every):
            s.step_real(every)
            series.append(dict(step=k, t=k * w["dt"], norm=s.norm(), rms=s.rms().tolist()))
        t_real = time.perf_counter() - t0
        e1, mu1 = s.energy_mu()
        log(f"[{tag} real] {real_steps} steps, norm drift {abs(series[-1]['norm'] - n0) / n0:.2e}")
    norms = np.array([p["norm"] for p in series])
    eps = 2.0 ** -24 if prec == gp.GP_C64 else 2.0 ** -53
    return dict(
        workload="quench_512x480x448", precision=tag, imag_dt=w["dt_imag"], real_dt=w["dt"],
        prep=dict(steps=nimag, tol=tol, seconds=t_prep, mu=mu0, energy=e0, rms=rms0, mu_history=hist[-5:]),
        quench=dict(g_from=w["g"], g_to=w["g_quench"], energy_after_quench=e_q, mu_after_quench=mu_q,
                    energy_end=e1, mu_end=mu1, energy_rel_change=abs(e1 - e_q) / abs(e_q),
                    steps=real_steps, seconds_incl_observables=t_real),
        norm_drift=float(abs(norms[-1] - norms[0]) / norms[0]),
        norm_max_dev=float(np.max(np.abs(norms - norms[0])) / norms[0]),
        sqrt_n_eps=math.sqrt(real_steps) * eps, series=series)


def precision(seeds=(0, 1, 2, 3, 4), steps=20000, n=384, dx=0.08, chunk=2000):
    import torch
    gp.load()
    out = []
    for seed in seeds:
        (nux, nuy, nuz), g = inputs.draw_trap(seed)
        w = dict(nx=n, ny=n, nz=n, dx=dx, dy=dx, dz=dx, nux=nux, nuy=nuy, nuz=nuz, g=g, dt=0.1 * dx * dx)
        res = dict(seed=seed, nu=[nux, nuy, nuz], g=g, grid=[n, n, n], dx=dx, dt=w["dt"], steps=steps)
        states = {}
        for prec in (gp.GP_C64, gp.GP_C128):
            tag = "c64" if prec == gp.GP_C64 else "c128"
            psi0 = inputs.gaussian_psi(n, n, n, dx, dx, dx, nux, nuy, nuz,
                                       dtype=np.complex64 if prec == gp.GP_C64 else np.complex128)
            psi = torch.from_numpy(psi0).to("cuda")
            del psi0
            mus = []
            with gp.Solver.from_workload(psi, w) as s:
                t0 = time.perf_counter()
                done = 0
                while done < steps:
                    k = min(chunk, steps - done)
                    s.step_imag(k)
                    done += k
                    mus.append(s.energy_mu()[1])
                    log(f"[precision seed {seed} {tag}] {done} steps, mu {mus[-1]:.12f}, "
                        f"{time.perf_counter() - t0:.1f} s")
                wall = time.perf_counter() - t0
                e, mu = s.energy_mu()
                res[tag] = dict(mu=mu, energy=e, rms=s.rms().tolist(), norm=s.norm(), seconds=wall,
                                max_abs_psi=float(psi.abs().max()),
                                mu_last_chunk_rel_change=abs(mus[-1] - mus[-2]) / abs(mus[-1]))
            states[tag] = psi
        a, b = states["c64"].to(torch.complex128), states["c128"]
        res["c64_vs_c128"] = dict(
            mu_rel=abs(res["c64"]["mu"] - res["c128"]["mu"]) / abs(res["c128"]["mu"]),
            energy_rel=abs(res["c64"]["energy"] - res["c128"]["energy"]) / abs(res["c128"]["energy"]),
            max_dpsi_rel=float((a - b).abs().max() / b.abs().max()),
            max_dpsi_abs=float((a - b).abs().max()))
        log(f"[precision seed {seed}] {json.dumps(res['c64_vs_c128'])}")
        del a, b, states
        torch.cuda.empty_cache()
        out.append(res)
    return dict(workload="precision_384cube_dx0.08", runs=out)


def strang(dts=(0.008, 0.004, 0.002, 0.001), t_real=0.4, tol=1e-13):
    """Lie against Strang splitting on the 48x40x32 workload, complex128.

    Imaginary time: for each dt, both splittings from the trap's Gaussian to the fixed
    point (stopping rule at `tol`, then 20% more steps); mu, E, rms, the estimate mu_est
    and the fixed point's distance between the two splittings.  Real time: from a seeded
    perturbed state to t_real, the state's change under dt halving (its error at fixed t
    shrinks like dt^p: p = 1 Lie, 2 Strang)."""
    import torch
    gp.load()
    w0 = dict(inputs.WORKLOADS["imag_48x40x32"])
    nx, ny, nz = w0["nx"], w0["ny"], w0["nz"]
    g0 = inputs.gaussian_psi(nx, ny, nz, w0["dx"], w0["dy"], w0["dz"], w0["nux"], w0["nuy"], w0["nuz"])
    imag = []
    for dt in dts:
        row = dict(dt=dt)
        states = {}
        for split, name in ((gp.GP_SPLIT_LIE, "lie"), (gp.GP_SPLIT_STRANG, "strang")):
            psi = torch.from_numpy(g0).to("cuda")
            with gp.Solver.from_workload(psi, dict(w0, dt=dt), split=split) as s:
                steps, mu, conv = s.converge_imag(tol=tol, check_every=max(1, round(0.05 / dt)), max_steps=10 ** 6)
                s.step_imag(max(1, steps // 5))
                e, mu = s.energy_mu()
                row[name] = dict(steps=int(steps), converged=bool(conv), mu=mu, energy=e, rms=s.rms().tolist(),
                                 mu_est=s.status()[1])
                torch.cuda.synchronize()
                states[name] = psi.cpu().numpy()
            log(f"[strang imag dt {dt}] {name}: mu {row[name]['mu']:.12f} E {row[name]['energy']:.12f}")
        a, b = states["lie"], states["strang"]
        row["max_dpsi_lie_strang"] = float(np.max(np.abs(a - b)) / np.max(np.abs(a)))
        imag.append(row)
    # dt -> 0 differences: first-order (Lie mu) and second-order (E) behaviour
    for key in ("lie", "strang"):
        for q in ("mu", "energy"):
            v = [r[key][q] for r in imag]
            d = [v[k] - v[k + 1] for k in range(len(v) - 1)]
            imag_order = [math.log2(d[k] / d[k + 1]) if d[k + 1] != 0 and d[k] / d[k + 1] > 0 else None
                          for k in range(len(d) - 1)]
            for r, o in zip(imag[2:], imag_order):
                r.setdefault("observed_order", {})[f"{key}_{q}"] = o
    # real time from a smooth start (the Gaussian of a tighter trap: splitting error
    # dominates) and from a start with grid-scale noise (the sweeps' own O(dt^2) error
    # dominates for both splittings)
    starts = {"smooth": inputs.gaussian_psi(nx, ny, nz, w0["dx"], w0["dy"], w0["dz"], 2.0, 2.6, 3.2),
              "noisy": inputs.perturbed_psi(nx, ny, nz, w0["dx"], w0["dy"], w0["dz"], 1.3, 1.6, 2.0, seed=21,
                                            amp=0.15)}
    real = {}
    for start, psi0 in starts.items():
        for split, name in ((gp.GP_SPLIT_LIE, "lie"), (gp.GP_SPLIT_STRANG, "strang")):
            res = []
            for dt in dts:
                psi = torch.from_numpy(psi0).to("cuda")
                with gp.Solver.from_workload(psi, dict(w0, dt=dt), split=split) as s:
                    s.step_real(int(round(t_real / dt)))
                    torch.cuda.synchronize()
                    res.append(psi.cpu().numpy())
            diffs = [float(np.max(np.abs(res[k] - res[k + 1]))) for k in range(len(res) - 1)]
            real[f"{start}_{name}"] = dict(dt=list(dts), successive_max_diff=diffs,
                                           observed_order=[math.log2(diffs[k] / diffs[k + 1])
                                                           for k in range(len(diffs) - 1)])
            log(f"[strang real] {start} {name}: {real[f'{start}_{name}']}")
    return dict(workload="imag_48x40x32", precision="complex128", imag=imag, real=dict(t=t_real, **real))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=("quench", "precision", "strang"))
    ap.add_argument("--prec", choices=("c64", "c128"), default="c64")
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--seeds", default="0,1,2,3,4")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.what == "quench":
        r = quench(gp.GP_C64 if a.prec == "c64" else gp.GP_C128, tol=a.tol)
    elif a.what == "strang":
        r = strang()
    else:
        r = precision(tuple(int(v) for v in a.seeds.split(",")), steps=a.steps)
    txt = json.dumps(r, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    print(txt if not a.out else json.dumps({k: v for k, v in r.items() if k != "series"}), flush=True)


if __name__ == "__main__":
    main()
