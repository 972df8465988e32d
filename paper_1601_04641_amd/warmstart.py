"""Learned warm start for imaginary-time ground-state searches.

    python -m paper_1601_04641_amd.warmstart [--train 4096] [--test 512] [--epochs 40] [--out F]

Pipeline (every numerical step runs in the library's HIP kernels; this module sequences
calls):
  1. Ground states for training: n^3 grids (n = 64, dx = 0.25, dt = 0.1 dx^2), problems
     (nu_x, nu_y, nu_z, g) with nu ~ U[0.5, 4]^3 and g log-uniform on [1, 1000]
     (inputs.draw_nn_params), Gaussian starts, batched imaginary time (gp.Batch) until
     mu changes by at most `data_tol` relative per check.
  2. Training: the gpnn network (include/gpnn.h) with Adam on the L2 distance to the
     ground states, cosine learning-rate decay, mini-batches in a seeded random order.
  3. Inference on held-out problems straight into the solver's complex64 buffer.
  4. Residual gate: per problem, the network's start is kept only if its
     stationary-equation residual ||H[phi] phi - mu phi|| (gp_batch_residual) is below
     the Gaussian's and below `gate` * mu; otherwise the Gaussian is used.
  5. Time to ground state at mu tolerance `tol` (the solver's stopping rule: mu checked
     every K steps, its change and Aitken-extrapolated distance to the limit within
     tol |mu|), in complex128: (a) Gaussian starts, one single-grid solver after another;
     (b) Gaussian starts, batched; (c) gated network starts (inference and gate
     included in the time), batched.
The propagation is the paper's imaginary-time method (program summary (i)); the network
only changes the initial state.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import gp, inputs, nn

N_GRID, DX = 64, 0.25
DT = 0.1 * DX * DX


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def problem(row):
    nux, nuy, nuz, g = (float(v) for v in row)
    return dict(nx=N_GRID, ny=N_GRID, nz=N_GRID, dx=DX, dy=DX, dz=DX, nux=nux, nuy=nuy, nuz=nuz, g=g, dt=DT)


def _offsets(m):
    return np.arange(m, dtype=np.int64) * N_GRID ** 3


def gaussian_starts(torch, prm, out=None, complex128=False):
    host = inputs.gaussian_cube_batch(prm, N_GRID, DX, dtype=np.complex128 if complex128 else np.complex64)
    t = torch.from_numpy(host.reshape(-1))
    if out is None:
        return t.to("cuda")
    out.copy_(t)
    return out


def ground_states(torch, prm, tol, chunk=512, max_steps=40000, tag="data", complex128=False):
    """Ground states (FP32 real part, [M, n, n, n] on the device), their mu, the steps
    each took and how many stopped at max_steps instead of meeting tol (complex64 storage
    puts a noise floor near 1e-9 on the relative mu change of some problems; complex128
    runs the same scheme in FP64, for reference values)."""
    M = len(prm)
    tgt = torch.empty((M, N_GRID, N_GRID, N_GRID), dtype=torch.float32, device="cuda")
    mus, steps = np.zeros(M), np.zeros(M, dtype=np.int64)
    capped = 0
    t0 = time.perf_counter()
    for c0 in range(0, M, chunk):
        sl = slice(c0, min(M, c0 + chunk))
        psi = gaussian_starts(torch, prm[sl], complex128=complex128)
        with gp.Batch(psi, [problem(r) for r in prm[sl]], _offsets(sl.stop - sl.start)) as b:
            st, mu, conv = b.converge_imag(tol=tol, check_every=0, max_steps=max_steps)
        capped += int(np.sum(~conv.astype(bool)))
        tgt[sl] = psi.view(-1, N_GRID, N_GRID, N_GRID).real.float()
        mus[sl], steps[sl] = mu, st
        log(f"[{tag}] {sl.stop}/{M} ground states, steps {int(st.min())}..{int(st.max())}, "
            f"{time.perf_counter() - t0:.1f} s, {capped} stopped at {max_steps} steps")
        del psi
    return tgt, mus, steps, capped


def train(torch, net, prm, tgt, epochs, batch, lr0, seed=0, lr_min=1e-5, log_every=1):
    """Adam on mini-batches in a seeded random order, cosine decay from lr0 to lr_min."""
    M = len(prm)
    prm_d = torch.from_numpy(np.asarray(prm, dtype=np.float32)).cuda()
    out = torch.empty((batch, N_GRID, N_GRID, N_GRID), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    steps_per_epoch = M // batch
    total = epochs * steps_per_epoch
    hist = []
    t = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(M)[:steps_per_epoch * batch].astype(np.int64)).cuda()
        acc = 0.0
        for k in range(steps_per_epoch):
            idx = order[k * batch:(k + 1) * batch]
            pb = prm_d.index_select(0, idx)
            tb = tgt.index_select(0, idx)
            net.forward(pb, out)
            want = (k == steps_per_epoch - 1)
            loss = net.loss_backward(tb, want_loss=want)
            t += 1
            lr = lr_min + 0.5 * (lr0 - lr_min) * (1 + math.cos(math.pi * t / total))
            net.adam_step(lr, t)
            if want:
                acc = loss
        hist.append(acc)
        if ep % log_every == 0 or ep == epochs - 1:
            torch.cuda.synchronize()
            log(f"[train] epoch {ep + 1}/{epochs}: last-batch loss {acc:.3e}, lr {lr:.2e}, "
                f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def infer(torch, net, prm_d, out_c, batch):
    """Network starts for every problem, written into the complex64 or complex128 solver
    buffer out_c ([M * n^3])."""
    M = prm_d.shape[0]
    view = out_c.view(M, N_GRID, N_GRID, N_GRID)
    for c0 in range(0, M, batch):
        c1 = min(M, c0 + batch)
        net.forward(prm_d[c0:c1], view[c0:c1], complex_out=True)


def eval_l2(torch, net, prm, tgt, batch):
    """Relative L2 distance of the normalised network output to each target."""
    M = len(prm)
    prm_d = torch.from_numpy(np.asarray(prm, dtype=np.float32)).cuda()
    out = torch.empty((batch, N_GRID, N_GRID, N_GRID), dtype=torch.float32, device="cuda")
    errs = np.zeros(M)
    for c0 in range(0, M, batch):
        c1 = min(M, c0 + batch)
        net.forward(prm_d[c0:c1], out[:c1 - c0])
        o = out[:c1 - c0].double()
        t = tgt[c0:c1].double()
        o = o / o.pow(2).sum(dim=(1, 2, 3), keepdim=True).sqrt()
        t = t / t.pow(2).sum(dim=(1, 2, 3), keepdim=True).sqrt()
        errs[c0:c1] = (o - t).pow(2).sum(dim=(1, 2, 3)).sqrt().cpu().numpy()
    return errs


def gated_starts(torch, net, prm_d, probs, offs, psi, gauss, gate, batch):
    """Network starts for every problem written into psi (complex64, back to back at
    offs), then the residual gate: a problem keeps the network's start only if its
    stationary-equation residual is finite, below the Gaussian start's (gauss) and below
    gate * |mu|; otherwise its slice of psi is replaced by the Gaussian start (the
    fallback, also taken when corrupted weights give a non-finite or wrong state).
    Returns (use_net, r_net, r_gauss, mu_net, mu_gauss)."""
    M = len(probs)
    with gp.Batch(gauss, probs, offs) as bg:
        r_gauss, mu_gauss = bg.residual()
    infer(torch, net, prm_d, psi, batch)
    with gp.Batch(psi, probs, offs) as b:
        r_net, mu_net = b.residual(allow_nonfinite=True)
    ok = np.isfinite(r_net) & np.isfinite(mu_net)
    use_net = ok & (np.where(ok, r_net, np.inf) < r_gauss) & (np.where(ok, r_net, np.inf) < gate * np.abs(mu_net))
    pv, gv = psi.view(M, -1), gauss.view(M, -1)
    for i in np.nonzero(~use_net)[0]:
        pv[i].copy_(gv[i])
    return use_net, r_net, r_gauss, mu_net, mu_gauss


def time_to_ground_state(torch, net, prm, tol, gate, batch, mu_ref, serial=True, complex128=False):
    """Time to the ground state at tolerance tol from three starts (see the module text);
    complex128: every propagation in FP64 (the network's start is written in complex128),
    so the stopped states can meet tol against an FP64 reference mu_ref."""
    M = len(prm)
    probs = [problem(r) for r in prm]
    offs = _offsets(M)
    res = {"precision": "complex128" if complex128 else "complex64"}
    # (a) Gaussian starts, one single-grid solver after another
    if serial:
        psi = gaussian_starts(torch, prm, complex128=complex128)
        views = psi.view(M, N_GRID, N_GRID, N_GRID)
        solvers = [gp.Solver.from_workload(views[i], p) for i, p in enumerate(probs)]
        torch.cuda.synchronize()
        steps, mus = np.zeros(M, dtype=np.int64), np.zeros(M)
        t0 = time.perf_counter()
        for i, s in enumerate(solvers):
            steps[i], mus[i], _ = s.converge_imag(tol=tol, check_every=0)
        torch.cuda.synchronize()
        res["gaussian_serial"] = dict(seconds=time.perf_counter() - t0, steps_mean=float(steps.mean()),
                                      steps_max=int(steps.max()),
                                      mu_rel_err_max=float(np.max(np.abs(mus - mu_ref) / mu_ref)))
        for s in solvers:
            s.close()
        del psi, views
        log(f"[ttgs] gaussian serial: {res['gaussian_serial']}")
    # (b) Gaussian starts, batched
    psi = gaussian_starts(torch, prm, complex128=complex128)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with gp.Batch(psi, probs, offs) as b:
        st, mu, conv = b.converge_imag(tol=tol, check_every=0)
    torch.cuda.synchronize()
    res["gaussian_batched"] = dict(seconds=time.perf_counter() - t0, steps_mean=float(st.mean()),
                                   steps_max=int(st.max()), converged=int(np.sum(conv)),
                                   mu_rel_err_max=float(np.max(np.abs(mu - mu_ref) / mu_ref)))
    log(f"[ttgs] gaussian batched: {res['gaussian_batched']}")
    # (c) network starts (inference + gate included), batched
    gauss = gaussian_starts(torch, prm, complex128=complex128)  # fallback states, built on the host like (a), (b)
    prm_d = torch.from_numpy(np.asarray(prm, dtype=np.float32)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    use_net, r_net, r_gauss, mu_net, mu_gauss = gated_starts(torch, net, prm_d, probs, offs, psi, gauss, gate,
                                                             batch)
    bad = np.nonzero(~use_net)[0]
    t_gate = time.perf_counter() - t0
    with gp.Batch(psi, probs, offs) as b:
        st, mu, conv = b.converge_imag(tol=tol, check_every=0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    err_net = np.abs(mu - mu_ref) / mu_ref
    worst = np.argsort(err_net)[::-1][:5]
    res["net_worst"] = [dict(index=int(i), mu_rel_err=float(err_net[i]), steps=int(st[i]),
                             prm=[float(v) for v in prm[i]], used_net=bool(use_net[i])) for i in worst]
    res["net_mu_rel_err_quantiles"] = [float(np.quantile(err_net, q)) for q in (0.5, 0.9, 0.99, 1.0)]
    res["net_batched"] = dict(seconds=elapsed, inference_and_gate_seconds=t_gate, steps_mean=float(st.mean()),
                              steps_max=int(st.max()), converged=int(np.sum(conv)),
                              fallbacks=int(len(bad)), gate=gate,
                              residual_net_median=float(np.median(r_net / np.abs(mu_net))),
                              residual_gauss_median=float(np.median(r_gauss / np.abs(mu_gauss))),
                              mu_rel_err_max=float(np.max(np.abs(mu - mu_ref) / mu_ref)))
    log(f"[ttgs] net batched: {res['net_batched']}")
    a = res.get("gaussian_serial", {}).get("seconds")
    bsec, csec = res["gaussian_batched"]["seconds"], res["net_batched"]["seconds"]
    res["speedup_serial_gaussian_over_net_batched"] = (a / csec) if a else None
    res["speedup_batched_gaussian_over_net_batched"] = bsec / csec
    res["step_ratio_gaussian_over_net"] = res["gaussian_batched"]["steps_mean"] / res["net_batched"]["steps_mean"]
    return res


def run(n_train=4096, n_test=512, epochs=40, batch=16, lr0=1e-3, data_tol=1e-8, tol=1e-7, gate=0.5,
        serial=True, arch=None, save_weights=None, load_weights=None):
    import torch
    gp.load()
    arch = arch or dict(base=4, hidden=384, ch=(64, 64, 64, 32, 16))
    prm_train = inputs.draw_nn_params(1, n_train)
    prm_test = inputs.draw_nn_params(2, n_test)
    out = dict(grid=N_GRID, dx=DX, dt=DT, n_train=n_train, n_test=n_test, epochs=epochs, batch=batch, lr0=lr0,
               data_tol=data_tol, tol=tol, arch=dict(arch, ch=list(arch["ch"])))
    t0 = time.perf_counter()
    if load_weights is None:
        tgt, mu_train, st_train, cap_tr = ground_states(torch, prm_train, data_tol, tag="train data")
    tgt_test, mu_test, st_test, cap_te = ground_states(torch, prm_test, data_tol, tag="test data")
    out["data_seconds"] = time.perf_counter() - t0
    # reference mu: the same scheme in FP64 until the change is below 1e-12
    _, mu_ref, _, cap_ref = ground_states(torch, prm_test, 1e-12, tag="reference mu", complex128=True)
    out["mu_reference"] = dict(precision="complex128", tol=1e-12, capped=cap_ref,
                               c64_data_vs_ref_max=float(np.max(np.abs(mu_test - mu_ref) / mu_ref)))
    if load_weights is None:
        out["data_capped"] = [cap_tr, cap_te]
        out["data_steps_mean"] = float(st_train.mean())
    with nn.Net(dx=DX, max_batch=batch, **arch) as net:
        out["n_params"] = net.n_params
        if load_weights is None:
            net.set_params(inputs.nn_init_weights(net.shapes, seed=0))
            hist, tsec = train(torch, net, prm_train, tgt, epochs, batch, lr0)
            out["train_seconds"] = tsec
            out["loss_history"] = hist
            e_tr = eval_l2(torch, net, prm_train[:512], tgt[:512], batch)
            out["rel_l2_train_median"] = float(np.median(e_tr))
            del tgt
            if save_weights:
                np.save(save_weights, net.get_params())
        else:
            net.set_params(np.load(load_weights))
        e_te = eval_l2(torch, net, prm_test, tgt_test, batch)
        out["rel_l2_test_median"] = float(np.median(e_te))
        out["rel_l2_test_p90"] = float(np.percentile(e_te, 90))
        log(f"[eval] relative L2: test median {np.median(e_te):.2e}, p90 {np.percentile(e_te, 90):.2e}")
        torch.cuda.empty_cache()
        out["time_to_ground_state"] = time_to_ground_state(torch, net, prm_test, tol, gate, batch, mu_ref,
                                                            serial=serial, complex128=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--test", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--gate", type=float, default=0.5)
    ap.add_argument("--no-serial", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("--save-weights", default=None, help="write the trained FP32 parameters (.npy)")
    ap.add_argument("--load-weights", default=None, help="skip training; use these parameters (.npy)")
    a = ap.parse_args(argv)
    r = run(a.train, a.test, a.epochs, a.batch, a.lr, gate=a.gate, serial=not a.no_serial,
            save_weights=a.save_weights, load_weights=a.load_weights)
    txt = json.dumps(r, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    print(json.dumps({k: v for k, v in r.items() if k != "loss_history"}), flush=True)


if __name__ == "__main__":
    main()
