"""GPU: checkpoint/resume, continuation on another buffer, forced allocation failures and
the warm start's fallback when the network's weights are corrupted.

* Resume: a run interrupted after n1 steps (psi copied to the host with the step count,
  the context destroyed, a new context created on a fresh device copy) continues bitwise
  as the uninterrupted run, in imaginary time and after a quench in real time.
* gp_set_psi: the same continuation on a copied device buffer.
* GP_ERR_OOM: an allocation cap (gp_set_alloc_cap) makes context, batch, autotuner and
  network allocations fail with the OOM code; a failed autotune leaves the context's
  mapping, state and psi as they were.
* Corrupted network weights (NaN, or weights that overflow the output): every problem
  falls back to the Gaussian start, and the propagation from there is the plain method's.
"""
import sys

import numpy as np
import pytest

from paper_1601_04641_amd import gp, inputs, nn, warmstart

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gp.load()
    yield
    gp.set_alloc_cap(None)


def c1():
    w = dict(inputs.WORKLOADS["imag_48x40x32"])
    psi0 = inputs.gaussian_psi(w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"])
    return w, psi0


def dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(
        device="cuda", dtype=torch.complex128 if prec == gp.GP_C128 else torch.complex64)


@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
def test_resume_from_host_checkpoint_is_bitwise(prec):
    w, psi0 = c1()
    n1, n2, n3 = 37, 45, 29   # imaginary, imaginary after resume, real after the quench
    # uninterrupted
    a = dev(psi0, prec)
    with gp.Solver.from_workload(a, w) as s:
        s.step_imag(n1)
        s.step_imag(n2)
        s.set_g(w["g"] / 2)
        s.step_real(n3)
        total = s.status()[0]
    # interrupted after n1 steps: checkpoint = host psi + step count, context destroyed
    b = dev(psi0, prec)
    with gp.Solver.from_workload(b, w) as s:
        s.step_imag(n1)
        steps_ckpt = s.status()[0]
        torch.cuda.synchronize()
        ckpt = b.cpu().numpy().copy()
    del b
    torch.cuda.empty_cache()
    c = dev(ckpt, prec)
    with gp.Solver.from_workload(c, w) as s:
        s.step_imag(n2)
        s.set_g(w["g"] / 2)
        s.step_real(n3)
        resumed_steps = steps_ckpt + s.status()[0]
    torch.cuda.synchronize()
    say(f"case: resume prec {prec}: bitwise {torch.equal(a, c)}")
    assert resumed_steps == total == n1 + n2 + n3
    assert torch.equal(a, c)


@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
def test_set_psi_continues_bitwise_on_a_copy(prec):
    w, psi0 = c1()
    a = dev(psi0, prec)
    with gp.Solver.from_workload(a, w) as s:
        s.step_imag(40)
        s.step_real(20)
    b = dev(psi0, prec)
    with gp.Solver.from_workload(b, w) as s:
        s.step_imag(24)          # 16-step graph + eager remainder on b
        c = b.clone()
        b.zero_()
        s.set_psi(c)             # continue on the copy (graphs are rebuilt for it)
        s.step_imag(16)
        s.step_real(20)
        torch.cuda.synchronize()
        assert s.status()[0] == 60
    assert torch.equal(a, c)
    assert float(b.abs().max()) == 0.0   # the old buffer is no longer touched


def _hip():
    import ctypes
    h = ctypes.CDLL("libamdhip64.so")
    h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    h.hipFree.argtypes = [ctypes.c_void_p]
    return h


def hip_alloc(nbytes):
    """A plain device allocation of exactly nbytes (outside torch's caching allocator,
    whose segments are larger than the tensors in them)."""
    import ctypes
    p = ctypes.c_void_p()
    assert _hip().hipMalloc(ctypes.byref(p), nbytes) == 0
    return p


def hip_free(p):
    assert _hip().hipFree(p) == 0


def test_set_psi_rejects_mismatched_buffers():
    w, psi0 = c1()
    a = dev(psi0, gp.GP_C128)
    with gp.Solver.from_workload(a, w) as s:
        for bad in (a[:-1].clone(), a.to(torch.complex64), a.transpose(0, 1), a.reshape(-1).clone()):
            with pytest.raises(ValueError):
                s.set_psi(bad)
        # the C-ABI itself: a pointer into a device allocation smaller than the grid
        small = hip_alloc(1600)
        try:
            rc = gp.load().gp_set_psi(s._h, small.value)
        finally:
            hip_free(small)
        assert rc == gp.GP_ERR_INVALID
        s.step_imag(3)   # still usable on its own buffer
        assert abs(s.norm() - 1.0) <= 1e-12


def test_allocation_cap_forces_oom():
    w, psi0 = c1()
    a = dev(psi0, gp.GP_C128)
    try:
        gp.set_alloc_cap(64)
        with pytest.raises(gp.GPError) as ei:
            gp.Solver.from_workload(a, w)
        assert ei.value.code == gp.GP_ERR_OOM
        with pytest.raises(gp.GPError) as ei:
            gp.Batch(a.reshape(-1), [w], [0])
        assert ei.value.code == gp.GP_ERR_OOM
        with pytest.raises(nn.NNError) as ei:
            nn.Net(base=2, hidden=32, ch=(32, 32, 16), dx=0.5, max_batch=2)
        assert ei.value.code == nn.GPNN_ERR_OOM
        gp.set_alloc_cap(None)
        with gp.Solver.from_workload(a, w) as s:
            s.step_imag(5)
            before_map = s.get_mapping()
            before_psi = a.clone()
            before_steps = s.status()[0]
            # the autotuner's copy of psi (983,040 bytes) exceeds the cap: OOM, nothing changed
            gp.set_alloc_cap(a.numel() * 16 - 1)
            with pytest.raises(gp.GPError) as ei:
                s.autotune("imag", steps=1)
            assert ei.value.code == gp.GP_ERR_OOM
            gp.set_alloc_cap(None)
            assert s.get_mapping() == before_map
            assert torch.equal(a, before_psi)
            assert s.status()[0] == before_steps
            s.step_imag(5)
    finally:
        gp.set_alloc_cap(None)


@pytest.mark.parametrize("corrupt", ["nan", "overflow"])
def test_corrupted_network_weights_fall_back_to_gaussian(corrupt):
    """The residual gate: starts whose stationary residual is not finite, or not below
    the Gaussian's, are replaced by the Gaussian start."""
    prm = inputs.draw_nn_params(2, 6)
    M = len(prm)
    probs = [warmstart.problem(r) for r in prm]
    offs = warmstart._offsets(M)
    with nn.Net(dx=warmstart.DX, max_batch=4) as net:
        wv = nn.flatten(inputs.nn_init_weights(net.shapes, seed=0), net.shapes).astype(np.float32)
        if corrupt == "nan":
            wv[::97] = np.nan
        else:
            wv[:] = 80.0          # exp(min(f, 10)) saturates: a flat, wrong state
        net.set_params(wv)
        psi = torch.empty(M * warmstart.N_GRID ** 3, dtype=torch.complex64, device="cuda")
        gauss = warmstart.gaussian_starts(torch, prm)
        prm_d = torch.from_numpy(np.asarray(prm, dtype=np.float32)).cuda()
        use_net, r_net, r_gauss, _, _ = warmstart.gated_starts(torch, net, prm_d, probs, offs, psi, gauss, 0.5, 4)
    say(f"case: corrupted weights ({corrupt}): use_net {use_net.tolist()}, r_net {r_net}, r_gauss {r_gauss}")
    assert not np.any(use_net)
    assert torch.equal(psi, gauss)
    with gp.Batch(psi, probs, offs) as b:
        st, mu, conv = b.converge_imag(tol=1e-6, check_every=0, max_steps=4000)
    assert np.all(conv) and np.all(np.isfinite(mu))
