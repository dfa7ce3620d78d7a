"""Parity at the full sizes of the named workloads, on sampled outputs the oracle
computes one by one.

* clustered_2m_active: 2,097,152 particles in 400 Plummer spheres, a random 10%
  active subset walked with the relative criterion (alpha = 0.005, geometric
  guard 0.7); |a_old| is the oracle's FP64 Barnes-Hut (theta = 0.5) walk of the
  active particles.
* zoom_6m: tree, sampled FP64/FP32 forces and the full 8-step FP32 rollout
  gradient (consistency with the FP64 rollout gradient).
* adjoint on clustered_262k: the FP64 adjoint against the oracle's per-particle
  gradient on 4,096 random particles, the oracle's central differences of the
  frozen-decision loss against its analytic gradient on the same particles,
  and the FP32 adjoint error; plus the direct-sum (theta = 0) gradient at
  N = 4,096 against autograd of the dense pair sum.
"""
import numpy as np
import pytest
import torch

from paper_2606_17145_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_17145_amd as sg
    return sg


def _t(a):
    return torch.tensor(a, device=DEV)


def rel_err(a, ref):
    nr = np.linalg.norm(ref, axis=1)
    return np.linalg.norm(a - ref, axis=1) / np.maximum(nr, 1e-6 * np.median(nr))


def test_clustered_2m_active_relative(sg, oracle):
    w = WL.clustered_2m_active()
    print(f"clustered_2m_active: N={w.n} active={w.active.size}", flush=True)
    ref = oracle.Tree(w.pos, w.mass, w.eps)
    act = w.active.astype(np.int64)
    a_bh, _ = oracle.walk(ref, dict(w.params("fp64"), criterion="bh", theta=0.5), targets=act)
    a_old = np.zeros(w.n)
    a_old[act] = np.linalg.norm(a_bh, axis=1)
    p = w.params("fp64")
    t = sg.tree_build(_t(w.pos), _t(w.mass), eps=_t(w.eps))
    active = _t(w.active)
    ao = _t(a_old)
    acc, cnt = sg.shortrange_accel(t, p, active=active, a_old=ao)
    sample = np.sort(np.random.default_rng(51).choice(w.active.size, 4096, replace=False))
    acc_ref, cnt_ref = oracle.walk(ref, p, targets=act[sample], a_old=a_old)
    assert np.array_equal(cnt.cpu().numpy()[sample], cnt_ref)
    e = rel_err(acc.cpu().numpy()[sample], acc_ref)
    print(f"   fp64 max rel err {e.max():.3e}; interactions/target {cnt_ref.sum() / sample.size:.0f}", flush=True)
    assert e.max() <= 1e-12
    acc32, cnt32 = sg.shortrange_accel(t, dict(p, precision="fp32"), active=active, a_old=ao)
    e32 = rel_err(acc32.double().cpu().numpy()[sample], acc_ref)
    flips = np.mean(np.any(cnt32.cpu().numpy()[sample] != cnt_ref, axis=1))
    print(f"   fp32 median {np.median(e32):.3e} p99.9 {np.quantile(e32, 0.999):.3e} count flips {flips:.2e}",
          flush=True)
    assert np.median(e32) <= 1e-5 and np.quantile(e32, 0.999) <= 1e-4


def test_adjoint_clustered_262k(sg, oracle):
    w = WL.clustered_262k()
    wt = WL.adjoint_weights(w.n)
    js = WL.fd_subset(w.n)
    print(f"adjoint clustered_262k: N={w.n}, {js.size} sampled particles", flush=True)
    t = sg.tree_build(_t(w.pos), _t(w.mass), eps=_t(w.eps))
    p = w.params("fp64")
    sg.shortrange_accel(t, p)
    dx, dm = sg.shortrange_accel_adjoint(t, p, _t(wt))
    ref = oracle.Tree(w.pos, w.mass, w.eps)
    gx, gm = oracle.gradient_of(ref, p, wt, js)
    dxs, dms = dx.cpu().numpy()[js], dm.cpu().numpy()[js]
    sx, sm = np.sqrt(np.mean(gx ** 2)), np.sqrt(np.mean(gm ** 2))
    ex = np.abs(dxs - gx) / np.maximum(np.abs(gx), 1e-6 * sx)
    em = np.abs(dms - gm) / np.maximum(np.abs(gm), 1e-6 * sm)
    print(f"   fp64 adjoint vs oracle: dx max {ex.max():.2e}, dm max {em.max():.2e}", flush=True)
    assert ex.max() <= 1e-9 and em.max() <= 1e-9
    # the oracle's analytic gradient against central differences (position step 1e-6 L,
    # mass step 1e-6 m) of the loss with every decision frozen
    fx, fm = oracle.fd_gradient_of(ref, p, wt, js, hx=1e-6, hm_rel=1e-6)
    fdx = np.abs(fx - gx) / np.maximum(np.abs(fx), 1e-6 * sx)
    fdm = np.abs(fm - gm) / np.maximum(np.abs(fm), 1e-6 * sm)
    print(f"   FD vs analytic: dx median {np.median(fdx):.2e} p99 {np.quantile(fdx, 0.99):.2e}; "
          f"dm median {np.median(fdm):.2e} p99 {np.quantile(fdm, 0.99):.2e}", flush=True)
    assert np.quantile(fdx, 0.99) <= 1e-4 and np.quantile(fdm, 0.99) <= 1e-4
    # FP32 forward and adjoint (the configuration's precision), and FP32 pair terms
    # with FP64 sums
    for prec in ("fp32", "fp32_acc64"):
        p32 = w.params(prec)
        tok = sg.shortrange_accel(t, p32)[0] is not None and t.list_token
        wdt = torch.float32 if prec == "fp32" else torch.float64
        dx32, dm32 = sg.shortrange_accel_adjoint(t, p32, _t(wt).to(wdt), list_token=tok)
        e32x = np.linalg.norm(dx32.cpu().numpy()[js] - gx, axis=1) / np.maximum(np.linalg.norm(gx, axis=1), 1e-6 * sx)
        e32m = np.abs(dm32.cpu().numpy()[js] - gm) / np.maximum(np.abs(gm), 1e-6 * sm)
        print(f"   {prec} adjoint: dx median {np.median(e32x):.2e} p99.9 {np.quantile(e32x, 0.999):.2e}; "
              f"dm median {np.median(e32m):.2e} p99.9 {np.quantile(e32m, 0.999):.2e}", flush=True)
        assert np.median(e32x) <= 1e-4 and np.median(e32m) <= 1e-4
        if prec == "fp32_acc64":
            # FP32 pair terms summed in FP64: the tail is held to the forward's bar
            assert np.quantile(e32x, 0.999) <= 1e-4 and np.quantile(e32m, 0.999) <= 1e-4


def test_direct_sum_gradient_4096(sg, oracle):
    from oracle import frozen
    w = WL.clustered_4k_for_gradient()
    wt = np.random.default_rng(304).standard_normal((w.n, 3))
    p = dict(w.params("fp64"), theta=0.0)
    print(f"direct-sum gradient: N={w.n}", flush=True)
    t = sg.tree_build(_t(w.pos), _t(w.mass), eps=_t(w.eps))
    acc, _ = sg.shortrange_accel(t, p)
    dx, dm = sg.shortrange_accel_adjoint(t, p, _t(wt))
    acc_ref, gx, gm = frozen.direct_pair_gradient(w.pos, w.mass, w.eps, p, wt)
    assert np.allclose(acc.cpu().numpy(), acc_ref, rtol=1e-11, atol=1e-11 * np.abs(acc_ref).max())
    assert np.allclose(dx.cpu().numpy(), gx, rtol=1e-9, atol=1e-10 * np.abs(gx).max())
    assert np.allclose(dm.cpu().numpy(), gm, rtol=1e-9, atol=1e-10 * np.abs(gm).max())


def test_zoom_6m_step_and_rollout(sg, oracle):
    """zoom_6m (4,194,304 + 128^3 particles, two masses, two softenings): the tree
    against the oracle's (node count, permutation, per-node particle counts), the
    FP64 and FP32 forces of 2,048 sampled targets against the oracle's walk, and
    the full 8-step FP32 rollout gradient of L = sum w . x_8; its agreement with
    the FP64 rollout gradient is a consistency property (the oracle's rollout is
    checked at small N in test_gpu_rollout)."""
    from paper_2606_17145_amd import rollout as RL
    w = WL.zoom_6m()
    print(f"zoom_6m: N={w.n}", flush=True)
    pos, mass, eps = _t(w.pos), _t(w.mass), _t(w.eps)
    t = sg.tree_build(pos, mass, eps=eps)
    ref = oracle.Tree(w.pos, w.mass, w.eps)
    ex = t.export()
    assert t.node_count() == ref.n_nodes
    assert np.array_equal(ex["perm"].cpu().numpy(), ref.perm)
    nd = ref.nodes()
    assert np.array_equal(ex["count"].cpu().numpy(), nd["count"])
    assert np.array_equal(ex["comX"].cpu().numpy().view(np.uint32), nd["comX"])
    del nd
    sample = np.sort(np.random.default_rng(61).choice(w.n, 2048, replace=False))
    p = w.params("fp64")
    acc_ref, cnt_ref = oracle.walk(ref, p, targets=sample)
    del ref
    acc, cnt = sg.shortrange_accel(t, p)
    assert np.array_equal(cnt.cpu().numpy()[sample], cnt_ref)
    e = rel_err(acc.cpu().numpy()[sample], acc_ref)
    print(f"   fp64 max rel err {e.max():.3e}; interactions/target {cnt_ref.sum() / sample.size:.0f}", flush=True)
    assert e.max() <= 1e-12
    acc32, _ = sg.shortrange_accel(t, w.params("fp32"))
    e32 = rel_err(acc32.double().cpu().numpy()[sample], acc_ref)
    print(f"   fp32 median {np.median(e32):.3e} p99.9 {np.quantile(e32, 0.999):.3e}", flush=True)
    assert np.median(e32) <= 1e-5 and np.quantile(e32, 0.999) <= 1e-4
    del t
    vel = _t(w.extra["vel"])
    wx = _t(w.extra["loss_w"])
    ns, dt = w.extra["n_steps"], w.extra["dt"]
    gx32, gv32, x32, _ = RL.kdk_rollout_grad(pos, vel, mass, eps, w.params("fp32"), ns, dt, wx)
    gx64, gv64, x64, _ = RL.kdk_rollout_grad(pos, vel, mass, eps, w.params("fp64"), ns, dt, wx)
    for name, a32, a64 in (("dL/dx0", gx32, gx64), ("dL/dv0", gv32, gv64)):
        a32, a64 = a32.cpu().numpy(), a64.cpu().numpy()
        assert np.all(np.isfinite(a32))
        r = np.linalg.norm(a32 - a64, axis=1) / np.maximum(np.linalg.norm(a64, axis=1),
                                                            1e-6 * np.median(np.linalg.norm(a64, axis=1)))
        print(f"   rollout {name}: fp32 vs fp64 median {np.median(r):.2e} p99.9 {np.quantile(r, 0.999):.2e}",
              flush=True)
        assert np.median(r) <= 1e-4
    dx = np.abs(x32.cpu().numpy() - x64.cpu().numpy()).max()
    print(f"   final positions fp32 vs fp64: max |dx| {dx:.2e}", flush=True)
    assert dx <= 1e-6
