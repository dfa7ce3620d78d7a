"""Pins of the oracle's rollout gradient: the hand-composed adjoint of the
kick-drift-kick steps against autograd through a replay of the same rollout
with every force evaluation's interaction lists frozen."""
import numpy as np
import torch

from paper_2606_17145_amd import workloads as WL


def _case(n=240, seed=31, mixed=True):
    rng = np.random.default_rng(seed)
    x = WL.clustered_positions(rng, n, 4)
    v = 0.3 * rng.standard_normal((n, 3))
    m = rng.uniform(0.5, 1.5, n) / n
    eps = np.where(rng.random(n) < 0.5, 1 / 150, 1 / 600) if mixed else np.full(n, 1 / 300)
    p = dict(G=1.0, r_s=1.25 / 14, r_cut=4.5 * 1.25 / 14, theta=0.5, criterion="bh", alpha=0.0)
    return x, v, m, eps, p


def test_rollout_forward_matches_replay(oracle):
    from oracle import rollout as R
    x, v, m, eps, p = _case()
    xf, vf = R.rollout(x, v, m, eps, p, 3, 2e-3)
    f = R.frozen_replay(x, v, m, eps, p, 3, 2e-3)
    xt, vt = f(torch.tensor(x), torch.tensor(v))
    assert np.allclose(xt.detach().numpy(), xf, rtol=0, atol=1e-13)
    assert np.allclose(vt.detach().numpy(), vf, rtol=1e-11, atol=1e-11 * np.abs(vf).max())
    assert np.abs(xf - x).max() > 1e-4          # the particles did move


def test_rollout_gradient_matches_autograd_of_frozen_replay(oracle):
    from oracle import rollout as R
    x, v, m, eps, p = _case()
    wx = np.random.default_rng(32).standard_normal(x.shape)
    gx, gv = R.rollout_grad(x, v, m, eps, p, 3, 2e-3, wx)
    f = R.frozen_replay(x, v, m, eps, p, 3, 2e-3)
    xt = torch.tensor(x, requires_grad=True)
    vt = torch.tensor(v, requires_grad=True)
    xf, _ = f(xt, vt)
    (torch.tensor(wx) * xf).sum().backward()
    assert np.allclose(gx, xt.grad.numpy(), rtol=1e-9, atol=1e-10 * np.abs(gx).max())
    assert np.allclose(gv, vt.grad.numpy(), rtol=1e-9, atol=1e-10 * np.abs(gv).max())
    # the rollout is not the identity map: the force terms matter in the gradient
    assert np.abs(gx - wx).max() > 1e-6 * np.abs(wx).max()


def test_pm_autograd_agrees_with_forward_and_adjoint():
    # the PyTorch PM gives the same forces, and autograd through it the same
    # gradient that pm_adjoint composes from the transposed steps
    from oracle import pm
    rng = np.random.default_rng(33)
    x = rng.uniform(-0.5, 1.5, (50, 3))
    m = rng.uniform(0.5, 1.5, 50)
    w = rng.standard_normal((50, 3))
    xt = torch.tensor(x, requires_grad=True)
    mt = torch.tensor(m, requires_grad=True)
    a = pm.pm_accel_torch(xt, mt, 1.0, 12, 1.25 / 12)
    ref = pm.pm_accel(x, m, 1.0, 12, 1.25 / 12)
    assert np.abs(a.detach().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    (torch.tensor(w) * a).sum().backward()
    dx, dm = pm.pm_adjoint(x, m, 1.0, 12, 1.25 / 12, w)
    assert np.abs(xt.grad.numpy() - dx).max() <= 1e-11 * np.abs(dx).max()
    assert np.abs(mt.grad.numpy() - dm).max() <= 1e-11 * np.abs(dm).max()


def test_treepm_rollout_gradient_matches_autograd_of_frozen_replay(oracle):
    # short-range tree force plus the PM force on a 14^3 mesh (r_s = 1.25 L / 14)
    from oracle import rollout as R
    x, v, m, eps, p = _case(n=160, seed=34)
    wx = np.random.default_rng(35).standard_normal(x.shape)
    gx, gv = R.rollout_grad(x, v, m, eps, p, 2, 2e-3, wx, n_mesh=14)
    f = R.frozen_replay(x, v, m, eps, p, 2, 2e-3, n_mesh=14)
    xt = torch.tensor(x, requires_grad=True)
    vt = torch.tensor(v, requires_grad=True)
    xf, _ = f(xt, vt)
    xr, _ = R.rollout(x, v, m, eps, p, 2, 2e-3, n_mesh=14)
    assert np.allclose(xf.detach().numpy(), xr, rtol=0, atol=1e-13)
    (torch.tensor(wx) * xf).sum().backward()
    assert np.allclose(gx, xt.grad.numpy(), rtol=1e-9, atol=1e-10 * np.abs(gx).max())
    assert np.allclose(gv, vt.grad.numpy(), rtol=1e-9, atol=1e-10 * np.abs(gv).max())
    # the mesh force changes the result
    xs, _ = R.rollout(x, v, m, eps, p, 2, 2e-3)
    assert np.abs(xs - xr).max() > 1e-6


def test_rollout_with_tree_reuse_matches_autograd_of_frozen_replay(oracle):
    # trees rebuilt every second force evaluation and drifted in between
    # (evaluations 0 and 2 build, 1 and 3 drift the last build)
    from oracle import rollout as R
    x, v, m, eps, p = _case(n=200, seed=36)
    wx = np.random.default_rng(37).standard_normal(x.shape)
    xr, vr = R.rollout(x, v, m, eps, p, 3, 4e-3, rebuild_every=2)
    f = R.frozen_replay(x, v, m, eps, p, 3, 4e-3, rebuild_every=2)
    xt = torch.tensor(x, requires_grad=True)
    vt = torch.tensor(v, requires_grad=True)
    xf, vf = f(xt, vt)
    assert np.allclose(xf.detach().numpy(), xr, rtol=0, atol=1e-13)
    assert np.allclose(vf.detach().numpy(), vr, rtol=1e-11, atol=1e-11 * np.abs(vr).max())
    gx, gv = R.rollout_grad(x, v, m, eps, p, 3, 4e-3, wx, rebuild_every=2)
    (torch.tensor(wx) * xf).sum().backward()
    assert np.allclose(gx, xt.grad.numpy(), rtol=1e-9, atol=1e-10 * np.abs(gx).max())
    assert np.allclose(gv, vt.grad.numpy(), rtol=1e-9, atol=1e-10 * np.abs(gv).max())
    # the reused trees give a different (drifted-tree) rollout, close to the rebuilt one
    xb, _ = R.rollout(x, v, m, eps, p, 3, 4e-3)
    dev = np.abs(xb - xr).max()
    assert 0 < dev < 1e-2 * np.abs(xb - x).max()
    # rebuilding every evaluation is the plain rollout
    x1, v1 = R.rollout(x, v, m, eps, p, 3, 4e-3, rebuild_every=1)
    assert np.array_equal(x1, xb)
