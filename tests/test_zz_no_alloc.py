"""The allocation-free forward (shortrange_accel_noalloc) against shortrange_accel.

Both entry points run the same traversal and evaluation kernels; the variant
keeps its lists in the library's fixed per-GPU buffer.  Per-group lists and
their order do not depend on which workgroup made them, so accelerations and
interaction counts must agree bit for bit.  Two calls in a row, the second on
a smaller input, check that the buffer's contents from the first call (it
keeps them) do not leak into the second.
"""
import numpy as np
import pytest
import torch

from paper_2606_17145_amd import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_17145_amd as sg
    from paper_2606_17145_amd import _lib
    _lib.lib()
    return sg


def gpu_tree(sg, w):
    pos = torch.tensor(w.pos, device=DEV)
    mass = torch.tensor(w.mass, device=DEV)
    eps = torch.tensor(w.eps, device=DEV)
    return sg.tree_build(pos, mass, eps=eps, box=w.box)


def both(sg, tree, params, active=None, a_old=None):
    acc, cnt = sg.shortrange_accel(tree, params, active=active, a_old=a_old)
    n_t = acc.shape[0]
    out = torch.full_like(acc, float("nan"))
    cnt2 = torch.full((n_t, 2), -7, dtype=torch.int32, device=DEV)
    sg.shortrange_accel_noalloc(tree, params, active=active, a_old=a_old, out=out, counts=cnt2)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), cnt.cpu().numpy(), out.cpu().numpy(), cnt2.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_acc64"])
def test_noalloc_matches_shortrange_accel(sg, precision):
    # first call: 40,000 clustered particles (several hundred groups, many units)
    w1 = WL.clustered(40000, seed=21, n_spheres=12)
    say(f"noalloc {precision}: clustered N={w1.n}")
    t1 = gpu_tree(sg, w1)
    a_ref, c_ref, a, c = both(sg, t1, w1.params(precision))
    assert np.array_equal(c, c_ref)
    assert np.array_equal(a, a_ref)
    assert c.sum() > 50 * w1.n
    # second call, smaller: 3,001 particles (a ragged last group), a 10% active
    # subset under the relative criterion
    w2 = WL.clustered(3001, seed=22, n_spheres=3)
    say(f"noalloc {precision}: clustered N={w2.n}, active subset, relative criterion")
    t2 = gpu_tree(sg, w2)
    rng = np.random.default_rng(23)
    active = torch.tensor(np.sort(rng.choice(w2.n, 301, replace=False)).astype(np.int32), device=DEV)
    p = dict(w2.params(precision), criterion="relative", alpha=0.005, theta=0.7)
    a0, _ = sg.shortrange_accel(t2, w2.params("fp64"))
    a_old = a0.norm(dim=1)
    a_ref, c_ref, a, c = both(sg, t2, p, active=active, a_old=a_old)
    assert a.shape == (301, 3)
    assert np.array_equal(c, c_ref)
    assert np.array_equal(a, a_ref)
    # and the first tree again, after the smaller call
    say(f"noalloc {precision}: first tree again")
    a_ref, c_ref, a, c = both(sg, t1, w1.params(precision))
    assert np.array_equal(c, c_ref)
    assert np.array_equal(a, a_ref)


def test_noalloc_single_particle_empty_and_limits(sg):
    from paper_2606_17145_amd import _lib
    w = WL.uniform(1, seed=3, n_mesh=16)
    say("noalloc: one particle")
    t = gpu_tree(sg, w)
    out = torch.full((1, 3), float("nan"), dtype=torch.float64, device=DEV)
    cnt = torch.full((1, 2), -1, dtype=torch.int32, device=DEV)
    sg.shortrange_accel_noalloc(t, w.params("fp64"), out=out, counts=cnt)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.zeros((1, 3)))
    assert np.array_equal(cnt.cpu().numpy(), np.zeros((1, 2), dtype=np.int32))
    # no targets
    w = WL.uniform(2000, seed=4, n_mesh=16)
    t = gpu_tree(sg, w)
    say("noalloc: empty active list")
    acc, _ = sg.shortrange_accel_noalloc(t, w.params("fp64"), active=torch.empty(0, dtype=torch.int32,
                                                                                   device=DEV))
    assert acc.shape == (0, 3)
    # more targets than the entry point takes: refused before any device work
    n_big = 2 ** 18 + 1
    say(f"noalloc: {n_big} targets (refused)")
    w = WL.uniform(n_big, seed=5, n_mesh=64)
    t = gpu_tree(sg, w)
    with pytest.raises(_lib.SrgravError) as ei:
        sg.shortrange_accel_noalloc(t, w.params("fp32"))
    assert ei.value.code == -1 and "at most" in str(ei.value)
    # the handle still works through the allocating entry point afterwards
    acc, cnt = sg.shortrange_accel(t, w.params("fp32"))
    assert torch.isfinite(acc).all()
