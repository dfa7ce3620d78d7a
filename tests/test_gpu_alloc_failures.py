"""Out-of-memory paths, forced from the host with the library's allocation-failure
hook (srgrav_inject_alloc_failure): every failing call returns SR_ENOMEM, frees
what it had allocated, and leaves the library and the handles usable.  No
kernel is made to fail; the injected failure replaces a hipMalloc."""
import numpy as np
import pytest
import torch

from paper_2606_17145_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SR_ENOMEM = -2


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_17145_amd as sg
    from paper_2606_17145_amd import _lib
    _lib.lib()
    yield sg
    _lib.lib().srgrav_inject_alloc_failure(-1)


def inject(after):
    from paper_2606_17145_amd import _lib
    _lib.check(_lib.lib().srgrav_inject_alloc_failure(after))


def tensors(w):
    return (torch.tensor(w.pos, device=DEV), torch.tensor(w.mass, device=DEV), torch.tensor(w.eps, device=DEV))


def test_tree_build_failures(sg):
    w = WL.clustered(5000, seed=51, n_spheres=4)
    pos, mass, eps = tensors(w)
    p = w.params("fp64")
    ref_acc, ref_cnt = sg.shortrange_accel(sg.tree_build(pos, mass, eps=eps), p)
    # the first, a middle and the last of the workspace's device allocations
    for k in (0, 17, 52):
        say(f"alloc failure: tree_build, allocation {k}")
        inject(k)
        with pytest.raises(sg.SrgravError) as ei:
            sg.tree_build(pos, mass, eps=eps)
        inject(-1)
        assert ei.value.code == SR_ENOMEM
    # a handle that grows: built small, rebuilt larger under an injected failure
    small = WL.clustered(1000, seed=52, n_spheres=2)
    t = sg.tree_build(*tensors(small)[:2], eps=tensors(small)[2])
    inject(0)
    with pytest.raises(sg.SrgravError) as ei:
        t.build(pos, mass, eps=eps)
    inject(-1)
    assert ei.value.code == SR_ENOMEM
    # its old tree went with the old workspace: the handle now reads as never built
    with pytest.raises(sg.SrgravError) as ei:
        sg.shortrange_accel(t, small.params("fp64"))
    assert ei.value.code == -4
    t.build(pos, mass, eps=eps)
    acc, cnt = sg.shortrange_accel(t, p)
    assert torch.equal(cnt, ref_cnt) and torch.equal(acc, ref_acc)


def test_list_drift_and_noalloc_failures(sg):
    w = WL.clustered(8000, seed=53, n_spheres=4)
    pos, mass, eps = tensors(w)
    p = w.params("fp32")
    ref_acc, ref_cnt = sg.shortrange_accel(sg.tree_build(pos, mass, eps=eps), p)
    t = sg.tree_build(pos, mass, eps=eps)
    say("alloc failure: interaction lists")
    inject(0)
    with pytest.raises(sg.SrgravError) as ei:
        sg.shortrange_accel(t, p)
    inject(-1)
    assert ei.value.code == SR_ENOMEM
    acc, cnt = sg.shortrange_accel(t, p)
    assert torch.equal(cnt, ref_cnt) and torch.equal(acc, ref_acc)
    say("alloc failure: drift buffers")
    inject(0)
    with pytest.raises(sg.SrgravError) as ei:
        t.drift(torch.zeros((w.n, 3), dtype=torch.float64, device=DEV))
    inject(-1)
    assert ei.value.code == SR_ENOMEM
    t.drift(torch.zeros((w.n, 3), dtype=torch.float64, device=DEV))
    acc, cnt = sg.shortrange_accel(t, p)
    assert torch.equal(cnt, ref_cnt) and torch.equal(acc, ref_acc)
    # the allocation-free forward allocates nothing: an armed failure is still armed after it
    say("alloc failure armed across shortrange_accel_noalloc")
    out = torch.empty_like(acc)
    inject(0)
    try:
        sg.shortrange_accel_noalloc(t, p, out=out)
        with pytest.raises(sg.SrgravError) as ei:
            sg.tree_build(pos, mass, eps=eps)
        assert ei.value.code == SR_ENOMEM
    finally:
        inject(-1)
    assert torch.equal(out, ref_acc)


def test_pm_failures(sg):
    w = WL.uniform(4096, seed=54, n_mesh=16)
    pos, mass, _ = tensors(w)
    ref = sg.PM(16).accel(pos, mass, box=1.0, r_s=w.r_s)
    say("alloc failure: pm_create")
    for k in (0, 2):
        inject(k)
        with pytest.raises(sg.SrgravError) as ei:
            sg.PM(16)
        inject(-1)
        assert ei.value.code == SR_ENOMEM
    pm = sg.PM(16)
    say("alloc failure: PM particle workspace")
    inject(0)
    with pytest.raises(sg.SrgravError) as ei:
        pm.accel(pos, mass, box=1.0, r_s=w.r_s)
    inject(-1)
    assert ei.value.code == SR_ENOMEM
    # (the mesh assignment adds with device atomics: equal to rounding)
    assert torch.allclose(pm.accel(pos, mass, box=1.0, r_s=w.r_s), ref, rtol=0, atol=1e-12 * ref.abs().max().item())
    wt = torch.tensor(np.random.default_rng(55).standard_normal((w.n, 3)), device=DEV)
    ref_dx, ref_dm = sg.PM(16).accel_adjoint(pos, mass, wt, box=1.0, r_s=w.r_s)
    say("alloc failure: PM adjoint meshes")
    inject(0)
    with pytest.raises(sg.SrgravError) as ei:
        pm.accel_adjoint(pos, mass, wt, box=1.0, r_s=w.r_s)
    inject(-1)
    assert ei.value.code == SR_ENOMEM
    dx, dm = pm.accel_adjoint(pos, mass, wt, box=1.0, r_s=w.r_s)
    assert torch.allclose(dx, ref_dx, rtol=0, atol=1e-12 * ref_dx.abs().max().item())
    assert torch.allclose(dm, ref_dm, rtol=0, atol=1e-12 * ref_dm.abs().max().item())
