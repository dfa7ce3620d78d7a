"""Tree reuse between rebuilds on the device (tree_drift) against the oracle's
drifted tree (paper App. A: between rebuilds the tree nodes drift with their
particles; the topology stays, the moments and node cubes follow the particles).

* topology and particle order kept; masses, refolded centres of mass, FP32 node
  records and the grown cube sides bit-exact against the oracle's drift;
* FP64 walk on the drifted tree: interaction counts bit-exact, accelerations
  within 1e-12 relative (all targets; also a 10% active subset under the
  relative criterion); FP32 within the forward's error bar; FP64 adjoint
  against the oracle's adjoint of the drifted tree;
* zero displacement gives the built tree back bit for bit; a second drift is
  measured from the built positions (not cumulative); a rebuild afterwards is
  a plain build; a non-finite displacement is refused; a drift voids the list
  token of an earlier forward call.
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


def workload(case):
    w = WL.clustered(20_000, seed=31, n_spheres=10)
    if case == "mixed":
        w.eps = w.eps.copy()
        w.eps[::4] /= 4
    if case == "duplicates":
        w.pos = w.pos.copy()
        w.pos[200:260] = w.pos[200]
    return w


def displacement(w, seed, scale=1.0):
    """Most particles move a few tenths of the mean spacing, 2% move ten times
    that, and particles near the box faces are pushed across them."""
    rng = np.random.default_rng(seed)
    spacing = 1.0 / round(w.n ** (1 / 3))
    d = 0.3 * spacing * scale * rng.standard_normal((w.n, 3))
    far = rng.random(w.n) < 0.02
    d[far] *= 10.0
    u = np.mod(w.pos, 1.0)
    d[u < 2e-3] -= 4e-3 * scale
    d[u > 1.0 - 2e-3] += 4e-3 * scale
    return d


def gpu_tree(sg, w):
    return sg.tree_build(torch.tensor(w.pos, device=DEV), torch.tensor(w.mass, device=DEV),
                         eps=torch.tensor(w.eps, device=DEV), box=w.box)


def rel_err(a, ref):
    nr = np.linalg.norm(ref, axis=1)
    return np.linalg.norm(a - ref, axis=1) / np.maximum(nr, 1e-6 * np.median(nr))


def check_tree(t, d):
    ex = {k: v.cpu().numpy() for k, v in t.export().items()}
    nd = d.nodes()
    assert np.array_equal(ex["perm"], d.perm)
    for k in ("level", "first", "count", "parent", "skip"):
        assert np.array_equal(ex[k], nd[k]), k
    assert np.array_equal(ex["M"], nd["M"])
    assert np.array_equal(ex["com"], nd["com"])
    assert np.array_equal(ex["M32"], nd["M32"])
    assert np.array_equal(ex["comX"].view(np.uint32), nd["comX"])
    side = 2.0 * nd["half"] if "half" in nd else np.ldexp(1.0, -nd["level"].astype(np.int64))
    assert np.array_equal(ex["side"], side)
    return ex


@pytest.mark.parametrize("case", ["clustered", "mixed", "duplicates"])
def test_drift_matches_oracle(sg, oracle, case):
    w = workload(case)
    disp = displacement(w, seed=32)
    say(f"drift: {case} N={w.n}")
    t = gpu_tree(sg, w)
    ref = oracle.Tree(w.pos, w.mass, w.eps)
    d = ref.drift(disp)
    grown = int((2.0 * d.nodes()["half"] != np.ldexp(1.0, -d.nodes()["level"].astype(np.int64))).sum())
    assert grown > 100
    t.drift(torch.tensor(disp, device=DEV))
    check_tree(t, d)
    p = w.params("fp64")
    acc, cnt = sg.shortrange_accel(t, p)
    acc_ref, cnt_ref = oracle.walk(d, p)
    assert np.array_equal(cnt.cpu().numpy(), cnt_ref)
    e = rel_err(acc.cpu().numpy(), acc_ref)
    say(f"   {grown} grown nodes; fp64 max rel err {e.max():.3e}")
    assert e.max() <= 1e-12
    acc32, _ = sg.shortrange_accel(t, w.params("fp32"))
    e32 = rel_err(acc32.double().cpu().numpy(), acc_ref)
    say(f"   fp32 median {np.median(e32):.3e} p99.9 {np.quantile(e32, 0.999):.3e}")
    assert np.median(e32) <= 1e-5 and np.quantile(e32, 0.999) <= 1e-4
    wt = np.random.default_rng(33).standard_normal((w.n, 3))
    dx, dm = sg.shortrange_accel_adjoint(t, p, torch.tensor(wt, device=DEV))
    gx, gm = oracle.adjoint(d, p, wt)
    sx, sm = np.abs(gx).max(), np.abs(gm).max()
    say(f"   adjoint dx err {np.abs(dx.cpu().numpy() - gx).max() / sx:.3e}  dm err {np.abs(dm.cpu().numpy() - gm).max() / sm:.3e}")
    assert np.allclose(dx.cpu().numpy(), gx, rtol=1e-10, atol=1e-11 * sx)
    assert np.allclose(dm.cpu().numpy(), gm, rtol=1e-10, atol=1e-11 * sm)


def test_drift_deep_chains(sg, oracle):
    """A 28-deep tree whose 512-particle runs all end inside nested chains: the
    refold passes over partition-crossing nodes hold hundreds of nodes per block."""
    w = WL.deep_chains()
    rng = np.random.default_rng(34)
    disp = 1e-4 * rng.standard_normal((w.n, 3))
    say(f"drift: deep chains N={w.n}")
    t = gpu_tree(sg, w)
    d = oracle.Tree(w.pos, w.mass, w.eps).drift(disp)
    t.drift(torch.tensor(disp, device=DEV))
    check_tree(t, d)
    p = w.params("fp64")
    acc, cnt = sg.shortrange_accel(t, p)
    acc_ref, cnt_ref = oracle.walk(d, p)
    assert np.array_equal(cnt.cpu().numpy(), cnt_ref)
    e = rel_err(acc.cpu().numpy(), acc_ref)
    say(f"   fp64 max rel err {e.max():.3e}")
    assert e.max() <= 1e-12


def test_drift_active_subset_relative(sg, oracle):
    w = workload("clustered")
    disp = displacement(w, seed=34)
    say(f"drift: active subset, relative criterion, N={w.n}")
    t = gpu_tree(sg, w)
    ref = oracle.Tree(w.pos, w.mass, w.eps)
    d = ref.drift(disp)
    t.drift(torch.tensor(disp, device=DEV))
    a0, _ = oracle.walk(d, w.params("fp64"))
    a_old = np.linalg.norm(a0, axis=1)
    active = np.sort(np.random.default_rng(35).choice(w.n, w.n // 10, replace=False))
    p = dict(w.params("fp64"), criterion="relative", alpha=0.005, theta=0.7)
    acc, cnt = sg.shortrange_accel(t, p, active=torch.tensor(active.astype(np.int32), device=DEV),
                                   a_old=torch.tensor(a_old, device=DEV))
    acc_ref, cnt_ref = oracle.walk(d, p, targets=active, a_old=a_old)
    assert np.array_equal(cnt.cpu().numpy(), cnt_ref)
    assert rel_err(acc.cpu().numpy(), acc_ref).max() <= 1e-12


def test_zero_second_and_rebuild(sg, oracle):
    from paper_2606_17145_amd import _lib
    w = workload("clustered")
    say(f"drift: zero, second, rebuild, N={w.n}")
    t = gpu_tree(sg, w)
    p = w.params("fp64")
    ex0 = {k: v.cpu().numpy() for k, v in t.export().items()}
    acc0, cnt0 = sg.shortrange_accel(t, p)
    tok = t.list_token
    # zero displacement: the built tree, bit for bit
    t.drift(torch.zeros((w.n, 3), dtype=torch.float64, device=DEV))
    ex1 = {k: v.cpu().numpy() for k, v in t.export().items()}
    for k in ex0:
        assert np.array_equal(ex0[k], ex1[k]), k
    # the drift voided the forward's token
    with pytest.raises(_lib.SrgravError) as ei:
        sg.shortrange_accel_adjoint(t, p, torch.zeros((w.n, 3), dtype=torch.float64, device=DEV),
                                    list_token=tok)
    assert ei.value.code == -4
    acc1, cnt1 = sg.shortrange_accel(t, p)
    assert torch.equal(cnt0, cnt1) and torch.equal(acc0, acc1)
    # two drifts: the second is measured from the built positions
    ref = oracle.Tree(w.pos, w.mass, w.eps)
    t.drift(torch.tensor(displacement(w, seed=36), device=DEV))
    disp2 = displacement(w, seed=37, scale=0.5)
    t.drift(torch.tensor(disp2, device=DEV))
    d2 = ref.drift(disp2)
    check_tree(t, d2)
    acc2, cnt2 = sg.shortrange_accel(t, p)
    acc_ref, cnt_ref = oracle.walk(d2, p)
    assert np.array_equal(cnt2.cpu().numpy(), cnt_ref)
    assert rel_err(acc2.cpu().numpy(), acc_ref).max() <= 1e-12
    # a non-finite displacement is refused
    bad = torch.zeros((w.n, 3), dtype=torch.float64, device=DEV)
    bad[5, 2] = float("inf")
    with pytest.raises(_lib.SrgravError) as ei:
        t.drift(bad)
    assert ei.value.code == -1
    # a rebuild at the moved positions is a plain build again
    moved = np.mod(w.pos + disp2, 1.0)
    w2 = WL.Workload("moved", moved, w.mass, w.eps, r_s=w.r_s, r_cut=w.r_cut)
    t.build(torch.tensor(moved, device=DEV), torch.tensor(w.mass, device=DEV), eps=torch.tensor(w.eps, device=DEV))
    ref2 = oracle.Tree(moved, w.mass, w.eps)
    check_tree(t, ref2)
    acc3, cnt3 = sg.shortrange_accel(t, w2.params("fp64"))
    acc_ref, cnt_ref = oracle.walk(ref2, w2.params("fp64"))
    assert np.array_equal(cnt3.cpu().numpy(), cnt_ref)
    # then drifting again starts from the new build
    t.drift(torch.zeros((w.n, 3), dtype=torch.float64, device=DEV))
    check_tree(t, ref2)


def test_drift_single_particle(sg):
    w = WL.uniform(1, seed=3, n_mesh=16)
    t = gpu_tree(sg, w)
    t.drift(torch.full((1, 3), 0.25, dtype=torch.float64, device=DEV))
    acc, cnt = sg.shortrange_accel(t, w.params("fp64"))
    assert torch.count_nonzero(acc) == 0 and torch.count_nonzero(cnt) == 0
