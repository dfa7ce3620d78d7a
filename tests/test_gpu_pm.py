"""Parity of the PM long-range force (HIP path through the C ABI) with the PM
oracle.  Both are FP64; the mass assignment uses device atomics and the FFTs
are different implementations, so agreement is to rounding: the largest
difference must stay below 1e-10 of the largest acceleration."""
import numpy as np
import pytest
import torch

from oracle import pm as OPM
from paper_2606_17145_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_17145_amd as sg
    return sg


def check(sg, pos, mass, box, n_mesh, r_s, tag, scale=None):
    """Largest difference relative to `scale` (default: the largest oracle acceleration)."""
    print(f"pm parity: {tag} N={len(pos)} mesh={n_mesh}^3", flush=True)
    acc = sg.pm_accel(torch.tensor(pos, device=DEV), torch.tensor(mass, device=DEV), box=box, n_mesh=n_mesh,
                      r_s=r_s).cpu().numpy()
    ref = OPM.pm_accel(pos, mass, box, n_mesh, r_s)
    if scale is None:
        scale = np.abs(ref).max()
    err = np.abs(acc - ref).max() / scale
    print(f"   max |a - a_ref| / scale = {err:.3e}", flush=True)
    assert err <= 1e-10
    return acc, ref


MESH = {"uniform_32k": 64, "clustered_262k": 128, "clustered_2m_active": 256}


@pytest.mark.parametrize("case", ["uniform_32k", "clustered_262k", "clustered_2m_active"])
def test_pm_matches_oracle(sg, case):
    # each workload on its own mesh, up to 2,097,152 particles on 256^3
    w = getattr(WL, case)()
    n_mesh = MESH[case]
    r_s, _ = WL.split_scales(n_mesh, w.box)
    check(sg, w.pos, w.mass, w.box, n_mesh, r_s, case)


def test_pm_unwrapped_ragged_and_single(sg):
    rng = np.random.default_rng(31)
    pos = rng.uniform(-2.0, 3.0, (1001, 3))                  # positions outside the box wrap
    mass = rng.uniform(0.5, 1.5, 1001)
    check(sg, pos, mass, 1.0, 16, 1.25 / 16, "unwrapped")
    # one particle feels no force of its own: assignment and interpolation share their
    # weights and the gradient kernel is odd, so both sides are rounding noise next to
    # the pull G m / h^2 of that mass one cell away
    h = 1.0 / 8
    scale = mass[0] / h ** 2
    acc, ref = check(sg, pos[:1] + 0.013, mass[:1], 1.0, 8, 1.25 / 8, "single particle", scale)
    assert np.abs(acc).max() <= 1e-12 * scale and np.abs(ref).max() <= 1e-12 * scale
    acc, _ = check(sg, pos * 2.5, mass, 2.5, 32, 2.5 * 1.25 / 32, "box 2.5")
    # the shared mesh: a second call on the same handle gives the same accelerations
    h = sg.PM(32)
    a1 = h.accel(torch.tensor(pos * 2.5, device=DEV), torch.tensor(mass, device=DEV), box=2.5,
                 r_s=2.5 * 1.25 / 32).cpu().numpy()
    a2 = h.accel(torch.tensor(pos * 2.5, device=DEV), torch.tensor(mass, device=DEV), box=2.5,
                 r_s=2.5 * 1.25 / 32).cpu().numpy()
    assert np.abs(a1 - a2).max() <= 1e-13 * np.abs(acc).max()


def test_pm_error_paths(sg):
    with pytest.raises(sg.SrgravError):
        sg.PM(7)                                             # odd mesh
    h = sg.PM(8)
    x = torch.zeros((4, 3), dtype=torch.float64, device=DEV)
    m = torch.ones(4, dtype=torch.float64, device=DEV)
    with pytest.raises(sg.SrgravError):
        h.accel(x, m, box=0.0, r_s=0.1)
    with pytest.raises(sg.SrgravError):
        h.accel(x, m, box=1.0, r_s=0.0)


def check_adjoint(sg, pos, mass, w, box, n_mesh, r_s, tag, pm=None):
    print(f"pm adjoint parity: {tag} N={len(pos)} mesh={n_mesh}^3", flush=True)
    args = dict(box=box, n_mesh=n_mesh, r_s=r_s, pm=pm)
    dx, dm = sg.pm_accel_adjoint(torch.tensor(pos, device=DEV), torch.tensor(mass, device=DEV),
                                 torch.tensor(w, device=DEV), **args)
    rx, rm = OPM.pm_adjoint(pos, mass, box, n_mesh, r_s, w)
    ex = np.abs(dx.cpu().numpy() - rx).max() / np.abs(rx).max()
    em = np.abs(dm.cpu().numpy() - rm).max() / np.abs(rm).max()
    print(f"   dpos {ex:.3e}  dmass {em:.3e} (of the largest oracle value)", flush=True)
    assert ex <= 1e-10 and em <= 1e-10


@pytest.mark.parametrize("case", ["uniform_32k", "clustered_262k"])
def test_pm_adjoint_matches_oracle(sg, case):
    w = getattr(WL, case)()
    n_mesh = 64 if case == "uniform_32k" else 128
    r_s, _ = WL.split_scales(n_mesh, w.box)
    cot = np.random.default_rng(17).standard_normal((w.n, 3))
    check_adjoint(sg, w.pos, w.mass, cot, w.box, n_mesh, r_s, case)


def test_pm_adjoint_handle_reuse_and_autograd(sg):
    rng = np.random.default_rng(41)
    pos = rng.uniform(-1.0, 2.0, (3001, 3))
    mass = rng.uniform(0.5, 1.5, 3001)
    cot = rng.standard_normal((3001, 3))
    h = sg.PM(32)
    r_s = 1.25 / 32
    # two calls in a row on one handle, the second smaller: the lazily allocated
    # meshes are cleared and reused
    check_adjoint(sg, pos, mass, cot, 1.0, 32, r_s, "first call", pm=h)
    check_adjoint(sg, pos[:777], mass[:777], cot[:777], 1.0, 32, r_s, "second call, smaller", pm=h)
    # the autograd path gives the adjoint's gradients
    x = torch.tensor(pos, device=DEV, requires_grad=True)
    m = torch.tensor(mass, device=DEV, requires_grad=True)
    acc = sg.PMAccel.apply(x, m, h, 1.0, r_s)
    (acc * torch.tensor(cot, device=DEV)).sum().backward()
    rx, rm = OPM.pm_adjoint(pos, mass, 1.0, 32, r_s, cot)
    assert np.abs(x.grad.cpu().numpy() - rx).max() <= 1e-10 * np.abs(rx).max()
    assert np.abs(m.grad.cpu().numpy() - rm).max() <= 1e-10 * np.abs(rm).max()


def test_pm_adjoint_error_paths(sg):
    from paper_2606_17145_amd import _lib
    h = sg.PM(8)
    x = torch.zeros((4, 3), dtype=torch.float64, device=DEV)
    m = torch.ones(4, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        h.accel_adjoint(x, m, torch.zeros((4, 2), dtype=torch.float64, device=DEV), box=1.0, r_s=0.1)
    out = torch.empty((4, 3), dtype=torch.float64, device=DEV)
    rc = _lib.lib().pm_accel_adjoint(h._h, _lib.ptr(x), _lib.ptr(m), 4, 1.0, 0.1, 1.0, None, _lib.ptr(out),
                                     _lib.ptr(m), _lib.stream_handle())
    assert rc != 0
    with pytest.raises(sg.SrgravError):
        h.accel_adjoint(x, m, out, box=1.0, r_s=-1.0)
