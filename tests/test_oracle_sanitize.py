"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

oracle.c is compiled a second time with -fsanitize=address,undefined (gcc, host
code only) and driven through its ctypes wrapper in a child interpreter that
preloads the ASan runtime: tree build, walk (Barnes-Hut and relative criterion,
all targets and an active subset), exact direct sum, adjoint, per-particle
gradient, central differences and interaction lists, on small inputs that cover
the degenerate cases (one particle, two particles, duplicate positions, unequal
softening).  Any invalid access or undefined operation aborts the child.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import oracle as O
O.LIB_PATH = sys.argv[2]
rng = np.random.default_rng(7)

def run(pos, mass, eps, p, targets=None, a_old=None):
    t = O.Tree(pos, mass, eps)
    O.walk(t, p, targets=targets, a_old=a_old)
    n = pos.shape[0]
    nt = n if targets is None else len(targets)
    w = rng.standard_normal((nt, 3))
    O.adjoint(t, p, w, targets=targets, a_old=a_old)
    js = np.arange(min(n, 5))
    O.gradient_of(t, p, w, js, targets=targets, a_old=a_old)
    O.fd_gradient_of(t, p, w, js, targets=targets, a_old=a_old)
    O.interaction_lists(t, p, targets=targets, a_old=a_old)
    O.direct(pos, mass, eps, p, targets=targets)

p = dict(r_s=0.05, r_cut=0.225, theta=0.5)
run(rng.random((1, 3)), 1.0, 1e-3, p)
run(rng.random((2, 3)), 0.5, 1e-3, p)
x = rng.random((300, 3))
x[100:120] = x[100]                       # duplicate positions: one level-30 bucket
eps = np.where(np.arange(300) % 4 == 0, 2.5e-4, 1e-3)
run(x, 1.0 / 300, eps, p)
run(x, 1.0 / 300, eps, p, targets=np.arange(0, 300, 7))
a_old = np.abs(rng.standard_normal(300)) + 0.1
run(x, 1.0 / 300, 1e-3, dict(p, criterion="relative", alpha=0.005, theta=0.7),
    targets=np.arange(3, 300, 5), a_old=a_old)
print("sanitized oracle: ok")
"""


def test_oracle_under_asan_ubsan():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    with tempfile.TemporaryDirectory() as d:
        so = os.path.join(d, "liboracle_san.so")
        subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp", "-fPIC",
                        "-shared", "-o", so, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
        env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
        r = subprocess.run([sys.executable, "-c", DRIVER, ROOT, so], env=env, capture_output=True, text=True,
                           timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
