"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
every entry point the tests use, on small inputs (cold and supplied starts,
replay, the outer search over K, the FP32-rounding mode, standard EM with
K-means and Anderson mixing, the unpenalised finish, reconstruct in both
projections, the projection of given particles, features, the perceptron
forward and backward passes, decode and targets), in a subprocess that
preloads the ASan runtime; any report aborts it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import numpy as np
import oracle
from paper_2007_12273_amd import synth
oracle.build(force=True)
d = synth.random_cells(3, 5, 3, 40, 300, k_lo=1, k_hi=3)
v, a, off = d["v"], d["alpha"], d["cell_off"]
o = oracle.compress(v, a, off, kmax=8, seed=1, max_sweeps=40, trace=True)
oracle.compress(v, a, off, kmax=8, seed=1, fixed_sweeps=5, mode=oracle.MODE_ROUND32)
oracle.compress(v, a, off, kmax=8, seed=1, max_sweeps=40, mode=oracle.MODE_OUTER_K)
init = {k: o[k] for k in ("K", "omega", "mu", "sigma")}
oracle.compress(v, a, off, kmax=8, seed=1, max_sweeps=20, init=init)
oracle.compress_std(v, a, off, 4, seed=1, kmax=8, kmeans=True, aa_m=3, max_iter=30, trace=True)
c0 = slice(off[0], off[1])
oracle.mle_finish(v[c0], a[c0], o["omega"][0, :o["K"][0]], o["mu"][0, :o["K"][0]], o["sigma"][0, :o["K"][0]])
tg = oracle.targets_from_moments(o["moments"], 3)
oracle.reconstruct(o["K"], o["omega"], o["mu"], o["sigma"], off, tg, 3, 2, seed=4)
oracle.reconstruct_tensor(o["K"], o["omega"], o["mu"], o["sigma"], off, o["moments"], 3, 1, seed=4)
oracle.project(v, a, off, o["moments"], 3, tensor=True)
f, fr = oracle.features(v, a, off)
rng = np.random.default_rng(0)
P = {"W1": rng.normal(size=(105, 256)) * 0.05, "b1": np.zeros(256), "W2": rng.normal(size=(256, 256)) * 0.05,
     "b2": np.zeros(256), "W3": rng.normal(size=(256, 160)) * 0.05, "b3": np.zeros(160)}
_, _, Y = oracle.mlp_forward(f, P, bf16=True)
T = oracle.warm_targets(o, fr)
oracle.mlp_loss_backward(f, P, T, bf16=False)
oracle.warm_decode(Y.astype(np.float32), fr, off, 16)
print("sanitized oracle ok")
'''


@pytest.mark.slow
def test_oracle_clean_under_asan_and_ubsan():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no ASan runtime")
    env = dict(os.environ, GM_ORACLE_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.stdout[-3000:], r.stderr[-6000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
