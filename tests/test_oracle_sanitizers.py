"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): a copy built with both runs FK, clearances, edge checks, an ESDF
grid, the Halton sampler and a planner replay in a child process; any
report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import oracle as orc
from paper_2503_06757_amd import workloads as W
r7, r14 = W.robot_r7(), W.robot_r14()
rob7, rob14 = orc.OracleRobot(r7), orc.OracleRobot(r14)
prims = W.scene_s64(r7)
q = np.random.default_rng(1).uniform(-2.8, 2.8, (64, 7)).astype(np.float32)
orc.fk_spheres_batch(rob7, q, n_threads=2)
a, b = W.random_edges(r7, 300, seed=3)
orc.check_edges(rob7, prims, a, b, 32.0, early_exit=True, n_threads=2, want_m=True)
orc.check_edges(rob14, W.scene_shelf(r14), *W.random_edges(r14, 50, seed=4), 32.0, n_threads=1)
g = orc.EsdfGrid((-1.3, -1.3, -1.3), 2.6 / 15, orc.esdf_of_scene(prims, (-1.3, -1.3, -1.3), 2.6 / 15, (16, 16, 16)))
with g:
    orc.check_edges(rob7, np.zeros(0, W.PRIM_DTYPE), a[:50], b[:50], 32.0, n_threads=1)
for i in (0, 1, 12345, 2 ** 32 - 1):
    orc.radical_inverse(i, 53)
s, gl = W.query_candidates(r7, W.SEED_QUERY, 1)[0]
for sampler in (0, 2):
    orc.plan(rob7, W.scene_s12(r7, 0), s, gl, seed=3, workers=16, max_rounds=20, n_threads=2, sampler=sampler,
             dds_radius=0.3, dds_tries=2)
print("child ok")
"""


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc's AddressSanitizer runtime is not installed")
def test_oracle_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    import oracle
    lib = oracle.build(out=str(tmp_path / "liboracle_san.so"),
                       extra=("-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"))
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=_runtime("libasan.so"),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               PYTHONPATH=ROOT, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "child ok" in r.stdout, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
